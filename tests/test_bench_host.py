"""Host-side pieces of bench.py: the one-GPU guard, the far-field fraction and the source hash."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2412_13043_amd import workloads as wl  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_far_field_fraction_matches_a_direct_count():
    p = wl.momenta_log(16)
    n_q, q_max, n_x = 8, 10.0, 4
    xq, _ = np.polynomial.legendre.leggauss(n_q)
    q = 0.5 * q_max * (xq + 1.0)
    x, _ = np.polynomial.legendre.leggauss(n_x)
    far = 0
    for pj in p:
        for qa in q:
            for xb in x:
                far += (qa * qa + pj * pj + 2.0 * qa * pj * xb) >= bench.FAR_Y
    frac = bench.two_point_far_fraction(p, n_q, q_max, n_x)
    assert abs(frac - far / (p.size * n_q * n_x)) < 1e-12
    assert 0.0 < frac < 1.0


def test_source_hash_ignores_comments_only():
    h = bench.kernel_source_sha()
    assert isinstance(h, str) and len(h) == 16
    assert h == bench.kernel_source_sha()
