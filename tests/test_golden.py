"""The stored oracle fixtures under tests/golden/ still equal what the oracle computes."""
import os

import numpy as np

import oracle
from paper_2412_13043_amd import workloads as wl

HERE = os.path.join(os.path.dirname(__file__), "golden")


def test_three_point_fixture_matches_oracle():
    ref = np.loadtxt(os.path.join(HERE, "three_point_full.txt"))
    assert ref.shape == (1024,) and np.all(ref > 0)
    P, A, m2, Z = wl.three_point()
    idx = np.array([0, 1, 15, 16, 255, 512, 777, 1008, 1023])
    got = oracle.integrate(oracle.THREE_POINT, wl.THREE_NQ, wl.THREE_QMAX, n_x=wl.THREE_NX,
                           n_phi=wl.THREE_NPHI, ext=(P[idx], A[idx]), m2=m2[idx], Z=Z)
    assert np.array_equal(got, ref[idx])
