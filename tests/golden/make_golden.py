"""Write the FP64 oracle's values for the full-size workloads as text fixtures.

Calls only oracle/ (and the seeded input generators).  Fixtures:
  three_point_full.txt  -- I_e for all 1024 external pairs of the three-point workload
                           (64 |p| x 16 angles, GL 64 x 32 x 16 on [0, 10k], m2 ~ U[0.1, 2] seed 3,
                           Z seed 1), one value per line, %.17e.
Run from the repository root: python tests/golden/make_golden.py
"""
import os
import sys
import threading

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2412_13043_amd import workloads as wl  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def three_point_full(threads=8):
    P, A, m2, Z = wl.three_point()
    out = np.empty(P.size)
    chunks = np.array_split(np.arange(P.size), threads)

    def work(idx):
        out[idx] = oracle.integrate(oracle.THREE_POINT, wl.THREE_NQ, wl.THREE_QMAX,
                                    n_x=wl.THREE_NX, n_phi=wl.THREE_NPHI,
                                    ext=(P[idx], A[idx]), m2=m2[idx], Z=Z)

    ths = [threading.Thread(target=work, args=(c,)) for c in chunks]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    return out


if __name__ == "__main__":
    v = three_point_full()
    np.savetxt(os.path.join(HERE, "three_point_full.txt"), v, fmt="%.17e",
               header="FP64 oracle, three-point workload (all 1024 external pairs); "
                      "written by tests/golden/make_golden.py")
    print("wrote", v.size, "values")
