"""Write tests/golden/tiny_case.txt: a small fixed problem and the FP64
oracle's density at every voxel.  Calls only the oracle (Alg. PB-SYM,
Sec. 3.2, under the Epanechnikov reading of the kernels of Sec. 2.1).

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

GRID = dict(gx=7, gy=6, gt=9, hs=2.75, ht=2.5, sres=1.0, tres=1.0, x0=0.0, y0=0.0, t0=0.0)
POINTS = [
    (3.5, 3.0, 4.5),     # voxel-centred in x and t, on a voxel face in y
    (0.25, 5.75, 1.0),   # near a grid corner: footprint clipped
    (-1.5, 2.0, 8.75),   # outside the grid in x, still reaching columns X = 0, 1
    (6.0, 0.5, 10.0),    # outside in t, reaching the last rows
    (4.125, 2.625, 3.375),
]


def main():
    pts = np.array(POINTS, dtype=np.float64)
    f, evals = oracle.pbsym(pts, oracle.Grid(**GRID), nthreads=1)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_case.txt")
    with open(path, "w") as fh:
        fh.write("# Regression fixture for the FP64 oracle (Alg. PB-SYM, Sec. 3.2;\n")
        fh.write("# estimator and Epanechnikov-read kernels of Sec. 2.1).  Written by\n")
        fh.write("# tests/golden/make_golden.py, which calls only oracle/.\n")
        fh.write("grid " + " ".join(f"{k}={v!r}" for k, v in GRID.items()) + "\n")
        for p in POINTS:
            fh.write("point %r %r %r\n" % p)
        fh.write(f"evals {evals}\n")
        for X in range(GRID["gx"]):
            for Y in range(GRID["gy"]):
                for T in range(GRID["gt"]):
                    if f[X, Y, T] != 0.0:
                        fh.write(f"v {X} {Y} {T} {float(f[X, Y, T])!r}\n")
    print(path)


if __name__ == "__main__":
    main()
