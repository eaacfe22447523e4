"""Writes tests/golden/tiny_integer.json: a tiny block-angular instance with integer
entries, integer squared damping diagonal and lam = 1/100, together with the exact
rational LM step p of Eq. 1 computed by oracle.exact (brute-force Gaussian elimination
in fractions.Fraction).  Calls only oracle/.  Run: python tests/golden/make_golden.py
"""
import json
import os
import sys
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import dense, exact  # noqa: E402
from workloads import generators as gen  # noqa: E402


def main():
    rng = np.random.Generator(np.random.PCG64(20180212))
    m = [3, 2, 4]
    n, nB = 2, 2
    row_off = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
    M = int(row_off[-1])
    A = rng.integers(-9, 10, size=(M, n)).astype(np.float64)
    B = rng.integers(-9, 10, size=(M, nB)).astype(np.float64)
    b = rng.integers(-9, 10, size=M).astype(np.float64)
    N = len(m) * n + nB
    d2 = rng.integers(1, 5, size=N)
    lam = Fraction(1, 100)
    inst = gen.BlockAngular(row_off, n, A, B, b, np.sqrt(d2.astype(np.float64)), float(lam),
                            np.dtype(np.float64))
    J = dense.assemble_blockangular(inst)
    p = exact.solve_normal_equations(J, b, [Fraction(int(x)) for x in d2], lam)
    out = dict(
        description="tiny integer block-angular LM step; p is exact (fractions) for "
                    "(J^T J + lam diag(d2)) p = J^T b, the paper's Eq. 1",
        row_off=row_off.tolist(), n=n, A=A.astype(int).tolist(), B=B.astype(int).tolist(),
        b=b.astype(int).tolist(), d2=[int(x) for x in d2], lam=str(lam),
        p=[str(x) for x in p],
    )
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_integer.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
