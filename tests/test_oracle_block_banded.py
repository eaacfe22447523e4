"""Pins of the block-banded compressed-WY oracle (paper Section 4.4) against facts that do not
come from it: the R of the dense Householder oracle (unique up to row signs), LAPACK least
squares, R^T R = J^T J + lam D^2, the band structure of R, and planted mistakes."""
import dataclasses

import numpy as np
import pytest

from oracle import banded, block_banded, dense
from workloads import generators as gen


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _sign_fix(R, c):
    sg = np.where(np.diag(R) < 0, -1.0, 1.0)
    return R * sg[:, None], c * sg


CASES = [  # (N, w, rows_per_col, lam, r)
    (40, 3, 2, 1e-2, 16),
    (37, 12, 2, 1e-2, 16),
    (64, 15, 1, 0.1, 16),
    (50, 7, 3, 1e-3, 8),
    (16, 16, 2, 1e-2, 16),
    (9, 5, 2, 1.0, 16),
    (33, 1, 2, 0.3, 16),
    (45, 9, 2, 0.0, 16),
]


@pytest.mark.parametrize("case", CASES)
def test_block_banded_matches_dense_householder_and_lapack(case):
    N, w, rpc, lam, r = case
    inst = gen.make_banded(4000 + N + w, N=N, w=w, rows_per_col=rpc, lam=lam, dtype=np.float64)
    f = block_banded.factor(inst, r)
    o1 = banded.solve_dense_o1(inst)
    Rb, cb = _sign_fix(f["R"], f["c"])
    Ro, co = _sign_fix(o1["R"], o1["c"])
    scale = np.abs(Ro).max()
    assert np.abs(Rb - Ro).max() <= 1e-12 * scale
    assert np.abs(cb - co).max() <= 1e-12 * max(np.abs(co).max(), scale)
    assert abs(f["resid"] - o1["resid"]) <= 1e-10 * max(o1["resid"], 1.0)
    # R^T R = J^T J + lam D^2 (closed form)
    J = banded.assemble(inst)
    Mtx = J.T @ J + lam * np.diag(inst.d ** 2)
    assert np.abs(f["R"].T @ f["R"] - Mtx).max() <= 1e-12 * np.abs(Mtx).max()
    # upper bandwidth w - 1: the entries a step computes beyond it are roundoff
    far = np.triu(f["R"], w)
    assert np.abs(far).max(initial=0.0) <= 1e-13 * scale
    # the step's solution against LAPACK least squares on the augmented system
    p, _ = block_banded.solve(inst, r)
    Aaug = np.vstack([J, np.sqrt(lam) * np.diag(inst.d)])
    p_ls = np.linalg.lstsq(Aaug, np.concatenate([inst.b, np.zeros(N)]), rcond=None)[0]
    assert _rel(p, p_ls) <= 1e-11


def test_block_banded_irregular_row_starts():
    """Starts that jump over whole blocks, runs of equal starts and fewer rows than columns."""
    N, w = 70, 6
    rs = np.array(sorted([0, 0, 1, 2, 17, 17, 17, 18, 40, 41, 41, 60, 64, 64]), np.int32)
    rng = np.random.default_rng(4100)
    vals = rng.standard_normal((rs.size, w))
    b = rng.standard_normal(rs.size)
    d = gen.column_norms_banded(N, w, rs, vals)
    inst = gen.Banded(N, w, rs, vals, b, d, 0.05, np.dtype(np.float64))
    f = block_banded.factor(inst, 16)
    o1 = banded.solve_dense_o1(inst)
    Rb, cb = _sign_fix(f["R"], f["c"])
    Ro, co = _sign_fix(o1["R"], o1["c"])
    assert np.abs(Rb - Ro).max() <= 1e-12 * np.abs(Ro).max()
    assert np.abs(cb - co).max() <= 1e-12 * np.abs(Ro).max()


def test_compressed_wy_is_the_product_of_reflectors():
    """I + Y T Y^T equals H_0 H_1 ... H_{k-1} formed from the same reflectors one by one, and
    Q^T A from the WY form is upper triangular in the factored columns."""
    rng = np.random.default_rng(4200)
    A = rng.standard_normal((20, 9))
    Y, T = block_banded.compressed_wy(A, 6)
    _, _, refl = dense.householder_qr(A[:, :6])
    Q = dense.apply_q(refl, np.eye(20))
    assert np.abs(np.eye(20) + Y @ T @ Y.T - Q).max() <= 1e-14 * 20
    QtA = block_banded.apply_wy_transposed(Y, T, A)
    assert np.abs(np.tril(QtA[:, :6], -1)).max() <= 1e-14 * np.abs(A).max() * 20


def test_planted_mistakes_are_caught(monkeypatch):
    """T with LAPACK's sign, or the next block's damping rows left out, break the pins."""
    inst = gen.make_banded(4300, N=48, w=8, lam=0.05, dtype=np.float64)
    o1 = banded.solve_dense_o1(inst)
    Ro, _ = _sign_fix(o1["R"], o1["c"])
    orig = block_banded.compressed_wy

    def wrong_sign(A, ncols):
        Y, T = orig(A, ncols)
        return Y, -T
    monkeypatch.setattr(block_banded, "compressed_wy", wrong_sign)
    Rw, _ = _sign_fix(block_banded.factor(inst)["R"], np.zeros(inst.N))
    assert np.abs(Rw - Ro).max() > 1e-3 * np.abs(Ro).max()
    monkeypatch.setattr(block_banded, "compressed_wy", orig)
    no_damp = dataclasses.replace(inst, d=np.where(np.arange(inst.N) >= 16, 0.0, inst.d))
    Rn, _ = _sign_fix(block_banded.factor(no_damp)["R"], np.zeros(inst.N))
    assert np.abs(Rn - Ro).max() > 1e-3 * np.abs(Ro).max()
