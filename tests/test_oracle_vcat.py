"""Pins of the oracle's vertical concatenation (Section 4.5, Eq. vcatDecomp): merging the factors of
[J1; sqrt(lam) D] and of J2 must give the factor of the problem that has the rows of both, which
the structured factor computes directly (up to the sign of each row of R), whose solution LAPACK's
least squares on the dense stacked matrix gives, and merging is associative.  A planted mistake (the
second factor's blocks not interleaved with the first's, i.e. no row permutation P) fails."""
import dataclasses

import numpy as np
import pytest

from oracle import dense, structured
from oracle.dense import sign_normalise
from workloads import generators as gen


def _parts(seed, K=30, n=3, nB=7, lam=1e-2, parts=2):
    """Instances over the same columns (d shared), the first damped, the others not."""
    base = gen.make_blockangular(seed, K=K, m=(np.arange(K) % 5) + 4, n=n, nB=nB, lam=lam, dtype=np.float64)
    out = [base]
    for k in range(1, parts):
        o = gen.make_blockangular(seed + 17 * k, K=K, m=(np.arange(K) * (k + 1)) % 4 + 2, n=n, nB=nB, lam=0.0,
                                  dtype=np.float64)
        out.append(dataclasses.replace(o, d=base.d.copy()))
    return out


def _same_factor(fa, fb, tol=1e-11):
    K = fa.R_blk.shape[0]
    for i in range(K):
        Ra, Ca = sign_normalise(fa.R_blk[i], np.concatenate([fa.S[i], fa.c_blk[i][:, None]], axis=1))
        Rb, Cb = sign_normalise(fb.R_blk[i], np.concatenate([fb.S[i], fb.c_blk[i][:, None]], axis=1))
        scale = max(np.abs(Rb).max(), np.abs(Cb).max())
        assert np.abs(Ra - Rb).max() <= tol * scale
        assert np.abs(Ca - Cb).max() <= tol * scale
    if fa.R_B.size:
        Ra, ca = sign_normalise(fa.R_B, fa.c_B)
        Rb, cb = sign_normalise(fb.R_B, fb.c_B)
        scale = max(np.abs(Rb).max(), np.abs(cb).max())
        assert np.abs(Ra - Rb).max() <= tol * scale
        assert np.abs(ca - cb).max() <= tol * scale
    assert abs(fa.resid - fb.resid) <= tol * max(1.0, fb.resid)


@pytest.mark.parametrize("nB", [0, 1, 7, 20])
def test_vcat_equals_factor_of_stacked_rows(nB):
    i1, i2 = _parts(11 + nB, nB=nB)
    merged = structured.factor_vcat(structured.factor_blockangular(i1), structured.factor_blockangular(i2))
    direct = structured.factor_blockangular(gen.stack_rows([i1, i2]))
    _same_factor(merged, direct)


def test_vcat_solution_is_least_squares_of_stacked_matrix():
    i1, i2 = _parts(31)
    merged = structured.factor_vcat(structured.factor_blockangular(i1), structured.factor_blockangular(i2))
    p = structured.solve_factor(merged)
    J = np.vstack([dense.assemble_blockangular(i1), dense.assemble_blockangular(i2),
                   np.sqrt(i1.lam) * np.diag(i1.d)])
    rhs = np.concatenate([i1.b, i2.b, np.zeros(i1.N)])
    p_ls, *_ = np.linalg.lstsq(J, rhs, rcond=None)
    assert np.abs(p - p_ls).max() <= 1e-10 * np.abs(p_ls).max()
    # the residual norm of the merged factor is that of the stacked least-squares problem
    assert abs(merged.resid - np.linalg.norm(J @ p_ls - rhs)) <= 1e-10 * max(1.0, merged.resid)


def test_vcat_is_associative():
    i1, i2, i3 = _parts(41, parts=3)
    f1, f2, f3 = (structured.factor_blockangular(i) for i in (i1, i2, i3))
    left = structured.factor_vcat(structured.factor_vcat(f1, f2), f3)
    direct = structured.factor_blockangular(gen.stack_rows([i1, i2, i3]))
    _same_factor(left, direct)


def test_planted_mistake_without_the_interleave_fails():
    """Pairing block i of the first factor with block i+1 of the second (no block-wise row
    permutation) is a valid QR of some matrix, but not of [A1; A2]."""
    i1, i2 = _parts(51)
    f1, f2 = structured.factor_blockangular(i1), structured.factor_blockangular(i2)
    shifted = dataclasses.replace(f2, R_blk=np.roll(f2.R_blk, 1, axis=0), S=np.roll(f2.S, 1, axis=0),
                                  c_blk=np.roll(f2.c_blk, 1, axis=0))
    wrong = structured.factor_vcat(f1, shifted)
    direct = structured.factor_blockangular(gen.stack_rows([i1, i2]))
    with pytest.raises(AssertionError):
        _same_factor(wrong, direct)


def test_stack_rows_keeps_every_row():
    i1, i2 = _parts(61)
    st = gen.stack_rows([i1, i2])
    assert st.M == i1.M + i2.M and st.K == i1.K
    for k in range(st.K):
        a, e = int(st.row_off[k]), int(st.row_off[k + 1])
        want = np.vstack([i1.A[i1.row_off[k]:i1.row_off[k + 1]], i2.A[i2.row_off[k]:i2.row_off[k + 1]]])
        assert np.array_equal(st.A[a:e], want)
