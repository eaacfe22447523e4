"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what it pins:
  exact rational brute force of Eq. 1 (fractions), LAPACK least squares,
  Householder invariants (Q^T Q = I, R triangular, R^T R = J^T J + lam D^2),
  the normal-equation optimality condition, closed forms for orthogonal
  columns, special cases (no dense part, one block, lam = 0, lam -> inf),
  the golden fixture under tests/golden/, and planted mistakes.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import dense, exact, refine, structured
from workloads import generators as gen

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = np.finfo(np.float64).eps


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _small_inst(seed, K=4, m=5, n=3, nB=4, lam=1e-2, ragged=False):
    if ragged:
        rng = np.random.default_rng(seed + 1000)
        m = rng.integers(1, 7, size=K)
    return gen.make_blockangular(seed, K=K, m=m, n=n, nB=nB, lam=lam)


# ---------------------------------------------------------------- O1 invariants

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_o1_householder_invariants(seed):
    """I1-I3: Q^T Q = I, strict lower part of R exactly zero, R^T R = A^T A, A = QR."""
    inst = _small_inst(seed, K=5, m=4, nB=6)
    J = dense.assemble_blockangular(inst)
    Aaug = np.vstack([J, np.sqrt(inst.lam) * np.diag(inst.d)])
    m, N = Aaug.shape
    R, _, refl = dense.householder_qr(Aaug)
    Q = dense.apply_q(refl, np.eye(m))           # full m x m orthogonal factor
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 10 * m * np.sqrt(N) * EPS
    assert np.all(np.tril(R, -1) == 0.0)
    AtA = Aaug.T @ Aaug
    assert np.linalg.norm(R.T @ R - AtA) / np.linalg.norm(AtA) <= 10 * m * EPS
    QR = Q[:, :N] @ R
    assert np.linalg.norm(Aaug - QR) <= 10 * m * EPS * np.linalg.norm(Aaug)


def test_householder_vector_conventions():
    """sigma == 0 -> tau = 0 and the diagonal keeps its sign; sign(0) = +1."""
    v, tau, beta = dense.householder_vector(np.array([-3.0, 0.0, 0.0]))
    assert tau == 0.0 and beta == -3.0
    v, tau, beta = dense.householder_vector(np.array([0.0, 3.0, 4.0]))
    assert beta == -5.0 and tau == 1.0
    H = np.eye(3) - tau * np.outer(v, v)
    assert np.allclose(H @ np.array([0.0, 3.0, 4.0]), [-5.0, 0.0, 0.0], atol=1e-15)
    v, tau, beta = dense.householder_vector(np.array([-1.0, 2.0, 2.0]))
    assert beta == 3.0


# ------------------------------------------------------------ exact rational pin

def _exact_p(inst):
    J = dense.assemble_blockangular(inst)
    d2 = [Fraction(float(x)) ** 2 for x in inst.d]
    return exact.solve_normal_equations(J, inst.b.astype(np.float64), d2, inst.lam)


@pytest.mark.parametrize("seed", [3, 4])
def test_o1_o2_oext_vs_exact_rational(seed):
    """P3: O1 and O2 within 1e-13 of the exact rational solution; O-ext within 1e-17."""
    inst = _small_inst(seed, K=3, m=4, n=2, nB=3)
    p_ex = np.array([float(x) for x in _exact_p(inst)])
    p1 = dense.solve_blockangular_dense(inst)["p"]
    p2, f = structured.solve_blockangular(inst)
    assert _rel(p1, p_ex) <= 1e-13
    assert _rel(p2, p_ex) <= 1e-13
    p3 = refine.refine(inst, f, p2, sweeps=3)
    # compare in longdouble against the exact fractions
    p_ex_ld = np.array([np.longdouble(x.numerator) / np.longdouble(x.denominator) for x in _exact_p(inst)])
    err = float(np.linalg.norm((p3 - p_ex_ld).astype(np.float64)) / np.linalg.norm(p_ex))
    assert err <= 1e-17


def test_golden_integer_instance():
    """Golden fixture (tests/golden/tiny_integer.json): exact rational p of a tiny
    integer block-angular instance, written by tests/golden/make_golden.py."""
    with open(os.path.join(HERE, "golden", "tiny_integer.json")) as fh:
        g = json.load(fh)
    row_off = np.array(g["row_off"], np.int64)
    A = np.array(g["A"], np.float64)
    B = np.array(g["B"], np.float64)
    b = np.array(g["b"], np.float64)
    d = np.sqrt(np.array(g["d2"], np.float64))
    lam = float(Fraction(g["lam"]))
    inst = gen.BlockAngular(row_off, g["n"], A, B, b, d, lam, np.dtype(np.float64))
    p_gold = np.array([float(Fraction(s)) for s in g["p"]])
    # the fixture itself against a fresh brute-force solve
    J = dense.assemble_blockangular(inst)
    p_ex = exact.solve_normal_equations(J, b, [Fraction(x) for x in g["d2"]], Fraction(g["lam"]))
    assert [str(x) for x in p_ex] == g["p"]
    assert _rel(dense.solve_blockangular_dense(inst)["p"], p_gold) <= 1e-13
    assert _rel(structured.solve_blockangular(inst)[0], p_gold) <= 1e-13


# -------------------------------------------------------------- LAPACK pins

@pytest.mark.parametrize("seed,ragged", [(5, False), (6, True), (7, True)])
def test_o1_o2_vs_lstsq(seed, ragged):
    """P4 + P7: O1 and O2 agree with numpy.linalg.lstsq (LAPACK) on the augmented system."""
    inst = _small_inst(seed, K=6, m=5, n=3, nB=5, ragged=ragged)
    J = dense.assemble_blockangular(inst)
    Aaug = np.vstack([J, np.sqrt(inst.lam) * np.diag(inst.d)])
    y = np.concatenate([inst.b, np.zeros(inst.N)])
    p_ls = np.linalg.lstsq(Aaug, y, rcond=None)[0]
    cond = np.linalg.cond(Aaug)
    p1 = dense.solve_blockangular_dense(inst)["p"]
    p2 = structured.solve_blockangular(inst)[0]
    assert _rel(p1, p_ls) <= 100 * cond * EPS
    assert _rel(p2, p_ls) <= 100 * cond * EPS
    assert _rel(p1, p2) <= 1e-12


def test_o2_factor_matches_o1_factor():
    """The structured R = [[blkdiag(R_i), S], [0, R_B]] equals O1's dense R up to row signs."""
    inst = _small_inst(8, K=4, m=6, n=2, nB=3)
    o1 = dense.solve_blockangular_dense(inst)
    f = structured.factor_blockangular(inst)
    K, n, nB = inst.K, inst.n, inst.nB
    R = np.zeros((inst.N, inst.N))
    c = np.zeros(inst.N)
    for i in range(K):
        R[i * n:(i + 1) * n, i * n:(i + 1) * n] = f.R_blk[i]
        R[i * n:(i + 1) * n, K * n:] = f.S[i]
        c[i * n:(i + 1) * n] = f.c_blk[i]
    R[K * n:, K * n:] = f.R_B
    c[K * n:] = f.c_B
    Rs, cs = dense.sign_normalise(R, c)
    R1, c1 = dense.sign_normalise(o1["R"], o1["c"])
    assert np.allclose(Rs, R1, atol=1e-12)
    assert np.allclose(cs, c1, atol=1e-12)
    assert abs(f.resid - o1["resid"]) <= 1e-12 * max(1.0, o1["resid"])


# ------------------------------------------------------------- special cases

def test_lambda_zero_is_ordinary_least_squares():
    """P6: lam = 0 reduces to lstsq(J, b)."""
    inst = _small_inst(9, K=5, m=6, n=3, nB=4, lam=0.0)
    J = dense.assemble_blockangular(inst)
    p_ls = np.linalg.lstsq(J, inst.b, rcond=None)[0]
    assert _rel(structured.solve_blockangular(inst)[0], p_ls) <= 1e-12
    assert _rel(dense.solve_blockangular_dense(inst)["p"], p_ls) <= 1e-12


def test_no_dense_part_is_independent_blocks():
    """P6: nB = 0 splits into K independent small least-squares problems."""
    inst = _small_inst(10, K=7, m=5, n=3, nB=0, ragged=True)
    p2 = structured.solve_blockangular(inst)[0]
    for i in range(inst.K):
        r0, r1 = inst.row_off[i], inst.row_off[i + 1]
        Ai = np.vstack([inst.A[r0:r1], np.sqrt(inst.lam) * np.diag(inst.d[i * 3:(i + 1) * 3])])
        yi = np.concatenate([inst.b[r0:r1], np.zeros(3)])
        pi = np.linalg.lstsq(Ai, yi, rcond=None)[0]
        assert _rel(p2[i * 3:(i + 1) * 3], pi) <= 1e-12


def test_one_block_is_dense_problem():
    """P6: K = 1 is a dense problem [A_1 | B]."""
    inst = _small_inst(11, K=1, m=20, n=3, nB=6)
    J = np.hstack([inst.A, inst.B])
    Aaug = np.vstack([J, np.sqrt(inst.lam) * np.diag(inst.d)])
    y = np.concatenate([inst.b, np.zeros(inst.N)])
    p_ls = np.linalg.lstsq(Aaug, y, rcond=None)[0]
    assert _rel(structured.solve_blockangular(inst)[0], p_ls) <= 1e-12


def test_large_lambda_limit():
    """P6: lam -> inf gives p ~ J^T b / (lam d^2) to first order."""
    inst = _small_inst(12, K=4, m=5, n=3, nB=4, lam=1e8)
    J = dense.assemble_blockangular(inst)
    p_lim = (J.T @ inst.b) / (inst.lam * inst.d ** 2)
    p2 = structured.solve_blockangular(inst)[0]
    assert _rel(p2, p_lim) <= 1e-6


def test_block_fewer_rows_than_columns_with_damping():
    """m_i < n is allowed when lam > 0 (the damping rows restore full rank)."""
    inst = gen.make_blockangular(13, K=5, m=np.array([1, 2, 3, 1, 2]), n=3, nB=2, lam=0.5)
    J = dense.assemble_blockangular(inst)
    Aaug = np.vstack([J, np.sqrt(inst.lam) * np.diag(inst.d)])
    y = np.concatenate([inst.b, np.zeros(inst.N)])
    p_ls = np.linalg.lstsq(Aaug, y, rcond=None)[0]
    assert _rel(structured.solve_blockangular(inst)[0], p_ls) <= 1e-12
    with pytest.raises(np.linalg.LinAlgError):
        structured.solve_blockangular(inst.with_lambda(0.0))


# -------------------------------------------------------------- closed form

def orthogonal_column_instance(seed, K=50, m=6, n=3, nB=5, lam=1e-2):
    """Block-angular J whose N columns are mutually orthogonal: A_i = Q_i diag(s_i),
    B = orth(P_perp G) diag(s_B) with P_perp projecting each block's rows off span(A_i)."""
    rng = np.random.default_rng(seed)
    M = K * m
    row_off = np.arange(0, M + 1, m, dtype=np.int64)
    A = np.zeros((M, n))
    G = rng.standard_normal((M, nB))
    PG = np.zeros_like(G)
    for i in range(K):
        Qi, _ = np.linalg.qr(rng.standard_normal((m, n)))
        A[i * m:(i + 1) * m] = Qi * rng.uniform(0.5, 3.0, size=n)[None, :]
        Gi = G[i * m:(i + 1) * m]
        PG[i * m:(i + 1) * m] = Gi - Qi @ (Qi.T @ Gi)
    QB, _ = np.linalg.qr(PG)
    B = QB * rng.uniform(0.5, 3.0, size=nB)[None, :]
    b = rng.standard_normal(M)
    d = gen.column_norms_blockangular(row_off, n, A, B)
    return gen.BlockAngular(row_off, n, A, B, b, d, lam, np.dtype(np.float64))


def test_closed_form_orthogonal_columns():
    """P5: J^T J diagonal => p_j = a_j^T b / ((1 + lam) ||a_j||^2) with d = column norms."""
    inst = orthogonal_column_instance(14)
    J = dense.assemble_blockangular(inst)
    col2 = (J * J).sum(axis=0)
    assert np.allclose(J.T @ J, np.diag(col2), atol=1e-12)
    p_cf = (J.T @ inst.b) / ((1.0 + inst.lam) * col2)
    assert _rel(structured.solve_blockangular(inst)[0], p_cf) <= 1e-13
    assert _rel(dense.solve_blockangular_dense(inst)["p"], p_cf) <= 1e-13
    p_ext, _ = refine.reference_solution(inst)
    assert _rel(p_ext, p_cf) <= 1e-15


# ------------------------------------------------------------- optimality

def test_optimality_condition_at_scale():
    """P2: J^T (b - J p) = lam D^2 p within the rounding bound, on a mid-size instance."""
    inst = gen.make_blockangular(15, K=2000, m=12, n=3, nB=30, lam=1e-2, dtype=np.float32, scale_k=3.0)
    p, f = structured.solve_blockangular(inst)
    g = refine.normal_residual(inst, p, np.float64)
    JF = np.sqrt(float((inst.A.astype(np.float64) ** 2).sum() + (inst.B.astype(np.float64) ** 2).sum()))
    bound = 10 * (inst.M + inst.N) * EPS * (JF ** 2 * np.linalg.norm(p) + JF * np.linalg.norm(inst.b))
    assert np.linalg.norm(g.astype(np.float64)) <= bound
    # the refined reference drives the normal residual far below that bound
    p_ref = refine.refine(inst, f, p, sweeps=2)
    g2 = refine.normal_residual(inst, p_ref, np.longdouble)
    assert float(np.linalg.norm(g2.astype(np.float64))) <= 1e-3 * bound


# ----------------------------------------------------------- planted mistakes

def test_planted_mistakes_are_caught(monkeypatch):
    """Planting plausible mistakes in the oracle makes a pin fail (mutation check)."""
    inst = _small_inst(16, K=3, m=4, n=2, nB=3)
    p_ex = np.array([float(x) for x in _exact_p(inst)])

    def o2_err():
        return _rel(structured.solve_blockangular(inst)[0], p_ex)

    assert o2_err() <= 1e-13
    real_qr = np.linalg.qr

    # (a) Q applied instead of Q^T to the coupled columns
    real_matmul = np.matmul

    def bad_matmul(a, b, *args, **kw):
        if a.ndim == 3 and a.shape[1] == a.shape[2] and b.ndim == 3 and b.shape[1] == a.shape[1]:
            a = np.swapaxes(a, 1, 2)
        return real_matmul(a, b, *args, **kw)

    monkeypatch.setattr(structured.np, "matmul", bad_matmul)
    assert o2_err() > 1e-6
    monkeypatch.setattr(structured.np, "matmul", real_matmul)

    # (b) lam used where sqrt(lam) belongs in the damping rows
    monkeypatch.setattr(np, "sqrt", lambda x: x)
    err_b = o2_err()
    monkeypatch.undo()
    assert err_b > 1e-6

    # (c) refinement with D instead of D^2 in the normal residual
    def bad_normal_residual(inst_, p, dt=np.longdouble):
        p = np.asarray(p).astype(dt)
        r = inst_.b.astype(dt) - refine.apply_J(inst_, p, dt)
        return refine.apply_JT(inst_, r, dt) - dt(inst_.lam) * np.asarray(inst_.d).astype(dt) * p

    monkeypatch.setattr(refine, "normal_residual", bad_normal_residual)
    p3 = refine.refine(inst, structured.factor_blockangular(inst), structured.solve_blockangular(inst)[0])
    assert _rel(p3.astype(np.float64), p_ex) > 1e-8
    monkeypatch.undo()

    # (d) a transposed block in O1's assembly
    def bad_assemble(inst_):
        J = np.zeros((inst_.M, inst_.N))
        for i in range(inst_.K):
            r0, r1 = int(inst_.row_off[i]), int(inst_.row_off[i + 1])
            blkA = inst_.A[r0:r1]
            J[r0:r1, i * inst_.n:(i + 1) * inst_.n] = blkA[::-1]
        J[:, inst_.K * inst_.n:] = inst_.B
        return J

    monkeypatch.setattr(dense, "assemble_blockangular", bad_assemble)
    assert _rel(dense.solve_blockangular_dense(inst)["p"], p_ex) > 1e-6
    monkeypatch.undo()
    assert real_qr is np.linalg.qr
