"""Pins of the banded, adjoint and bf16 parts of the oracle."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import adjoint, banded, bf16, dense, exact, refine, structured
from workloads import generators as gen


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------------- banded

def test_banded_w1_closed_form():
    """w = 1: every column is touched by its own rows only, so J^T J is diagonal and
    p_j = sum(v b) / (sum v^2 + lam d_j^2)."""
    inst = gen.make_banded(1, N=30, w=1, lam=0.3, dtype=np.float64)
    J = banded.assemble(inst)
    col2 = (J * J).sum(axis=0)
    p_cf = (J.T @ inst.b) / (col2 + inst.lam * inst.d ** 2)
    assert _rel(banded.solve_dense_o1(inst)["p"], p_cf) <= 1e-14
    assert _rel(banded.reference_solution(inst)[0], p_cf) <= 1e-15


@pytest.mark.parametrize("w", [2, 5, 12])
def test_banded_vs_lstsq_and_bandwidth(w):
    """Banded O1 agrees with LAPACK lstsq; its R has upper bandwidth w-1."""
    inst = gen.make_banded(2 + w, N=40, w=w, lam=1e-2, dtype=np.float64)
    J = banded.assemble(inst)
    Aaug = np.vstack([J, np.sqrt(inst.lam) * np.diag(inst.d)])
    y = np.concatenate([inst.b, np.zeros(inst.N)])
    p_ls = np.linalg.lstsq(Aaug, y, rcond=None)[0]
    o1 = banded.solve_dense_o1(inst)
    assert _rel(o1["p"], p_ls) <= 1e-12
    R = o1["R"]
    assert np.all(np.triu(R, w) == 0.0) or np.max(np.abs(np.triu(R, w))) <= 1e-13 * np.max(np.abs(R))
    p_ref, R2, _ = banded.reference_solution(inst)
    assert _rel(p_ref, p_ls) <= 1e-12
    Rs = dense.sign_normalise(R)
    R2s = dense.sign_normalise(R2)
    assert np.allclose(Rs, R2s, atol=1e-12)


def test_banded_exact_rational():
    inst = gen.make_banded(7, N=8, w=3, lam=1e-2, dtype=np.float64)
    J = banded.assemble(inst)
    p_ex = exact.solve_normal_equations(J, inst.b, [Fraction(float(x)) ** 2 for x in inst.d], inst.lam)
    p_ex = np.array([float(x) for x in p_ex])
    assert _rel(banded.solve_dense_o1(inst)["p"], p_ex) <= 1e-13
    assert _rel(banded.reference_solution(inst)[0], p_ex) <= 1e-15


# ------------------------------------------------------------------ adjoint

def _loss_p(inst, p_star):
    p, _ = structured.solve_blockangular(inst)
    return 0.5 * float(np.sum((p - p_star) ** 2))


def test_adjoint_vs_central_differences():
    """Closed form vs float64 central differences (h = 1e-6) for L = 0.5||p - p*||^2."""
    inst = gen.make_blockangular(31, K=3, m=4, n=2, nB=3, lam=0.05)
    rng = np.random.default_rng(5)
    p_star = rng.standard_normal(inst.N)
    p, f = structured.solve_blockangular(inst)
    gr = adjoint.adjoint_blockangular(inst, f, p, p - p_star)
    h = 1e-6

    def fd(mutate):
        a = gen.BlockAngular(inst.row_off, inst.n, inst.A.copy(), inst.B.copy(), inst.b.copy(),
                             inst.d.copy(), inst.lam, inst.dtype)
        b_ = gen.BlockAngular(inst.row_off, inst.n, inst.A.copy(), inst.B.copy(), inst.b.copy(),
                              inst.d.copy(), inst.lam, inst.dtype)
        mutate(a, +h)
        mutate(b_, -h)
        return (_loss_p(a, p_star) - _loss_p(b_, p_star)) / (2 * h)

    for (r, c) in [(0, 0), (5, 1), (11, 0)]:
        def mut(x, e, r=r, c=c):
            x.A[r, c] += e
        assert abs(fd(mut) - gr["dA"][r, c]) <= 1e-6 * max(1.0, abs(gr["dA"][r, c]))
    for (r, c) in [(0, 2), (7, 0), (9, 1)]:
        def mut(x, e, r=r, c=c):
            x.B[r, c] += e
        assert abs(fd(mut) - gr["dB"][r, c]) <= 1e-6 * max(1.0, abs(gr["dB"][r, c]))
    for r in [0, 6, 11]:
        def mut(x, e, r=r):
            x.b[r] += e
        assert abs(fd(mut) - gr["db"][r]) <= 1e-6 * max(1.0, abs(gr["db"][r]))
    for j in [0, 4, 7]:
        def mut(x, e, j=j):
            x.d[j] += e
        assert abs(fd(mut) - gr["dd"][j]) <= 1e-6 * max(1.0, abs(gr["dd"][j]))

    def mut_lam(x, e):
        x.lam += e
    assert abs(fd(mut_lam) - gr["dlam"]) <= 1e-6 * max(1.0, abs(gr["dlam"]))


def test_adjoint_vs_torch_autograd():
    """Closed form vs torch autograd (float64) through torch.linalg.lstsq of the augmented system."""
    torch = pytest.importorskip("torch")
    inst = gen.make_blockangular(32, K=4, m=5, n=3, nB=4, lam=0.02)
    J = dense.assemble_blockangular(inst)
    rng = np.random.default_rng(6)
    gvec = rng.standard_normal(inst.N)
    p, f = structured.solve_blockangular(inst)
    gr = adjoint.adjoint_blockangular(inst, f, p, gvec)
    Jt = torch.tensor(J, dtype=torch.float64, requires_grad=True)
    bt = torch.tensor(inst.b, dtype=torch.float64, requires_grad=True)
    dt = torch.tensor(inst.d, dtype=torch.float64, requires_grad=True)
    lt = torch.tensor(inst.lam, dtype=torch.float64, requires_grad=True)
    Aaug = torch.cat([Jt, torch.sqrt(lt) * torch.diag(dt)], 0)
    y = torch.cat([bt, torch.zeros(inst.N, dtype=torch.float64)])
    pt = torch.linalg.lstsq(Aaug, y[:, None]).solution[:, 0]
    (pt * torch.tensor(gvec)).sum().backward()
    dJ_t = Jt.grad.numpy()
    K, n = inst.K, inst.n
    for i in range(K):
        r0, r1 = inst.row_off[i], inst.row_off[i + 1]
        assert np.allclose(gr["dA"][r0:r1], dJ_t[r0:r1, i * n:(i + 1) * n], atol=1e-10)
    assert np.allclose(gr["dB"], dJ_t[:, K * n:], atol=1e-10)
    assert np.allclose(gr["db"], bt.grad.numpy(), atol=1e-10)
    assert np.allclose(gr["dd"], dt.grad.numpy(), atol=1e-10)
    assert abs(gr["dlam"] - float(lt.grad)) <= 1e-10 * max(1, abs(gr["dlam"]))


def test_adjoint_closed_form_orthogonal_columns():
    """Orthogonal columns: u_j = g_j / (||a_j||^2 + lam d_j^2)."""
    from tests.test_oracle_pins import orthogonal_column_instance
    inst = orthogonal_column_instance(33, K=20)
    p, f = structured.solve_blockangular(inst)
    g = np.random.default_rng(7).standard_normal(inst.N)
    gr = adjoint.adjoint_blockangular(inst, f, p, g)
    J = dense.assemble_blockangular(inst)
    col2 = (J * J).sum(axis=0)
    assert _rel(gr["u"], g / (col2 + inst.lam * inst.d ** 2)) <= 1e-13


# --------------------------------------------------------------------- bf16

def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(8)
    x = (rng.standard_normal(100_000) * 10.0 ** rng.uniform(-20, 20, 100_000)).astype(np.float32)
    # exact ties: values whose low 16 bits are 0x8000
    top = rng.integers(0, 2**7, 1000).astype(np.uint32) << np.uint32(16)
    ties = np.uint32(0x3F800000) | top | np.uint32(0x8000)
    x = np.concatenate([x, ties.view(np.float32)])
    ours = bf16.bf16_round(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))


def test_bf16_split_accuracy_and_exact_products():
    rng = np.random.default_rng(9)
    a = rng.standard_normal(10_000).astype(np.float32)
    hi, lo = bf16.split(a)
    res = a.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64)
    assert np.all(np.abs(res) <= 2.0 ** -16 * np.abs(a.astype(np.float64)))
    # bf16 x bf16 products are exact in fp32
    b = rng.standard_normal(10_000).astype(np.float32)
    bh, _ = bf16.split(b)
    assert np.array_equal((hi * bh).astype(np.float64), hi.astype(np.float64) * bh.astype(np.float64))
    A = rng.standard_normal((16, 64)).astype(np.float32)
    B = rng.standard_normal((64, 16)).astype(np.float32)
    C = bf16.bf16x3_matmul(A, B)
    C64 = A.astype(np.float64) @ B.astype(np.float64)
    assert np.max(np.abs(C - C64)) <= 64 * 2.0 ** -15 * np.max(np.abs(A)) * np.max(np.abs(B))


# -------------------------------------------------------------- two-stage damping (Section 5.2)

def _structured_R(f, K, n, nB):
    """Assemble [[blkdiag(R_i), S], [0, R_B]] densely."""
    N = K * n + nB
    R = np.zeros((N, N))
    for i in range(K):
        R[i * n:(i + 1) * n, i * n:(i + 1) * n] = f.R_blk[i]
        R[i * n:(i + 1) * n, K * n:] = f.S[i]
    R[K * n:, K * n:] = f.R_B
    return R


@pytest.mark.parametrize("lam", [1e-4, 1e-2, 1.0])
def test_two_stage_matches_direct(lam):
    """Eq. LMTwoStep: the QR of [R; sqrt(lam) D] (R from J alone) gives the solution of the
    directly damped problem, R'^T R' = J^T J + lam D^2 (closed form), and the same residual norm."""
    inst = gen.make_blockangular(41, K=12, m=7, n=3, nB=5, lam=lam)
    f2 = structured.factor_two_stage(inst, lam)
    f1 = structured.factor_blockangular(inst)
    p2 = structured.solve_factor(f2)
    p1 = structured.solve_factor(f1)
    assert np.linalg.norm(p2 - p1) <= 1e-11 * np.linalg.norm(p1)
    J = dense.assemble_blockangular(inst)
    R2 = _structured_R(f2, inst.K, inst.n, inst.nB)
    M = J.T @ J + lam * np.diag(inst.d ** 2)
    assert np.abs(R2.T @ R2 - M).max() <= 1e-12 * np.abs(M).max()
    assert abs(f2.resid - f1.resid) <= 1e-10 * max(f1.resid, 1.0)
    # and against LAPACK least squares on the augmented system
    Aaug = np.vstack([J, np.sqrt(lam) * np.diag(inst.d)])
    p_ls = np.linalg.lstsq(Aaug, np.concatenate([inst.b, np.zeros(inst.N)]), rcond=None)[0]
    assert np.linalg.norm(p2 - p_ls) <= 1e-10 * np.linalg.norm(p_ls)


def test_two_stage_small_lambda_reproduces_R():
    """As lam -> 0 the second stage returns R itself (up to row signs): [R; 0] = I [R; 0]."""
    inst = gen.make_blockangular(42, K=5, m=6, n=2, nB=3, lam=0.0)
    f0 = structured.factor_blockangular(inst)
    f2 = structured.factor_two_stage(inst, 1e-30)
    R0 = _structured_R(f0, inst.K, inst.n, inst.nB)
    R2 = _structured_R(f2, inst.K, inst.n, inst.nB)
    s0 = np.sign(np.diag(R0))
    s2 = np.sign(np.diag(R2))
    assert np.abs(s2[:, None] * R2 - s0[:, None] * R0).max() <= 1e-12 * np.abs(R0).max()


def test_rotated_precision_generator():
    """The rotated stress instances: B's column scales 10^(k t) are rotated by an orthogonal H,
    so B^T B has the scaled spectrum (its singular values are those of B_0 diag(s)) while B's
    column norms stay within a modest range (unlike the column-scaled variant)."""
    import numpy as np

    from workloads import generators as gen
    for k in (3, 5):
        inst = gen.precision_rotated(400 + k, k, lam=0.0, dtype=np.float64)
        base = gen.make_blockangular(400 + k, K=100, m=8, n=3, nB=24, lam=0.0, dtype=np.float64)
        assert np.array_equal(inst.A, base.A) and np.array_equal(inst.b, base.b)
        sv_rot = np.linalg.svd(inst.B, compute_uv=False)
        cn = np.linalg.norm(inst.B, axis=0)
        assert sv_rot.max() / sv_rot.min() > 10.0 ** (k - 1)        # the spread survives the rotation
        assert cn.max() / cn.min() < 10.0                            # but not along the columns
        assert np.allclose(inst.d[inst.K * 3:], cn, rtol=1e-14)      # d = column norms of the stored B
