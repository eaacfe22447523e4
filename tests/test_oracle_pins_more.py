"""Pins of the oracle functions that the other pin files do not reach.

  dense.forward_substitute_transposed / back_substitute - LAPACK triangular solves (scipy)
  dense.apply_qt / apply_q                              - orthogonality, Q^T A = [R; 0], and the
                                                          LAPACK least-squares residual
  adjoint.adjoint_dense on a banded J                   - float64 central differences of the
                                                          oracle's solve and torch autograd
                                                          through LAPACK lstsq
  lm.bd_jacobian_instance / ba_jacobian_instance, c > 0 - central differences of the residual
                                                          functions, column norms from the
                                                          dense Jacobian
Each test also plants one plausible mistake and checks that the pin catches it.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import adjoint, banded, dense, lm
from workloads import generators as gen

EPS = np.finfo(np.float64).eps


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _upper(seed, n):
    rng = np.random.default_rng(seed)
    R = np.triu(rng.standard_normal((n, n)))
    R[np.arange(n), np.arange(n)] = np.sign(rng.standard_normal(n)) * (1.0 + rng.random(n))
    return R


# ------------------------------------------------------------------ triangular solves

@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_forward_substitute_transposed_vs_lapack(n):
    """R^T y = g against LAPACK's trtrs with trans='T'; a transposed operand is caught."""
    R = _upper(10 + n, n)
    g = np.random.default_rng(n).standard_normal(n)
    y = dense.forward_substitute_transposed(R, g)
    y_lp = scipy.linalg.solve_triangular(R, g, trans="T", lower=False)
    assert _rel(y, y_lp) <= 1e-13
    assert _rel(R.T @ y, g) <= 1e-13
    if n > 1:
        # planted: solving with R instead of R^T must not pass the same check
        wrong = scipy.linalg.solve_triangular(R.T.copy(), g, trans="T", lower=True)
        assert _rel(wrong, y_lp) > 1e-6


@pytest.mark.parametrize("n", [1, 5, 33])
def test_back_substitute_vs_lapack(n):
    R = _upper(20 + n, n)
    c = np.random.default_rng(n + 1).standard_normal(n)
    p = dense.back_substitute(R, c)
    assert _rel(p, scipy.linalg.solve_triangular(R, c, lower=False)) <= 1e-13


def test_back_substitute_singular_raises():
    R = _upper(3, 6)
    R[4, 4] = 1e-300
    with pytest.raises(dense.SingularError):
        dense.back_substitute(R, np.ones(6))


# --------------------------------------------------------------- stored reflectors (Q)

@pytest.mark.parametrize("shape", [(9, 4), (30, 12), (5, 5)])
def test_apply_qt_pins(shape):
    """Q^T from the kept reflectors: Q^T A = [R; 0] for the factored A; Q^T Q = I through
    apply_q; the norm of the tail of Q^T y is the LAPACK least-squares residual, and R p = c
    (first N entries of Q^T y) gives LAPACK's least-squares solution."""
    m, N = shape
    rng = np.random.default_rng(m * 100 + N)
    A = rng.standard_normal((m, N))
    y = rng.standard_normal(m)
    R, qty, refl = dense.householder_qr(A, y)
    QtA = dense.apply_qt(refl, A)
    assert np.abs(QtA[:N] - R).max() <= 50 * m * EPS * np.abs(A).max()
    assert np.abs(QtA[N:]).max(initial=0.0) <= 50 * m * EPS * np.abs(A).max()
    qt = dense.apply_qt(refl, y)
    assert np.abs(qt - qty).max() <= 50 * m * EPS * np.abs(y).max()
    assert abs(np.linalg.norm(qt) - np.linalg.norm(y)) <= 50 * m * EPS * np.linalg.norm(y)
    Y = rng.standard_normal((m, 3))
    assert np.abs(dense.apply_qt(refl, dense.apply_q(refl, Y)) - Y).max() <= 50 * m * EPS * np.abs(Y).max()
    p_ls, res, _, _ = np.linalg.lstsq(A, y, rcond=None)
    p = dense.back_substitute(R, qt[:N])
    assert _rel(p, p_ls) <= 1e-11
    if m > N:
        assert abs(np.linalg.norm(qt[N:]) ** 2 - float(res[0])) <= 1e-10 * max(float(res[0]), 1.0)
    # planted: applying the reflectors in the reverse order (that is Q, not Q^T) is caught
    assert np.abs(dense.apply_q(refl, A)[N:]).max(initial=1.0) > 1e-6 or m == N


# ------------------------------------------------------------ adjoint on a dense / banded J

def _banded_small(seed, N=8, w=3, lam=0.05):
    return gen.make_banded(seed, N=N, w=w, lam=lam, dtype=np.float64)


def _loss_banded(inst, p_star):
    p = banded.solve_dense_o1(inst)["p"]
    return 0.5 * float(np.sum((p - p_star) ** 2))


def _copy_banded(inst):
    return gen.Banded(inst.N, inst.w, inst.row_start.copy(), inst.vals.copy(), inst.b.copy(),
                      inst.d.copy(), inst.lam, inst.dtype)


def _adjoint_banded(inst, g):
    o1 = banded.solve_dense_o1(inst)
    J = banded.assemble(inst)
    return adjoint.adjoint_dense(J, inst.b, inst.d, inst.lam, o1["p"], g, o1["R"]), o1["p"]


def test_adjoint_dense_banded_vs_central_differences():
    """adjoint_dense on a banded J: dL/dvals (on the band), dL/db, dL/dd and dL/dlam against
    float64 central differences (h = 1e-6) of L = 0.5||p - p*||^2 through the oracle solve."""
    inst = _banded_small(61)
    rng = np.random.default_rng(62)
    p_star = rng.standard_normal(inst.N)
    gr, p = _adjoint_banded(inst, banded.solve_dense_o1(inst)["p"] - p_star)
    h = 1e-6

    def fd(mutate):
        a, b_ = _copy_banded(inst), _copy_banded(inst)
        mutate(a, +h)
        mutate(b_, -h)
        return (_loss_banded(a, p_star) - _loss_banded(b_, p_star)) / (2 * h)

    for (r, k) in [(0, 0), (5, 2), (11, 1), (15, 0)]:
        col = int(inst.row_start[r]) + k

        def mut(x, e, r=r, k=k):
            x.vals[r, k] += e
        ref = fd(mut)
        assert abs(ref - gr["dJ"][r, col]) <= 1e-6 * max(1.0, abs(ref)), (r, k)
    for r in [0, 7, 15]:
        def mut(x, e, r=r):
            x.b[r] += e
        assert abs(fd(mut) - gr["db"][r]) <= 1e-6 * max(1.0, abs(gr["db"][r]))
    for j in [0, 3, 7]:
        def mut(x, e, j=j):
            x.d[j] += e
        assert abs(fd(mut) - gr["dd"][j]) <= 1e-6 * max(1.0, abs(gr["dd"][j]))

    def mut_lam(x, e):
        x.lam += e
    ref = fd(mut_lam)
    assert abs(ref - gr["dlam"]) <= 1e-6 * max(1.0, abs(ref))


def test_adjoint_dense_banded_vs_torch_autograd():
    """adjoint_dense against torch autograd (float64) through torch.linalg.lstsq of the
    assembled augmented banded system, for a random g = dL/dp."""
    torch = pytest.importorskip("torch")
    inst = _banded_small(63, N=10, w=4, lam=0.02)
    g = np.random.default_rng(64).standard_normal(inst.N)
    gr, _ = _adjoint_banded(inst, g)
    J = banded.assemble(inst)
    Jt = torch.tensor(J, dtype=torch.float64, requires_grad=True)
    bt = torch.tensor(inst.b, dtype=torch.float64, requires_grad=True)
    dt = torch.tensor(inst.d, dtype=torch.float64, requires_grad=True)
    lt = torch.tensor(inst.lam, dtype=torch.float64, requires_grad=True)
    Aaug = torch.cat([Jt, torch.sqrt(lt) * torch.diag(dt)], 0)
    y = torch.cat([bt, torch.zeros(inst.N, dtype=torch.float64)])
    pt = torch.linalg.lstsq(Aaug, y[:, None]).solution[:, 0]
    (pt * torch.tensor(g)).sum().backward()
    mask = J != 0.0
    assert np.allclose(gr["dJ"][mask], Jt.grad.numpy()[mask], atol=1e-10, rtol=1e-9)
    assert np.allclose(gr["db"], bt.grad.numpy(), atol=1e-10, rtol=1e-9)
    assert np.allclose(gr["dd"], dt.grad.numpy(), atol=1e-10, rtol=1e-9)
    assert abs(gr["dlam"] - float(lt.grad)) <= 1e-9 * max(1.0, abs(gr["dlam"]))
    # planted: u from R^{-1} g alone (one triangular solve dropped) is caught
    o1 = banded.solve_dense_o1(inst)
    u_wrong = dense.back_substitute(o1["R"], g)
    assert _rel(J @ u_wrong, bt.grad.numpy()) > 1e-3


# ------------------------------------------------------------- LM Jacobians at c != 0

def _fd_jacobian(fun, x, h=1e-6):
    cols = []
    for j in range(x.size):
        e = np.zeros_like(x)
        e[j] = h
        cols.append((fun(x + e) - fun(x - e)) / (2 * h))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("c", [0.1, 0.5])
def test_banded_lm_jacobian_vs_central_differences(c):
    """bd_jacobian_instance at c > 0: J(x) = J0 diag(phi'(x)) against central differences of
    bd_residual, b = -f(x), and d = column norms of the dense J(x) (1 for an empty column)."""
    inst0, y, x0, _ = gen.lm_banded(71, N=12, w=3, c=c, dtype=np.float64)
    model = lm.BandedModel(inst0, y.astype(np.float64), c)
    step, f = lm.bd_jacobian_instance(model, x0, 0.3)
    Jfd = _fd_jacobian(lambda x: lm.bd_residual(model, x), x0)
    J = banded.assemble(step)
    assert np.abs(J - Jfd).max() <= 1e-7 * max(1.0, np.abs(J).max())
    assert np.array_equal(step.b, -f)
    assert np.abs(f - (lm.bd_residual(model, x0))).max() == 0.0
    d_ref = np.sqrt((J * J).sum(axis=0))
    d_ref[d_ref == 0.0] = 1.0
    assert _rel(step.d, d_ref) <= 1e-14
    assert step.lam == 0.3
    # the residual itself against its definition written densely
    J0 = banded.assemble(inst0)
    assert _rel(lm.bd_residual(model, x0), J0 @ (x0 + c * x0 ** 3) - model.y) <= 1e-14
    # planted: phi' without the factor 3 is caught by the difference check
    wrong = J0 * (1.0 + c * x0 ** 2)[None, :]
    assert np.abs(wrong - Jfd).max() > 1e-4


@pytest.mark.parametrize("c", [0.1])
def test_blockangular_lm_jacobian_vs_central_differences(c):
    """ba_jacobian_instance at c > 0 against central differences of ba_residual."""
    inst0, y, x0, _ = gen.lm_blockangular(72, K=4, m=5, n=3, nB=4, c=c, dtype=np.float64)
    model = lm.BlockAngularModel(inst0, y.astype(np.float64), c)
    step, f = lm.ba_jacobian_instance(model, x0, 0.2)
    Jfd = _fd_jacobian(lambda x: lm.ba_residual(model, x), x0)
    J = dense.assemble_blockangular(step)
    assert np.abs(J - Jfd).max() <= 1e-7 * max(1.0, np.abs(J).max())
    assert np.array_equal(step.b, -f)
    d_ref = np.sqrt((J * J).sum(axis=0))
    d_ref[d_ref == 0.0] = 1.0
    assert _rel(step.d, d_ref) <= 1e-14
    J0 = dense.assemble_blockangular(inst0)
    assert _rel(lm.ba_residual(model, x0), J0 @ (x0 + c * x0 ** 3) - model.y) <= 1e-14
