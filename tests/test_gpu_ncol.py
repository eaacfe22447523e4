"""Blocks of their own widths (qrk_create_blockangular_ncol, Section 4.1's m_i x n_i blocks)
through the C ABI, against the oracle: the damped least-squares solution of the assembled J
(LAPACK on the dense matrix, pinned in test_oracle_ncol.py).  Block widths 1..8 mixed, blocks
with fewer rows than columns among them, dense parts of 0, 40 and 100 columns; float32 with fp32
and BF16x3 dense-part updates and float64.  Unrefined bound as for uniform blocks (float32 1e-5
at cond <= 1e3, scaled by cond / 1e3 above it; float64 1e-12), 1e-10 after two sweeps."""
import numpy as np
import pytest

from oracle import dense
from tests.gpu_util import log, p_err
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _instance(seed, K=300, nB=40, lam=1e-2, dtype=np.float32, ncol=None):
    if ncol is None:
        ncol = (np.arange(K) * 5 + seed) % 8 + 1
    return gen.make_blockangular_ncol(seed, K=K, m=(np.arange(K) % 9) + 2, ncol=ncol, nB=nB, lam=lam, dtype=dtype)


def _reference(inst):
    J = dense.assemble_blockangular_ncol(inst)
    Aaug = np.vstack([J, np.sqrt(inst.lam) * np.diag(inst.d)])
    rhs = np.concatenate([inst.b.astype(np.float64), np.zeros(inst.N)])
    p, *_ = np.linalg.lstsq(Aaug, rhs, rcond=None)
    return p, np.linalg.cond(Aaug)


def _device(inst):
    import torch
    A = torch.from_numpy(np.ascontiguousarray(inst.A)).cuda()
    B = torch.from_numpy(np.ascontiguousarray(inst.B)).cuda() if inst.nB else None
    b = torch.from_numpy(np.ascontiguousarray(inst.b)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(inst.d)).cuda()
    return A, B, b, d


@pytest.mark.parametrize("dtype,mode", [(np.float32, "plain"), (np.float32, "bf16x3"), (np.float64, "plain")])
@pytest.mark.parametrize("nB", [0, 40, 100])
def test_ncol_matches_oracle(dtype, mode, nB):
    import torch
    from paper_1802_03773_amd import BlockAngularNcolSolver
    inst = _instance(7 + nB, nB=nB, dtype=dtype)
    p_ref, cond = _reference(inst)
    s = BlockAngularNcolSolver(inst.row_off, inst.ncol, nB, dtype=np.dtype(dtype).name, mode=mode)
    A, B, b, d = _device(inst)
    s.factor(A, B, b, d, inst.lam)
    p0 = s.solve(sweeps=0).cpu().numpy()
    p2 = s.solve(sweeps=2).cpu().numpy()
    torch.cuda.synchronize()
    assert s.status()[0] == 0
    e0, e2 = p_err(p0, p_ref, inst.d), p_err(p2, p_ref, inst.d)
    log(f"ncol {np.dtype(dtype).name} {mode} nB={nB} (cond {cond:.3g}): unrefined {e0:.2e}, two sweeps {e2:.2e}")
    tol0 = (1e-5 if dtype == np.float32 else 1e-12) * max(1.0, cond / 1e3)
    assert e0 <= tol0
    assert e2 <= 1e-10


def test_ncol_uniform_widths_equal_the_uniform_handle():
    """Every block 3 wide: the same factor and p, bit for bit, as qrk_create_blockangular."""
    import torch
    from paper_1802_03773_amd import BlockAngularNcolSolver, BlockAngularSolver
    inst = _instance(3, K=500, nB=30, ncol=np.full(500, 3))
    A, B, b, d = _device(inst)
    s1 = BlockAngularNcolSolver(inst.row_off, inst.ncol, 30)
    s1.factor(A, B, b, d, inst.lam)
    s2 = BlockAngularSolver(inst.row_off, 3, 30)
    s2.factor(A.view(inst.M, 3), B, b, d, inst.lam)
    for x, y in zip(s1.get_factor(), s2.get_factor()):
        assert torch.equal(x, y)
    assert torch.equal(s1.solve(sweeps=1), s2.solve(sweeps=1))


def test_ncol_solve_tol():
    import torch
    from paper_1802_03773_amd import BlockAngularNcolSolver
    inst = _instance(41, nB=60)
    p_ref, _ = _reference(inst)
    s = BlockAngularNcolSolver(inst.row_off, inst.ncol, 60, mode="bf16x3")
    A, B, b, d = _device(inst)
    s.factor(A, B, b, d, inst.lam)
    p, sweeps, converged = s.solve_tol(max_sweeps=4, rel_tol=1e-13)
    torch.cuda.synchronize()
    e = p_err(p.cpu().numpy(), p_ref, inst.d)
    log(f"ncol solve_tol: {sweeps} sweeps, converged {converged}, error {e:.2e}")
    assert converged and 1 <= sweeps <= 4 and e <= 1e-10


def test_ncol_refusals():
    """lambda = 0 (the added unknowns would have no damping) and the calls this handle does not
    take are refused."""
    import torch
    from paper_1802_03773_amd import BlockAngularNcolSolver, QRKError
    inst = _instance(51, K=60, nB=10)
    A, B, b, d = _device(inst)
    s = BlockAngularNcolSolver(inst.row_off, inst.ncol, 10)
    with pytest.raises(QRKError):
        s.factor(A, B, b, d, 0.0)
    s.factor(A, B, b, d, 1e-2)
    with pytest.raises(QRKError):
        s.solve_rhs(b)
    with pytest.raises(QRKError):
        s.set_keep_q(True)
    with pytest.raises(QRKError):
        s.factor_lambda(1e-2)
    p = s.solve(sweeps=1)
    with pytest.raises(QRKError):
        s.solve_adjoint(p, torch.ones_like(p))
    torch.cuda.synchronize()
