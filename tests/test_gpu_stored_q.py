"""Stored Q (qrk_set_keep_q, qrk_apply_qt and qrk_solve_qt through the C ABI) against the oracle.

For a new right-hand side b2 with the same J, d and lambda, the oracle's structured factorisation
of [J | b2] gives R and c(b2); Q^T b2 from the stored reflectors must match c(b2) up to the sign of
each row of R (the stored factor gives the GPU's signs), and p = R^{-1} Q^T b2 must match the
oracle's solution for b2.  Float32 block-angular handles: fp32 and BF16x3 dense-part updates; one
problem with the pipelined merge tree (one leaf, even and odd leaf counts); dense parts wider than
six column blocks, whose leaves merge inside the leaf launch; ragged batches over several dense
widths (the persistent leaf launch).  Tolerances as for the factor itself: float32 unrefined 1e-5
at cond(J) <= 1e3 (2e-5 for the factor's entries), 1e-10 after one refinement sweep."""
import dataclasses

import numpy as np
import pytest

from oracle import dense, refine
from tests.gpu_util import log, p_err, sign_fix_rows, to_device
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _new_b(inst, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(inst.b.shape[0]).astype(inst.dtype)


def _check_c(solver, inst, c, f2, tol):
    """c (Q^T b2, laid out like p) against the oracle's c of [J | b2], up to the row signs of R."""
    Rblk, _, RB = [t.cpu().numpy().astype(np.float64) for t in solver.get_factor()]
    K, n, nB = inst.K, inst.n, inst.nB
    worst = 0.0
    for i in range(0, K, max(1, K // 64)):
        Rg, cg = sign_fix_rows(Rblk[i], c[i * n:(i + 1) * n])
        Ro, co = sign_fix_rows(f2.R_blk[i], f2.c_blk[i])
        e = np.abs(cg - co).max() / max(np.abs(co).max(), np.abs(Ro).max())
        worst = max(worst, e)
        assert e <= tol, f"c_{i}: {e:.2e}"
    if nB:
        Rg, cg = sign_fix_rows(RB[:nB, :nB], c[K * n:])
        Ro, co = sign_fix_rows(f2.R_B, f2.c_B)
        e = np.abs(cg - co).max() / max(np.abs(co).max(), np.abs(Ro).max())
        worst = max(worst, e)
        assert e <= tol, f"c_B: {e:.2e}"
    return worst


def _solver(inst, mode, leaves=0):
    from paper_1802_03773_amd import BlockAngularSolver
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode=mode)
    if leaves:
        s.set_tsqr_shape(leaves=leaves)
    s.set_keep_q(True)
    return s


@pytest.mark.parametrize("leaves", [0, 1, 8, 5])
@pytest.mark.parametrize("mode", ["plain", "bf16x3"])
def test_apply_qt_single_problem(mode, leaves):
    """Three dense column blocks (the pipelined merge tree unless there is one leaf): the default
    leaf count (29 leaves), one, eight and five (a carried leaf at two levels)."""
    import torch
    inst = gen.make_blockangular(1001, K=400, m=(np.arange(400) % 7) + 6, n=3, nB=40, lam=1e-2,
                                 dtype=np.float32)
    b2 = _new_b(inst, 1002)
    p_ref2, f2 = refine.reference_solution(dataclasses.replace(inst, b=b2))
    A, B, b, d = to_device(inst)
    s = _solver(inst, mode, leaves)
    s.factor(A, B, b, d, inst.lam)
    b2d = torch.from_numpy(b2).cuda()
    c = s.apply_qt(b2d).cpu().numpy()
    ec = _check_c(s, inst, c, f2, 2e-5)
    p0 = s.solve_qt(b2d, sweeps=0).cpu().numpy()
    p1 = s.solve_qt(b2d, sweeps=1).cpu().numpy()
    e0, e1 = p_err(p0, p_ref2, inst.d), p_err(p1, p_ref2, inst.d)
    log(f"stored Q {mode} leaves={leaves}: c {ec:.2e}, p unrefined {e0:.2e}, one sweep {e1:.2e}")
    assert s.status()[0] == 0
    assert e0 <= 1e-5
    assert e1 <= 1e-10


@pytest.mark.parametrize("mode", ["plain", "bf16x3"])
def test_apply_qt_own_rhs_is_the_factor_c(mode):
    """Q^T b for the factor call's own b reproduces the c the factorisation carried as a column.
    Storing Q leaves the per-block factor bit for bit as it is without; at 6 column blocks the
    leaves that store Q stream 64-row tiles where the others stream 128, so R_B | c_B agrees up to
    row signs and rounding."""
    import torch
    from paper_1802_03773_amd import BlockAngularSolver
    inst = gen.make_blockangular(1011, K=1500, m=(np.arange(1500) % 5) + 8, n=3, nB=90, lam=1e-2,
                                 dtype=np.float32)
    A, B, b, d = to_device(inst)
    s = _solver(inst, mode)
    s.factor(A, B, b, d, inst.lam)
    ref = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode=mode)
    ref.factor(A, B, b, d, inst.lam)
    fk = s.get_factor()
    fr = ref.get_factor()
    assert torch.equal(fk[0], fr[0]) and torch.equal(fk[1], fr[1])
    RBk = sign_fix_rows(fk[2].cpu().numpy())[0]
    RBr = sign_fix_rows(fr[2].cpu().numpy())[0]
    eRB = np.abs(RBk - RBr).max() / np.abs(RBr).max()
    log(f"R_B | c_B with and without the stored Q ({mode}): {eRB:.2e}")
    assert eRB <= (1e-5 if mode == "plain" else 1e-4)
    c = s.apply_qt(b).cpu().numpy()
    _, S, RB = [t.cpu().numpy().astype(np.float64) for t in fk]
    K, n, nB = inst.K, inst.n, inst.nB
    c_fac = np.concatenate([S[:, :, nB].reshape(-1), RB[:nB, nB]])
    e = np.abs(c - c_fac).max() / np.abs(c_fac).max()
    log(f"own right-hand side {mode}: max |c - c_factor| / max |c| = {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("mode", ["plain", "bf16x3"])
@pytest.mark.parametrize("nB", [90, 100, 127])
def test_apply_qt_wide_dense_part(nB, mode):
    """Six column blocks (the pipelined merge tree), seven and eight (merges inside the leaf
    launch): tiles of 64 rows."""
    import torch
    inst = gen.make_blockangular(1021 + nB, K=600, m=(np.arange(600) % 9) + 4, n=3, nB=nB, lam=1e-2,
                                 dtype=np.float32)
    b2 = _new_b(inst, 1022)
    p_ref2, f2 = refine.reference_solution(dataclasses.replace(inst, b=b2))
    A, B, b, d = to_device(inst)
    s = _solver(inst, mode)
    s.factor(A, B, b, d, inst.lam)
    b2d = torch.from_numpy(b2).cuda()
    ec = _check_c(s, inst, s.apply_qt(b2d).cpu().numpy(), f2, 2e-5)
    e0 = p_err(s.solve_qt(b2d).cpu().numpy(), p_ref2, inst.d)
    e1 = p_err(s.solve_qt(b2d, sweeps=1).cpu().numpy(), p_ref2, inst.d)
    log(f"stored Q nB={nB} {mode}: c {ec:.2e}, p unrefined {e0:.2e}, one sweep {e1:.2e}")
    assert e0 <= 1e-5
    assert e1 <= 1e-10


@pytest.mark.parametrize("mode", ["plain", "bf16x3"])
@pytest.mark.parametrize("scale_k", [0.0, 3.0])
def test_solve_qt_ragged_batch(scale_k, mode):
    """Dense widths 1, 2, 5, 6 and 8 column blocks in one batch (the persistent leaf launch for
    the widths up to six), column scales 1 and 10^(3t).  With the scales some of these small
    problems pass cond(J) = 1e3, where the unrefined bound is stated; above it the bound scales
    with the condition number, and two sweeps reach 1e-10."""
    import torch
    from paper_1802_03773_amd import BlockAngularBatch
    insts = [gen.make_blockangular(1030 + k, K=K, m=(np.arange(K) % 5) + 4, n=3, nB=nB, lam=1e-2,
                                   dtype=np.float32, scale_k=scale_k)
             for k, (K, nB) in enumerate([(120, 30), (40, 6), (75, 0), (200, 90), (150, 70), (90, 127)])]
    st = gen.stack_batch(insts)
    dev = {k: torch.from_numpy(np.ascontiguousarray(st[k])).cuda() for k in ("A", "B", "b", "d", "lam")}
    bt = BlockAngularBatch(st["K"], st["nB"], st["row_off"], st["n"], dtype="float32", mode=mode)
    bt.set_keep_q(True)
    bt.factor(dev["A"], dev["B"], dev["b"], dev["d"], dev["lam"])
    b2s = [_new_b(i, 1040 + q) for q, i in enumerate(insts)]
    b2d = torch.from_numpy(np.concatenate(b2s)).cuda()
    p0 = bt.solve_qt(b2d).cpu().numpy()
    p2 = bt.solve_qt(b2d, sweeps=2).cpu().numpy()
    offs = np.concatenate([[0], np.cumsum([i.N for i in insts])])
    for q, inst in enumerate(insts):
        p_ref, _ = refine.reference_solution(dataclasses.replace(inst, b=b2s[q]))
        Jaug = np.vstack([dense.assemble_blockangular(inst), np.sqrt(inst.lam) * np.diag(inst.d)])
        cond = np.linalg.cond(Jaug)
        e0 = p_err(p0[offs[q]:offs[q + 1]], p_ref, inst.d)
        e2 = p_err(p2[offs[q]:offs[q + 1]], p_ref, inst.d)
        log(f"batch {mode} scale_k={scale_k} problem {q} (nB={inst.nB}, cond {cond:.3g}): unrefined {e0:.2e}, "
            f"two sweeps {e2:.2e}")
        assert e0 <= 1e-5 * max(1.0, cond / 1e3)
        assert e2 <= 1e-10


def test_stored_q_refused_or_stale():
    """A handle with a block of fewer rows than columns, a float64 handle and a banded handle refuse
    to store Q; apply_qt needs a factor that stored it, and the two-stage factor makes it stale."""
    import torch
    from paper_1802_03773_amd import BandedSolver, BlockAngularSolver, QRKError
    short = gen.make_blockangular(1050, K=20, m=(np.arange(20) % 6), n=3, nB=4, lam=1e-2, dtype=np.float32)
    with pytest.raises(QRKError):
        BlockAngularSolver(short.row_off, short.n, short.nB, dtype="float32").set_keep_q(True)
    inst = gen.make_blockangular(1051, K=50, m=8, n=3, nB=10, lam=0.0, dtype=np.float32)
    with pytest.raises(QRKError):
        BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float64").set_keep_q(True)
    with pytest.raises(QRKError):
        BandedSolver(40, 30, 4, dtype="float32").set_keep_q(True)
    A, B, b, d = to_device(inst)
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32")
    s.factor(A, B, b, d, 0.0)
    with pytest.raises(QRKError):
        s.apply_qt(b)  # Q was not stored
    s.set_keep_q(True)
    s.factor(A, B, b, d, 0.0)
    s.apply_qt(b)
    with pytest.raises(QRKError):
        s.solve_qt(b, sweeps=9)
    s.factor_lambda(1e-2)
    with pytest.raises(QRKError):
        s.apply_qt(b)  # stale after the two-stage factor
    torch.cuda.synchronize()
