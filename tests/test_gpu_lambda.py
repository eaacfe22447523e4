"""GPU parity of Moré's two-stage damping (Section 5.2, Eq. LMTwoStep; qrk_factor_lambda): the
factor of [R; sqrt(lam) D] built from the kept factor of J, against the oracle's two-stage
factor (up to row signs) and the directly damped solution.  Tolerances: float64 1e-12 vs the
longdouble-refined reference; float32 unrefined 1e-5; refined 1e-10."""
import dataclasses

import numpy as np
import pytest

from oracle import refine, structured
from tests.gpu_util import p_err, log, rel_err, sign_fix_rows, to_device
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _solver(inst, mode="plain"):
    from paper_1802_03773_amd import BlockAngularSolver
    return BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype=np.dtype(inst.dtype).name, mode=mode)


def _check_factor(inst, s, f, tol):
    Rblk, S, RB = [t.cpu().numpy().astype(np.float64) for t in s.get_factor()]
    nB = inst.nB
    for i in range(0, inst.K, max(1, inst.K // 32)):
        Rg, Sg = sign_fix_rows(Rblk[i], S[i])
        Ro, So = sign_fix_rows(f.R_blk[i], np.concatenate([f.S[i], f.c_blk[i][:, None]], axis=1))
        assert np.abs(Rg - Ro).max() <= tol * np.abs(Ro).max(), f"R_{i}"
        assert np.abs(Sg - So).max() <= tol * max(np.abs(So).max(), np.abs(Ro).max()), f"S_{i}"
    Rg, cg = sign_fix_rows(RB[:nB, :nB], RB[:nB, nB])
    Ro, co = sign_fix_rows(f.R_B, f.c_B)
    assert np.abs(Rg - Ro).max() <= tol * np.abs(Ro).max()
    assert np.abs(cg - co).max() <= tol * max(np.abs(co).max(), np.abs(Ro).max())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_two_stage_tiny(dtype):
    """100 blocks of 8x3 + 800x24: one factor of J, then three damping values."""
    import torch
    inst = gen.tiny_blockangular(3, dtype=dtype, lam=0.0)
    s = _solver(inst)
    A, B, b, d = to_device(inst)
    s.factor(A, B, b, d, 0.0)
    for lam in (1e-4, 1e-2, 1.0):
        log(f"two-stage tiny {np.dtype(dtype).name} lam={lam}")
        s.factor_lambda(lam)
        p0 = s.solve(sweeps=0).cpu().numpy()
        p2 = s.solve(sweeps=2).cpu().numpy()
        s.raise_on_status()
        inst_l = dataclasses.replace(inst, lam=lam)
        p_ref, _ = refine.reference_solution(inst_l)
        if dtype == np.float64:
            assert p_err(p0, p_ref, inst_l.d) <= 1e-12
            _check_factor(inst, s, structured.factor_two_stage(inst, lam), 1e-11)
        else:
            assert p_err(p0, p_ref, inst_l.d) <= 1e-5
            _check_factor(inst, s, structured.factor_two_stage(inst, lam), 2e-4)
        assert p_err(p2, p_ref, inst_l.d) <= 1e-10
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", ["plain", "bf16x3"])
def test_two_stage_scale_k_and_many_leaves(mode):
    """5,000 blocks of 12x3 + 60,000x90 with column scales logspace(0,3): the second stage's
    dense part has 15,091 rows over many leaves and the pipelined tree; refined to 1e-10."""
    inst = gen.make_blockangular(51, K=5000, m=12, n=3, nB=90, lam=0.0, dtype=np.float32, scale_k=3.0)
    s = _solver(inst, mode)
    A, B, b, d = to_device(inst)
    s.factor(A, B, b, d, 0.0)
    for lam in (1e-2, 1e-4):
        log(f"two-stage K=5000 {mode} lam={lam}")
        s.factor_lambda(lam)
        p1 = s.solve(sweeps=2).cpu().numpy()
        s.raise_on_status()
        p_ref, _ = refine.reference_solution(dataclasses.replace(inst, lam=lam))
        assert p_err(p1, p_ref, inst.d) <= 1e-10


def test_two_stage_new_base_and_errors():
    from paper_1802_03773_amd import qrkit
    inst = gen.tiny_blockangular(4, dtype=np.float32, lam=0.0)
    s = _solver(inst)
    L = qrkit.lib()
    # before any factor
    assert L.qrk_factor_lambda(s._h, 1e-2, None) == qrkit.QRK_EINVAL
    A, B, b, d = to_device(inst)
    # a damped factor is not a factor of J alone
    s.factor(A, B, b, d, 1e-2)
    assert L.qrk_factor_lambda(s._h, 1e-2, None) == qrkit.QRK_EINVAL
    s.factor(A, B, b, d, 0.0)
    assert L.qrk_factor_lambda(s._h, 0.0, None) == qrkit.QRK_EINVAL
    assert L.qrk_factor_lambda(s._h, float("nan"), None) == qrkit.QRK_EINVAL
    s.factor_lambda(1e-2)
    p_ref, _ = refine.reference_solution(dataclasses.replace(inst, lam=1e-2))
    assert p_err(s.solve(sweeps=2).cpu().numpy(), p_ref, inst.d) <= 1e-10
    # a new factor of J (other data) replaces the kept one
    inst2 = gen.tiny_blockangular(5, dtype=np.float32, lam=0.0)
    A2, B2, b2, d2 = to_device(inst2)
    s.factor(A2, B2, b2, d2, 0.0)
    s.factor_lambda(1e-1)
    p_ref2, _ = refine.reference_solution(dataclasses.replace(inst2, lam=1e-1))
    assert p_err(s.solve(sweeps=2).cpu().numpy(), p_ref2, inst2.d) <= 1e-10


@pytest.mark.parametrize("nB", [0, 5])
def test_two_stage_small_dense_parts(nB):
    """No dense part (the second stage's dense part is only the residual row) and a narrow one."""
    inst = gen.make_blockangular(61 + nB, K=40, m=6, n=3, nB=nB, lam=0.0, dtype=np.float64)
    s = _solver(inst)
    A, B, b, d = to_device(inst)
    s.factor(A, B, b, d, 0.0)
    for lam in (1e-3, 0.5):
        s.factor_lambda(lam)
        p = s.solve(sweeps=1).cpu().numpy()
        s.raise_on_status()
        p_ref, _ = refine.reference_solution(dataclasses.replace(inst, lam=lam))
        assert p_err(p, p_ref, inst.d) <= 1e-12
