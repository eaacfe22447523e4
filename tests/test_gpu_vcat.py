"""Vertical concatenation (qrk_factor_vcat through the C ABI, Section 4.5) against the oracle: the
merged factor of two (or three) factored problems over the same columns equals the oracle's
vertical concatenation of its own factors, and the factor of the problem with all the rows, up to
the sign of each row of R; the solution (unrefined, and refined against every part's rows) equals
the oracle's least-squares solution of the stacked problem."""
import dataclasses

import numpy as np
import pytest

from oracle import refine, structured
from tests.gpu_util import log, p_err, sign_fix_rows, to_device
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _parts(seed, K, nB, dtype, parts=2, lam2=0.0):
    base = gen.make_blockangular(seed, K=K, m=(np.arange(K) % 7) + 6, n=3, nB=nB, lam=1e-2, dtype=dtype)
    out = [base]
    for k in range(1, parts):
        o = gen.make_blockangular(seed + 31 * k, K=K, m=(np.arange(K) * (k + 2)) % 5 + 3, n=3, nB=nB, lam=lam2,
                                  dtype=dtype)
        out.append(dataclasses.replace(o, d=base.d.copy()))
    return out


def _factor(inst, mode="plain"):
    from paper_1802_03773_amd import BlockAngularSolver
    dev = to_device(inst)
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype=np.dtype(inst.dtype).name, mode=mode)
    s.factor(*dev, inst.lam)
    return s, dev


def _check_factor(solver, f, tol):
    Rblk, S, RB = [t.cpu().numpy().astype(np.float64) for t in solver.get_factor()]
    K, nB = Rblk.shape[0], RB.shape[0] - 1
    for i in range(0, K, max(1, K // 64)):
        Rg, Sg = sign_fix_rows(Rblk[i], S[i])
        Ro, So = sign_fix_rows(f.R_blk[i], np.concatenate([f.S[i], f.c_blk[i][:, None]], axis=1))
        scale = max(np.abs(Ro).max(), np.abs(So).max())
        assert np.abs(Rg - Ro).max() <= tol * scale, f"R_{i}"
        assert np.abs(Sg - So).max() <= tol * scale, f"S_{i}"
    if nB:
        Rg, cg = sign_fix_rows(RB[:nB, :nB], RB[:nB, nB])
        Ro, co = sign_fix_rows(f.R_B, f.c_B)
        scale = max(np.abs(Ro).max(), np.abs(co).max())
        assert np.abs(Rg - Ro).max() <= tol * scale
        assert np.abs(cg - co).max() <= tol * scale
    assert abs(abs(RB[nB, nB]) - f.resid) <= tol * max(1.0, f.resid) * 10


@pytest.mark.parametrize("dtype,mode", [(np.float64, "plain"), (np.float32, "plain"), (np.float32, "bf16x3")])
@pytest.mark.parametrize("nB", [0, 40, 100])
def test_vcat_two_parts(dtype, mode, nB):
    i1, i2 = _parts(1100 + nB, 300, nB, dtype)
    f1, f2 = structured.factor_blockangular(i1), structured.factor_blockangular(i2)
    stacked = gen.stack_rows([i1, i2])
    p_ref, f_direct = refine.reference_solution(stacked)
    s1, d1 = _factor(i1, mode)
    s2, d2 = _factor(i2, mode)
    s1.factor_vcat(s2)
    tol_f = 1e-12 if dtype == np.float64 else 2e-5
    _check_factor(s1, structured.factor_vcat(f1, f2), tol_f)
    _check_factor(s1, f_direct, tol_f)
    p0 = s1.solve(sweeps=0).cpu().numpy()
    p2 = s1.solve(sweeps=2).cpu().numpy()
    e0, e2 = p_err(p0, p_ref, stacked.d), p_err(p2, p_ref, stacked.d)
    log(f"vcat {np.dtype(dtype).name} {mode} nB={nB}: unrefined {e0:.2e}, two sweeps {e2:.2e}")
    assert s1.status()[0] == 0
    assert e0 <= (1e-12 if dtype == np.float64 else 1e-5)
    assert e2 <= 1e-10


def test_vcat_three_parts_and_damped_second_part():
    """Three parts, the second and third damped as well (the stacked problem's damping is then
    the sum of the parts': the same D, so lam1 + lam2 + lam3), refined against all their rows."""
    lam2 = 3e-3
    i1, i2, i3 = _parts(1130, 250, 60, np.float32, parts=3, lam2=lam2)
    stacked = dataclasses.replace(gen.stack_rows([i1, i2, i3]), lam=i1.lam + 2 * lam2)
    p_ref, _ = refine.reference_solution(stacked)
    s1, _ = _factor(i1, "bf16x3")
    s2, _ = _factor(i2, "bf16x3")
    s3, _ = _factor(i3, "bf16x3")
    s1.factor_vcat(s2)
    s1.factor_vcat(s3)
    p0 = s1.solve(sweeps=0).cpu().numpy()
    p2 = s1.solve(sweeps=2).cpu().numpy()
    e0, e2 = p_err(p0, p_ref, stacked.d), p_err(p2, p_ref, stacked.d)
    log(f"vcat three parts: unrefined {e0:.2e}, two sweeps {e2:.2e}")
    assert e0 <= 1e-5
    assert e2 <= 1e-10
    p_tol, sweeps, converged = s1.solve_tol(max_sweeps=4, rel_tol=1e-13)
    assert converged and p_err(p_tol.cpu().numpy(), p_ref, stacked.d) <= 1e-10


def test_vcat_rules_and_refactor():
    """Mismatched handles and a handle with itself are refused; the stacked factor refuses the calls
    that need its rows' b or a factor of its own rows alone; a new factor call drops the parts."""
    import torch
    from paper_1802_03773_amd import QRKError
    i1, i2 = _parts(1150, 80, 20, np.float32)
    s1, d1 = _factor(i1)
    s2, _ = _factor(i2)
    other = gen.make_blockangular(1151, K=80, m=6, n=3, nB=21, lam=0.0, dtype=np.float32)
    s3, _ = _factor(other)
    with pytest.raises(QRKError):
        s1.factor_vcat(s3)  # another nB
    with pytest.raises(QRKError):
        s1.factor_vcat(s1)
    s1.factor_vcat(s2)
    with pytest.raises(QRKError):
        s1.solve_rhs(torch.zeros(i1.M, dtype=torch.float32, device="cuda"), sweeps=2)
    with pytest.raises(QRKError):
        s1.factor_lambda(1e-2)
    with pytest.raises(QRKError):
        s2.factor_vcat(s1)  # s1 holds a concatenation
    # a new factor call of s1: its own rows only again
    s1.factor(*d1, i1.lam)
    p_ref, _ = refine.reference_solution(i1)
    assert p_err(s1.solve(sweeps=2).cpu().numpy(), p_ref, i1.d) <= 1e-10
