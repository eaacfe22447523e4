"""New right-hand sides with the stored factor (qrk_solve_rhs through the C ABI) against the
oracle's solution of the same least-squares problem with that right-hand side: block-angular
(float32 with fp32 and BF16x3 updates, float64), a ragged batch and banded problems.  The
handle's own right-hand side is left as it was: qrk_solve afterwards still returns its step."""
import dataclasses

import numpy as np
import pytest

from oracle import banded as obanded
from oracle import refine
from tests.gpu_util import p_err, log, rel_err, to_device
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _new_b(inst, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(inst.b.shape[0]).astype(inst.dtype)


@pytest.mark.parametrize("scale_k", [0.0, 3.0])
@pytest.mark.parametrize("dtype,mode", [(np.float32, "plain"), (np.float32, "bf16x3"), (np.float64, "plain")])
def test_blockangular_new_rhs(dtype, mode, scale_k):
    """Unscaled columns and column scales 10^(3t) (cond(J) about 1e3): four sweeps, the count
    the header states and the binding's default, reach 1e-10."""
    import torch
    from paper_1802_03773_amd import BlockAngularSolver
    inst = gen.make_blockangular(901, K=500, m=(np.arange(500) % 7) + 6, n=3, nB=40, lam=1e-2, dtype=dtype,
                                 scale_k=scale_k)
    b2 = _new_b(inst, 902)
    p_ref2, _ = refine.reference_solution(dataclasses.replace(inst, b=b2))
    p_ref1, _ = refine.reference_solution(inst)
    A, B, b, d = to_device(inst)
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype=str(inst.dtype), mode=mode)
    s.factor(A, B, b, d, inst.lam)
    b2d = torch.from_numpy(b2).cuda()
    errs = {}
    for sweeps in (1, 2, 3, 4):
        p2 = s.solve_rhs(b2d, sweeps=sweeps)
        torch.cuda.synchronize()
        errs[sweeps] = p_err(p2.cpu().numpy(), p_ref2, inst.d)
    log(f"block-angular {np.dtype(dtype).name} {mode} scale_k={scale_k}: error by sweeps {errs}")
    assert s.status()[0] == 0
    assert errs[4] <= 1e-10
    assert errs[2] < errs[1]
    p1 = s.solve(sweeps=2)
    assert p_err(p1.cpu().numpy(), p_ref1, inst.d) <= 1e-10


@pytest.mark.parametrize("scale_k", [0.0, 3.0])
def test_blockangular_batch_new_rhs(scale_k):
    import torch
    from paper_1802_03773_amd import BlockAngularBatch
    insts = [gen.make_blockangular(910 + k, K=K, m=(np.arange(K) % 5) + 4, n=3, nB=nB, lam=1e-2, dtype=np.float32,
                                   scale_k=scale_k)
             for k, (K, nB) in enumerate([(120, 30), (40, 6), (75, 0), (200, 90)])]
    st = gen.stack_batch(insts)
    dev = {k: torch.from_numpy(np.ascontiguousarray(st[k])).cuda() for k in ("A", "B", "b", "d", "lam")}
    bt = BlockAngularBatch(st["K"], st["nB"], st["row_off"], st["n"], dtype="float32")
    bt.factor(dev["A"], dev["B"], dev["b"], dev["d"], dev["lam"])
    b2s = [_new_b(i, 920 + q) for q, i in enumerate(insts)]
    p2 = bt.solve_rhs(torch.from_numpy(np.concatenate(b2s)).cuda()).cpu().numpy()  # default: 4 sweeps
    offs = np.concatenate([[0], np.cumsum([i.N for i in insts])])
    for q, inst in enumerate(insts):
        p_ref, _ = refine.reference_solution(dataclasses.replace(inst, b=b2s[q]))
        e = p_err(p2[offs[q]:offs[q + 1]], p_ref, inst.d)
        log(f"batch problem {q}: {e:.2e}")
        assert e <= 1e-10


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_banded_new_rhs(dtype):
    import torch
    from paper_1802_03773_amd import BandedSolver
    insts = [gen.make_banded(930 + k, N=300, w=7, lam=1e-2, dtype=dtype) for k in range(3)]
    i0 = insts[0]
    s = BandedSolver(i0.M, i0.N, i0.w, dtype=np.dtype(dtype).name, P=len(insts))
    rs = torch.from_numpy(np.stack([i.row_start for i in insts])).cuda()
    vals = torch.from_numpy(np.stack([i.vals for i in insts])).cuda()
    b = torch.from_numpy(np.stack([i.b for i in insts])).cuda()
    d = torch.from_numpy(np.stack([i.d for i in insts])).cuda()
    s.factor(rs, vals, b, d, i0.lam)
    b2s = [_new_b(i, 940 + q) for q, i in enumerate(insts)]
    p2 = s.solve_rhs(torch.from_numpy(np.stack(b2s)).cuda(), sweeps=4).cpu().numpy().reshape(len(insts), -1)
    for q, inst in enumerate(insts):
        p_ref, _, _ = obanded.reference_solution(dataclasses.replace(inst, b=b2s[q]))
        e = p_err(p2[q], p_ref, inst.d)
        log(f"banded {np.dtype(dtype).name} problem {q}: {e:.2e}")
        assert e <= 1e-10
    p1 = s.solve(sweeps=2).cpu().numpy().reshape(len(insts), -1)
    p_ref1, _, _ = obanded.reference_solution(insts[0])
    assert p_err(p1[0], p_ref1, insts[0].d) <= 1e-10


def test_rejects_bad_arguments():
    import torch
    from paper_1802_03773_amd import BlockAngularSolver, QRKError
    inst = gen.make_blockangular(950, K=10, m=6, n=3, nB=4, lam=1e-2, dtype=np.float32)
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32")
    b2 = torch.zeros(inst.b.shape[0], dtype=torch.float32, device="cuda")
    with pytest.raises(QRKError):
        s.solve_rhs(b2, sweeps=2)  # no factor yet
    A, B, b, d = to_device(inst)
    s.factor(A, B, b, d, inst.lam)
    for sweeps in (0, 9):
        with pytest.raises(QRKError):
            s.solve_rhs(b2, sweeps=sweeps)


def test_new_rhs_after_two_stage_factor():
    """J factored at lambda = 0, then the two-stage factor of [R; sqrt(lambda) D]: a new right-hand
    side is solved with that lambda."""
    import torch
    from paper_1802_03773_amd import BlockAngularSolver
    inst = gen.make_blockangular(960, K=300, m=(np.arange(300) % 7) + 6, n=3, nB=30, lam=0.0, dtype=np.float32)
    lam = 1e-2
    b2 = _new_b(inst, 961)
    p_ref, _ = refine.reference_solution(dataclasses.replace(inst, b=b2, lam=lam))
    A, B, b, d = to_device(inst)
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32")
    s.factor(A, B, b, d, 0.0)
    s.factor_lambda(lam)
    p2 = s.solve_rhs(torch.from_numpy(b2).cuda(), sweeps=4)
    torch.cuda.synchronize()
    e = p_err(p2.cpu().numpy(), p_ref, inst.d)
    log(f"two-stage factor, new right-hand side: {e:.2e}")
    assert s.status()[0] == 0
    assert e <= 1e-10
