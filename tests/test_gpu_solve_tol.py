"""qrk_solve_tol (refinement with an early stop on ||delta|| <= rel_tol ||p||) against the oracle:
it stops once every problem meets the tolerance, with the same p as qrk_solve with that many
sweeps; when the sweeps run out first it returns QRK_ENOTCONVERGED, keeps the last iterate, and
qrk_status_get reports the condition until the next factor call."""
import numpy as np
import pytest

from oracle import banded, refine
from tests.gpu_util import log, p_err, to_device
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def test_blockangular_solve_tol_stops_early_and_matches_fixed_sweeps():
    import torch
    from paper_1802_03773_amd import BlockAngularSolver, qrkit
    inst = gen.make_blockangular(1700, K=800, m=(np.arange(800) % 9) + 4, n=3, nB=40, lam=1e-2,
                                 dtype=np.float32, scale_k=3.0)
    p_ref, _ = refine.reference_solution(inst)
    A, B, b, d = to_device(inst)
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32")
    s.factor(A, B, b, d, inst.lam)
    p, done, ok = s.solve_tol(max_sweeps=6, rel_tol=1e-13)
    log(f"block-angular: {done} sweeps, converged {ok}, error {p_err(p.cpu().numpy(), p_ref, inst.d):.2e}")
    assert ok and 1 <= done < 6
    assert p_err(p.cpu().numpy(), p_ref, inst.d) <= 1e-10
    fixed = s.solve(sweeps=done).cpu().numpy()
    assert np.array_equal(fixed, p.cpu().numpy())
    assert s.status()[0] == qrkit.QRK_OK


def test_blockangular_solve_tol_reports_not_converged():
    """A zero tolerance is never met: every sweep runs, p is the last iterate (still at 1e-10),
    and the condition shows in qrk_status_get until the next factor."""
    import torch
    from paper_1802_03773_amd import BlockAngularSolver, qrkit
    inst = gen.make_blockangular(1701, K=300, m=8, n=3, nB=20, lam=1e-2, dtype=np.float32)
    p_ref, _ = refine.reference_solution(inst)
    A, B, b, d = to_device(inst)
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32")
    s.factor(A, B, b, d, inst.lam)
    p, done, ok = s.solve_tol(max_sweeps=2, rel_tol=0.0)
    assert not ok and done == 2
    assert p_err(p.cpu().numpy(), p_ref, inst.d) <= 1e-10
    st, bits = s.status()
    assert st == qrkit.QRK_ENOTCONVERGED and bits & 16
    s.factor(A, B, b, d, inst.lam)  # the next factor clears it
    assert s.status()[0] == qrkit.QRK_OK
    p0, done, ok = s.solve_tol(max_sweeps=0, rel_tol=0.0)
    assert ok and done == 0
    assert np.array_equal(p0.cpu().numpy(), s.solve(sweeps=0).cpu().numpy())


def test_banded_batch_solve_tol():
    import torch
    from paper_1802_03773_amd import BandedSolver
    insts = [gen.make_banded(1710 + k, N=300, w=9, lam=1e-2, dtype=np.float32) for k in range(5)]
    i0 = insts[0]
    s = BandedSolver(i0.M, i0.N, i0.w, dtype="float32", P=len(insts))
    dev = [torch.from_numpy(np.stack([getattr(i, k) for i in insts])).cuda() for k in ("row_start", "vals", "b", "d")]
    s.factor(*dev, i0.lam)
    p, done, ok = s.solve_tol(max_sweeps=5, rel_tol=1e-13)
    assert ok and 1 <= done < 5
    p = p.cpu().numpy().reshape(len(insts), -1)
    for k, inst in enumerate(insts):
        p_ref, _, _ = banded.reference_solution(inst)
        assert p_err(p[k], p_ref, inst.d) <= 1e-10
