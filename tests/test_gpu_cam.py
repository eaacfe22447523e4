"""Camera columns (qrk_create_blockangular_cam: the bundle-adjustment Jacobian of Section 6.2,
each row on one point block and at most one camera) through the C ABI, against the oracle.

The reference is the damped least-squares solution of the assembled J (LAPACK on the dense
matrix; the assembly is pinned in test_oracle_cam.py).  Configurations:
  * 14 cameras of 9 columns (nB = 126, two column slots per lane) and 4 cameras of 6 (nB = 24);
  * points seen by 1..6 cameras, so blocks of 2 rows (fewer rows than the 3 columns) occur;
  * rows without a camera, some with -1 and some with an index past the last camera;
  * float32 with fp32 and BF16x3 dense-part updates, and float64.
Bounds: unrefined as for dense-B problems (float32 1e-5 at cond <= 1e3, scaled by cond / 1e3
above it; float64 1e-12), 1e-10 after two sweeps.  The camera handle is also compared bit for
bit with a dense-B handle given the assembled B: the kernels read the same values.  The
autotuner and HIP-graph replay of the step read the camera rows as eager calls do."""
import numpy as np
import pytest

from oracle import dense, structured
from tests.gpu_util import log, p_err
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _instance(seed, K=400, ncam=14, cw=9, lam=1e-2, dtype=np.float32, prior_rows=1, obs=None):
    if obs is None:
        obs = (np.arange(K) * 7 + seed) % min(ncam, 6) + 1
    inst = gen.make_blockangular_cam(seed, K=K, obs=obs, ncam=ncam, cw=cw, n=3, lam=lam, prior_rows=prior_rows,
                                     dtype=dtype)
    # a few rows without a camera given as an index past the last one
    none = np.nonzero(inst.cam < 0)[0]
    inst.cam[none[::3]] = ncam + 5
    return inst


def _reference(inst, b=None):
    J = dense.assemble_blockangular(dense.blockangular_from_cam(inst))
    Aaug = np.vstack([J, np.sqrt(inst.lam) * np.diag(inst.d)])
    bb = inst.b if b is None else b
    rhs = np.concatenate([bb.astype(np.float64), np.zeros(inst.N)])
    p, *_ = np.linalg.lstsq(Aaug, rhs, rcond=None)
    return p, np.linalg.cond(Aaug)


def _device(inst):
    import torch
    A = torch.from_numpy(np.ascontiguousarray(inst.A)).cuda()
    Bv = torch.from_numpy(np.ascontiguousarray(inst.Bv)).cuda()
    cam = torch.from_numpy(np.ascontiguousarray(inst.cam)).cuda()
    b = torch.from_numpy(np.ascontiguousarray(inst.b)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(inst.d)).cuda()
    return A, Bv, cam, b, d


def _solver(inst, mode="plain"):
    from paper_1802_03773_amd import BlockAngularCamSolver
    return BlockAngularCamSolver(inst.row_off, inst.n, inst.ncam, inst.cw, dtype=np.dtype(inst.dtype).name,
                                 mode=mode)


def _tol0(dtype, cond):
    return (1e-5 if dtype == np.float32 else 1e-12) * max(1.0, cond / 1e3)


@pytest.mark.parametrize("dtype,mode", [(np.float32, "plain"), (np.float32, "bf16x3"), (np.float64, "plain")])
@pytest.mark.parametrize("ncam,cw,prior", [(14, 9, 1), (4, 6, 0)])
def test_cam_matches_oracle(dtype, mode, ncam, cw, prior):
    import torch
    inst = _instance(11 + ncam, ncam=ncam, cw=cw, dtype=dtype, prior_rows=prior)
    assert np.diff(inst.row_off).min() < inst.n or prior > 0  # short blocks when no prior rows
    p_ref, cond = _reference(inst)
    s = _solver(inst, mode)
    A, Bv, cam, b, d = _device(inst)
    log(f"cam {np.dtype(dtype).name} {mode} ncam={ncam} cw={cw} K={inst.K} M={inst.M}")
    s.factor(A, Bv, cam, b, d, inst.lam)
    p0 = s.solve(sweeps=0).cpu().numpy()
    p2 = s.solve(sweeps=2).cpu().numpy()
    torch.cuda.synchronize()
    assert s.status()[0] == 0
    e0, e2 = p_err(p0, p_ref, inst.d), p_err(p2, p_ref, inst.d)
    log(f"  cond {cond:.3g}: unrefined {e0:.2e}, two sweeps {e2:.2e}")
    assert e0 <= _tol0(dtype, cond)
    assert e2 <= 1e-10


@pytest.mark.parametrize("dtype,mode", [(np.float32, "plain"), (np.float32, "bf16x3"), (np.float64, "plain")])
def test_cam_equals_dense_handle(dtype, mode):
    """The same factor and the same refined p, bit for bit, as the dense-B handle given the
    assembled B (the oracle's camera_columns)."""
    import torch
    from paper_1802_03773_amd import BlockAngularSolver
    inst = _instance(5, K=700, dtype=dtype)
    A, Bv, cam, b, d = _device(inst)
    Bd = torch.from_numpy(np.ascontiguousarray(dense.camera_columns(inst).astype(dtype))).cuda()
    s1 = _solver(inst, mode)
    s1.factor(A, Bv, cam, b, d, inst.lam)
    s2 = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype=np.dtype(dtype).name, mode=mode)
    s2.factor(A, Bd, b, d, inst.lam)
    for x, y in zip(s1.get_factor(), s2.get_factor()):
        assert torch.equal(x, y)
    assert torch.equal(s1.solve(sweeps=1), s2.solve(sweeps=1))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_cam_colnorms(dtype):
    """d of the assembled J, with d_j = 1 for cameras no row touches."""
    inst = _instance(21, K=60, ncam=14, cw=9, obs=np.ones(60, dtype=np.int64) + (np.arange(60) % 2), dtype=dtype)
    s = _solver(inst)
    A, Bv, cam, b, d = _device(inst)
    dg = s.colnorms(A, Bv, cam).cpu().numpy()
    J = dense.assemble_blockangular(dense.blockangular_from_cam(inst))
    ref = np.sqrt((J * J).sum(axis=0))
    ref[ref == 0.0] = 1.0
    np.testing.assert_allclose(dg, ref, rtol=1e-12)


def test_cam_two_stage_new_rhs_and_stored_q():
    """qrk_factor_lambda, qrk_solve_rhs and qrk_solve_qt on a camera handle: their refinement
    sweeps read the compressed camera rows."""
    import torch
    inst = _instance(31, K=300)
    A, Bv, cam, b, d = _device(inst)
    rng = np.random.default_rng(3)
    b2 = rng.standard_normal(inst.M).astype(np.float32)
    b2d = torch.from_numpy(b2).cuda()
    # two-stage: J factored at lambda = 0, then [R; sqrt(lam) D] for two lambdas
    s = _solver(inst)
    s.factor(A, Bv, cam, b, d, 0.0)
    for lam in (1e-3, 1.0):
        s.factor_lambda(lam)
        p_ref, _ = _reference(inst.with_lambda(lam))
        e = p_err(s.solve(sweeps=2).cpu().numpy(), p_ref, inst.d)
        log(f"cam two-stage lam={lam}: {e:.2e}")
        assert e <= 1e-10
    # a new right-hand side with the factor at lam
    s.factor(A, Bv, cam, b, d, inst.lam)
    p_ref2, _ = _reference(inst, b=b2)
    e = p_err(s.solve_rhs(b2d, sweeps=4).cpu().numpy(), p_ref2, inst.d)
    log(f"cam new rhs (4 sweeps from 0): {e:.2e}")
    assert e <= 1e-10
    # the same with the stored Q
    s.set_keep_q(True)
    s.factor(A, Bv, cam, b, d, inst.lam)
    e = p_err(s.solve_qt(b2d, sweeps=2).cpu().numpy(), p_ref2, inst.d)
    log(f"cam stored Q: {e:.2e}")
    assert e <= 1e-10
    torch.cuda.synchronize()
    assert s.status()[0] == 0


def test_cam_refusals():
    from paper_1802_03773_amd import QRKError
    inst = _instance(41, K=40)
    s = _solver(inst)
    A, Bv, cam, b, d = _device(inst)
    import torch
    Bd = torch.zeros((inst.M, inst.nB), dtype=torch.float32, device="cuda")
    from paper_1802_03773_amd import BlockAngularSolver
    with pytest.raises(QRKError):
        BlockAngularSolver.factor(s, A, Bd, b, d, inst.lam)         # the dense-B factor call
    with pytest.raises(QRKError):
        BlockAngularSolver.colnorms(s, A, Bd)
    s.factor(A, Bv, cam, b, d, inst.lam)
    p = s.solve(sweeps=1)
    with pytest.raises(QRKError):
        s.solve_adjoint(p, p)


def test_cam_bundle_adjustment_size():
    """A bundle-adjustment-sized problem: 22,106 points seen by 2..6 of 14 cameras of 9
    parameters (about 177,000 rows, nB = 126), float32 BF16x3 with one sweep, against the
    structured oracle on the assembled problem (pinned to LAPACK in test_oracle_cam.py)."""
    import torch
    K = 22106
    obs = 2 + (np.arange(K) * 13) % 5
    inst = _instance(77, K=K, ncam=14, cw=9, obs=obs, prior_rows=0)
    log(f"cam bundle-adjustment size: K={K} M={inst.M} N={inst.N}")
    p_ref, _ = structured.solve_blockangular(dense.blockangular_from_cam(inst))
    s = _solver(inst, "bf16x3")
    A, Bv, cam, b, d = _device(inst)
    s.factor(A, Bv, cam, b, d, inst.lam)
    p1 = s.solve(sweeps=1).cpu().numpy()
    torch.cuda.synchronize()
    assert s.status()[0] == 0
    e1 = p_err(p1, p_ref, inst.d)
    log(f"  one sweep: {e1:.2e}")
    assert e1 <= 1e-10


def test_cam_autotune_and_graph_replay():
    """The autotuner's trial factors and a captured factor + solve read the camera rows as an
    eager call does: after autotuning p still matches the oracle, and every graph replay (with
    eager work between replays) gives p bit for bit equal to the eager step."""
    import torch
    inst = _instance(51, K=2000, obs=(np.arange(2000) % 5) + 2, prior_rows=1)
    p_ref, _ = structured.solve_blockangular(dense.blockangular_from_cam(inst))
    s = _solver(inst, "bf16x3")
    A, Bv, cam, b, d = _device(inst)
    s.factor(A, Bv, cam, b, d, inst.lam)
    s.autotune()
    s.factor(A, Bv, cam, b, d, inst.lam)
    p = torch.empty(inst.N, dtype=torch.float64, device="cuda")
    s.solve(sweeps=2, out=p)
    torch.cuda.synchronize()
    e = p_err(p.cpu().numpy(), p_ref, inst.d)
    log(f"cam after autotune: {e:.2e}")
    assert e <= 1e-10
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up off the default stream before capture
        s.factor(A, Bv, cam, b, d, inst.lam)
        s.solve(sweeps=1, out=p)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = p.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.factor(A, Bv, cam, b, d, inst.lam)
        s.solve(sweeps=1, out=p)
    for r in range(3):
        p.fill_(float("nan"))
        x = torch.ones(1 << 20, device="cuda").cumsum(0)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(p, eager), f"replay {r}"
        assert float(x[-1]) == float(1 << 20)
    assert s.status()[0] == 0
