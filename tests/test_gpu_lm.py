"""GPU Levenberg-Marquardt driver (model evaluation, structured factor + solve, gain ratio and
damping update on the device; optionally one iteration captured as a HIP graph and
replayed) against the Backtrack-LM oracle, and graph replays against eager iterations."""
import numpy as np
import pytest

from oracle import lm as olm
from tests.gpu_util import log, rel_err
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _setup(problems, dtype, c, sweeps=2, max_log=32, mode="plain"):
    """problems: list of (inst0, y, x0); returns (driver, batch-or-solver, device arrays)."""
    import torch
    from paper_1802_03773_amd import BlockAngularBatch, LMDriver
    insts = [p[0] for p in problems]
    st = gen.stack_batch(insts)
    td = torch.float32 if dtype == np.float32 else torch.float64
    bt = BlockAngularBatch(st["K"], st["nB"], st["row_off"], st["n"], dtype=np.dtype(dtype).name, mode=mode)
    A0 = torch.from_numpy(st["A"]).cuda()
    B0 = torch.from_numpy(st["B"]).cuda() if st["B"].size else None
    y = torch.from_numpy(np.concatenate([p[1] for p in problems]).astype(dtype)).cuda()
    assert A0.dtype == td
    drv = LMDriver(bt, A0, B0, y, c, sweeps=sweeps, max_log=max_log)
    x0 = torch.from_numpy(np.concatenate([p[2] for p in problems])).cuda()
    return drv, bt, x0, (A0, B0, y)


def _oracle_run(problem, c, lam0, iters, store):
    inst0, y, x0 = problem
    model = olm.BlockAngularModel(inst0, y.astype(np.float64), c)
    return olm.ba_lm(model, x0, lam0, iters, store=store)


def _significant(logq):
    """Iterations before the cost decrease falls to roundoff."""
    real = (logq[:, 0] - logq[:, 1]) > 1e-7 * logq[:, 0]
    return int(np.argmin(real)) if not real.all() else len(real)


def test_lm_float64_single_problem_matches_oracle():
    import torch
    inst0, y, x0, _ = gen.lm_blockangular(401, K=40, m=8, n=3, nB=10, c=0.1, dtype=np.float64)
    drv, bt, x0d, _ = _setup([(inst0, y, x0)], np.float64, 0.1)
    iters = 12
    drv.reset(x0d, torch.tensor([1e-2], dtype=torch.float64, device="cuda"))
    drv.run(iters)
    x, lam, lg, done = drv.get()
    assert done == iters
    xo, lamo, lgo = _oracle_run((inst0, y, x0), 0.1, 1e-2, iters, np.float64)
    lg = lg.cpu().numpy()[:, 0, :]
    k = _significant(lgo)
    log(f"float64 LM: {k} significant iterations, final F {lg[iters - 1, 0]:.6e} vs {lgo[-1, 0]:.6e}")
    assert k >= 3
    np.testing.assert_allclose(lg[:k, :3], lgo[:k, :3], rtol=1e-9)
    assert np.array_equal(lg[:k, 3], lgo[:k, 3])
    assert rel_err(x.cpu().numpy(), xo) <= 1e-9


@pytest.mark.parametrize("mode", ["plain", "bf16x3"])
def test_lm_float32_batch_matches_oracle(mode):
    import torch
    probs = []
    for k, (K, nB) in enumerate([(60, 30), (25, 6), (40, 0)]):
        inst0, y, x0, _ = gen.lm_blockangular(410 + k, K=K, m=10, n=3, nB=nB, c=0.1, dtype=np.float32)
        probs.append((inst0, y, x0))
    drv, bt, x0d, _ = _setup(probs, np.float32, 0.1, mode=mode)
    iters = 10
    lam0 = np.array([1e-2, 1e-1, 1.0])
    drv.reset(x0d, torch.from_numpy(lam0).cuda())
    drv.run(iters)
    x, lam, lg, done = drv.get()
    assert done == iters
    lg = lg.cpu().numpy()
    xs = np.split(x.cpu().numpy(), np.cumsum([p[0].N for p in probs])[:-1])
    for q, prob in enumerate(probs):
        xo, _, lgo = _oracle_run(prob, 0.1, lam0[q], iters, np.float32)
        k = _significant(lgo)
        log(f"float32 LM ({mode}) problem {q}: {k} significant iterations")
        assert k >= 2
        np.testing.assert_allclose(lg[:k, q, :3], lgo[:k, :3], rtol=1e-5)
        assert np.array_equal(lg[:k, q, 3], lgo[:k, 3])
        assert rel_err(xs[q], xo) <= 1e-6


def test_lm_graph_replays_match_eager():
    """Eight iterations eagerly, then the same eight as replays of one captured iteration with
    eager work and synchronisation between replays: identical logs and iterates."""
    import torch
    probs = [gen.lm_blockangular(420 + k, K=50, m=10, n=3, nB=nB, c=0.1, dtype=np.float32)[:3]
             for k, nB in enumerate([20, 90])]
    drv, bt, x0d, _ = _setup(probs, np.float32, 0.1)
    lam0 = torch.tensor([1e-2, 1e-2], dtype=torch.float64, device="cuda")
    iters = 8
    drv.reset(x0d, lam0)
    drv.run(iters, graph=False)
    x_e, lam_e, lg_e, _ = drv.get()
    x_e, lam_e, lg_e = x_e.cpu().numpy(), lam_e.cpu().numpy(), lg_e.cpu().numpy()
    drv.reset(x0d, lam0)
    scratch = torch.zeros(1 << 16, device="cuda")
    for k in range(iters):
        drv.run(1, graph=True)
        scratch.add_(1.0)  # eager work between replays
        torch.cuda.synchronize()
        _, _, _, done = drv.get()
        assert done == k + 1
    x_g, lam_g, lg_g, _ = drv.get()
    assert np.array_equal(x_g.cpu().numpy(), x_e)
    assert np.array_equal(lam_g.cpu().numpy(), lam_e)
    assert np.array_equal(lg_g.cpu().numpy(), lg_e)
    assert np.all(lg_e[:iters, :, 3] >= 0)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_lm_cost_at_unchanged_point_is_bit_identical(dtype):
    """With a damping so large that x + p == x in float64, F_new is the cost at the same point
    as F: the two passes (with and without the Jacobian) sum f^2 in the same order, so the
    values agree bit for bit and the gain ratio's numerator is exactly zero."""
    import torch
    probs = [gen.lm_blockangular(440 + k, K=K, m=10, n=3, nB=nB, c=0.1, dtype=dtype)[:3]
             for k, (K, nB) in enumerate([(300, 40), (70, 90)])]
    drv, bt, x0d, _ = _setup(probs, dtype, 0.1, sweeps=1)
    drv.reset(x0d, torch.tensor([1e30, 1e30], dtype=torch.float64, device="cuda"))
    drv.run(1)
    x, _, lg, done = drv.get()
    lg = lg.cpu().numpy()
    assert done == 1
    assert np.array_equal(x.cpu().numpy(), x0d.cpu().numpy())  # rejected: x unchanged
    for q in range(2):
        log(f"problem {q}: F = {lg[0, q, 0]!r}, F_new = {lg[0, q, 1]!r}")
        assert lg[0, q, 0] == lg[0, q, 1]
        assert lg[0, q, 3] == 0.0


def test_lm_graph_recaptured_after_leaf_shape_change():
    """A graph captured with one dense-part leaf layout, then qrk_set_tsqr_shape moves to another
    (new leaf tables, possibly new merge-tree workspace): the next graph run captures again, and
    its iterations match eager iterations under the new layout bit for bit."""
    import torch
    from paper_1802_03773_amd import BlockAngularSolver, LMDriver
    inst0, y, x0, _ = gen.lm_blockangular(430, K=120, m=10, n=3, nB=40, c=0.1, dtype=np.float32)
    A0 = torch.from_numpy(inst0.A).cuda()
    B0 = torch.from_numpy(inst0.B).cuda()
    yd = torch.from_numpy(y).cuda()
    x0d = torch.from_numpy(x0).cuda()
    lam0 = torch.tensor([1e-2], dtype=torch.float64, device="cuda")
    s = BlockAngularSolver(inst0.row_off, inst0.n, inst0.nB, dtype="float32")
    s.set_tsqr_shape(2)
    drv = LMDriver(s, A0, B0, yd, 0.1, sweeps=1, max_log=8)
    drv.reset(x0d, lam0)
    drv.run(3, graph=True)  # captured with two leaves
    torch.cuda.synchronize()
    s.set_tsqr_shape(9)  # more leaves: more slots, counters and tree nodes
    drv.reset(x0d, lam0)
    drv.run(4, graph=True)
    x_g, lam_g, lg_g, done = drv.get()
    assert done == 4
    drv.reset(x0d, lam0)
    drv.run(4, graph=False)
    x_e, lam_e, lg_e, _ = drv.get()
    assert np.array_equal(x_g.cpu().numpy(), x_e.cpu().numpy())
    assert np.array_equal(lg_g.cpu().numpy(), lg_e.cpu().numpy())
    xo, _, lgo = _oracle_run((inst0, y, x0), 0.1, 1e-2, 4, np.float32)
    k = _significant(lgo)
    np.testing.assert_allclose(lg_g.cpu().numpy()[:k, 0, :3], lgo[:k, :3], rtol=1e-5)


def _setup_banded(problems, dtype, c, sweeps=2, max_log=32):
    import torch
    from paper_1802_03773_amd import BandedSolver, LMDriver
    i0 = problems[0][0]
    s = BandedSolver(i0.M, i0.N, i0.w, dtype=np.dtype(dtype).name, P=len(problems))
    rs = torch.from_numpy(np.concatenate([p[0].row_start for p in problems]).astype(np.int32)).cuda()
    vals0 = torch.from_numpy(np.concatenate([p[0].vals for p in problems]).astype(dtype)).cuda()
    y = torch.from_numpy(np.concatenate([p[1] for p in problems]).astype(dtype)).cuda()
    drv = LMDriver(s, rs, vals0, y, c, sweeps=sweeps, max_log=max_log)
    x0 = torch.from_numpy(np.concatenate([p[2] for p in problems])).cuda()
    return drv, s, x0, (rs, vals0, y)


def _oracle_banded(problem, c, lam0, iters, store):
    inst0, y, x0 = problem
    model = olm.BandedModel(inst0, y.astype(np.float64), c)
    return olm.bd_lm(model, x0, lam0, iters, store=store)


def test_lm_banded_float64_matches_oracle():
    import torch
    inst0, y, x0, _ = gen.lm_banded(430, N=200, w=6, c=0.1, dtype=np.float64)
    drv, _, x0d, _ = _setup_banded([(inst0, y, x0)], np.float64, 0.1)
    iters = 12
    drv.reset(x0d, torch.tensor([1e-2], dtype=torch.float64, device="cuda"))
    drv.run(iters)
    x, lam, lg, done = drv.get()
    assert done == iters
    xo, _, lgo = _oracle_banded((inst0, y, x0), 0.1, 1e-2, iters, np.float64)
    lg = lg.cpu().numpy()[:, 0, :]
    k = _significant(lgo)
    log(f"banded float64 LM: {k} significant iterations")
    assert k >= 3
    np.testing.assert_allclose(lg[:k, :3], lgo[:k, :3], rtol=1e-9)
    assert np.array_equal(lg[:k, 3], lgo[:k, 3])
    assert rel_err(x.cpu().numpy(), xo) <= 1e-9


def test_lm_banded_float32_batch_oracle_and_graph():
    """Four banded problems (n = 256, w = 12): per-problem agreement with the oracle, then the
    same iterations as graph replays, identical to the eager run."""
    import torch
    probs = [gen.lm_banded(440 + k, N=256, w=12, c=0.1, dtype=np.float32)[:3] for k in range(4)]
    drv, _, x0d, _ = _setup_banded(probs, np.float32, 0.1)
    iters = 8
    lam0 = torch.tensor([1e-2, 1e-1, 1.0, 1e-3], dtype=torch.float64, device="cuda")
    drv.reset(x0d, lam0)
    drv.run(iters)
    x_e, lam_e, lg_e, done = drv.get()
    assert done == iters
    x_e, lam_e, lg_e = x_e.cpu().numpy(), lam_e.cpu().numpy(), lg_e.cpu().numpy()
    xs = np.split(x_e, len(probs))
    for q, prob in enumerate(probs):
        xo, _, lgo = _oracle_banded(prob, 0.1, float(lam0[q]), iters, np.float32)
        k = _significant(lgo)
        log(f"banded float32 LM problem {q}: {k} significant iterations")
        assert k >= 2
        np.testing.assert_allclose(lg_e[:k, q, :3], lgo[:k, :3], rtol=1e-5)
        assert np.array_equal(lg_e[:k, q, 3], lgo[:k, 3])
        assert rel_err(xs[q], xo) <= 1e-6
    drv.reset(x0d, lam0)
    for k in range(iters):
        drv.run(1, graph=True)
        torch.cuda.synchronize()
    x_g, lam_g, lg_g, done = drv.get()
    assert done == iters
    assert np.array_equal(x_g.cpu().numpy(), x_e)
    assert np.array_equal(lam_g.cpu().numpy(), lam_e)
    assert np.array_equal(lg_g.cpu().numpy(), lg_e)
