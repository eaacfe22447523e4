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
