"""GPU parity of the batched block-angular path (many independent problems in the same
launches) against the CPU oracle, problem by problem, and against the single-problem path."""
import numpy as np
import pytest

from oracle import refine
from tests.gpu_util import gpu_solve_blockangular, log, rel_err
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _batch_problems(dtype, seed=0):
    """Problems of every dense-part class the batch path groups by (nB 0 .. 127), ragged
    blocks, per-problem damping (one lambda = 0 problem with full-rank blocks)."""
    rng = np.random.default_rng(seed)
    shapes = [  # (K, m range, nB, lam)
        (40, (4, 12), 0, 1e-2),
        (120, (4, 20), 6, 1e-2),
        (300, (8, 16), 30, 1e-1),
        (60, (4, 40), 45, 0.0),
        (500, (4, 12), 90, 1e-2),
        (25, (3, 9), 17, 1.0),
        (200, (4, 30), 127, 1e-2),
        (80, (4, 40), 90, 1e-3),
    ]
    out = []
    for k, (K, (lo, hi), nB, lam) in enumerate(shapes):
        if lam == 0.0:
            lo = max(lo, 4)  # m_i > n keeps the blocks full rank without damping
        m = rng.integers(lo, hi + 1, size=K)
        out.append(gen.make_blockangular(1000 + 17 * k + seed, K=K, m=m, n=3, nB=nB, lam=lam, dtype=dtype))
    return out


def _to_dev(st):
    import torch
    return {k: (torch.from_numpy(np.ascontiguousarray(v)).cuda() if isinstance(v, np.ndarray) and k not in
                ("K", "nB", "row_off") else v) for k, v in st.items()}


def _run_batch(insts, sweeps=0, autotune=False):
    import torch
    from paper_1802_03773_amd import BlockAngularBatch
    st = gen.stack_batch(insts)
    dev = _to_dev(st)
    bt = BlockAngularBatch(st["K"], st["nB"], st["row_off"], st["n"], dtype=str(insts[0].dtype))
    bt.factor(dev["A"], dev["B"] if dev["B"].numel() else None, dev["b"], dev["d"], dev["lam"])
    scale = bt.autotune() if autotune else None
    p = bt.solve(sweeps=sweeps)
    torch.cuda.synchronize()
    bits = bt.status_problems()
    split = np.cumsum([i.N for i in insts])[:-1]
    return np.split(p.cpu().numpy(), split), bits, scale


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batch_matches_oracle_per_problem(dtype):
    insts = _batch_problems(dtype)
    log(f"batch of {len(insts)} problems, {np.dtype(dtype).name}")
    p0, bits, _ = _run_batch(insts, sweeps=0)
    p2, _, _ = _run_batch(insts, sweeps=2)
    assert np.all(bits == 0), bits
    tol = 1e-5 if dtype == np.float32 else 1e-11
    for q, inst in enumerate(insts):
        p_ref, _ = refine.reference_solution(inst)
        log(f"  problem {q}: K={inst.K} nB={inst.nB} lam={inst.lam}")
        assert rel_err(p0[q], p_ref) <= tol, q
        assert rel_err(p2[q], p_ref) <= 1e-10, q


def test_batch_agrees_with_single_problem_path():
    insts = _batch_problems(np.float32, seed=1)
    pb, _, _ = _run_batch(insts, sweeps=1)
    for q, inst in enumerate(insts):
        ps, st = gpu_solve_blockangular(inst, sweeps=1)
        assert st[0] == 0
        assert rel_err(pb[q], ps) <= 1e-12, q


def test_batch_status_is_per_problem():
    """lam = 0 and a block of 2 rows < 3 columns makes problem 2 singular; the others are fine."""
    insts = _batch_problems(np.float64, seed=2)[:4]
    bad = insts[2]
    m = np.diff(bad.row_off)
    m[5] = 2
    insts[2] = gen.make_blockangular(77, K=bad.K, m=m, n=3, nB=bad.nB, lam=0.0, dtype=np.float64)
    _, bits, _ = _run_batch(insts)
    assert bits[2] & 1, bits
    assert bits[0] == 0 and bits[1] == 0 and bits[3] == 0, bits


def test_batch_autotune_keeps_results():
    insts = _batch_problems(np.float32, seed=3)
    p, bits, scale = _run_batch(insts, sweeps=2, autotune=True)
    log(f"autotune scale {scale}")
    assert scale in (0.5, 1.0, 2.0, 4.0)
    assert np.all(bits == 0)
    for q, inst in enumerate(insts):
        p_ref, _ = refine.reference_solution(inst)
        assert rel_err(p[q], p_ref) <= 1e-10, q


def test_ragged_batch_sampled():
    """32 problems of the ragged-batch recipe (K ~ U{500..8000}, m_i ~ U{4,6,..,40},
    nB ~ U{6,30,90}); problems 0, 13 and 31 checked against the oracle."""
    log("ragged batch: generating")
    insts = gen.ragged_batch(200, P=32)
    log(f"ragged batch: {sum(i.K for i in insts)} blocks, {sum(i.M for i in insts)} rows")
    p0, bits, _ = _run_batch(insts, sweeps=0)
    p1, _, _ = _run_batch(insts, sweeps=1)
    assert np.all(bits == 0)
    for q in (0, 13, 31):
        log(f"ragged batch: oracle problem {q}")
        p_ref, _ = refine.reference_solution(insts[q])
        assert rel_err(p0[q], p_ref) <= 1e-5
        assert rel_err(p1[q], p_ref) <= 1e-10
