"""GPU parity of the batched block-angular path (many independent problems in the same
launches) against the CPU oracle, problem by problem, and against the single-problem path."""
import numpy as np
import pytest

from oracle import refine
from tests.gpu_util import gpu_solve_blockangular, log, p_err, rel_err, to_device
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
        assert p_err(p0[q], p_ref, inst.d) <= tol, q
        assert p_err(p2[q], p_ref, inst.d) <= 1e-10, q


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
        assert p_err(p[q], p_ref, inst.d) <= 1e-10, q


def test_autotune_cache_file_round_trip(tmp_path):
    """The autotuner's choice is written to the cache file under the batch's shape key, and a new
    handle of the same shape starts from it (in a process that reads the file afresh the key
    and the file are the same; here the file is re-read into the process map).  The file also
    holds whatever the process tuned before (the process map is written out whole), so the
    batch's entry is looked up by its key."""
    import json
    import torch
    from paper_1802_03773_amd import BlockAngularBatch, qrkit
    path = tmp_path / "tune.json"
    qrkit.set_tune_cache(path)
    try:
        insts = _batch_problems(np.float32, seed=4)
        st = gen.stack_batch(insts)
        dev = _to_dev(st)
        bt = BlockAngularBatch(st["K"], st["nB"], st["row_off"], st["n"], dtype="float32")
        bt.factor(dev["A"], dev["B"], dev["b"], dev["d"], dev["lam"])
        scale = bt.autotune()
        chosen = qrkit.tune_choice(bt)
        log(f"autotune choice {chosen}")
        assert chosen["leaf_scale"] == scale
        data = json.loads(path.read_text())
        entries = data["entries"]
        mine = [k for k in entries if k.startswith("gfx950/f32/plain/P8/n3/")]
        assert len(mine) == 1, entries
        rec = entries[mine[0]]
        assert rec["leaf_scale"] == chosen["leaf_scale"] and rec["refine_scale"] == chosen["refine_scale"]
        assert rec["leaf_queue"] == chosen["leaf_queue"]
        qrkit.set_tune_cache(path)  # reload
        bt2 = BlockAngularBatch(st["K"], st["nB"], st["row_off"], st["n"], dtype="float32")
        assert qrkit.tune_choice(bt2) == chosen
        bt2.factor(dev["A"], dev["B"], dev["b"], dev["d"], dev["lam"])
        p = np.split(bt2.solve(sweeps=2).cpu().numpy(), np.cumsum([i.N for i in insts])[:-1])
        torch.cuda.synchronize()
        for q in (0, 4, 7):
            p_ref, _ = refine.reference_solution(insts[q])
            assert p_err(p[q], p_ref, insts[q].d) <= 1e-10, q
    finally:
        qrkit.set_tune_cache(None)


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
        assert p_err(p0[q], p_ref, insts[q].d) <= 1e-5
        assert p_err(p1[q], p_ref, insts[q].d) <= 1e-10


def test_ragged_batch_full_512():
    """The full ragged recipe: 512 problems (K_p ~ U{500..8000}, m_i ~ U{4,6,..,40}, n = 3,
    nB ~ U{6,30,90}, about 2.2M blocks and 48M rows) in the launch configuration the benchmark
    times; problems 0, 255 and 511 against the oracle (unrefined and one sweep), every status
    word clear."""
    log("ragged 512: generating")
    insts = gen.ragged_batch(200, P=512)
    log(f"ragged 512: {sum(i.K for i in insts)} blocks, {sum(i.M for i in insts)} rows")
    p0, bits, _ = _run_batch(insts, sweeps=0)
    p1, _, _ = _run_batch(insts, sweeps=1)
    assert np.all(bits == 0)
    for q in (0, 255, 511):
        log(f"ragged 512: oracle problem {q} (K={insts[q].K}, nB={insts[q].nB})")
        p_ref, _ = refine.reference_solution(insts[q])
        e0, e1 = p_err(p0[q], p_ref, insts[q].d), p_err(p1[q], p_ref, insts[q].d)
        log(f"  errors {e0:.2e} / {e1:.2e}")
        assert e0 <= 1e-5
        assert e1 <= 1e-10


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_colnorms_blockangular(dtype):
    """qrk_colnorms_blockangular: d_j = ||J e_j||_2 in float64 of the stored values (the
    generator's column norms), and an all-zero column (a zeroed block column and a zeroed dense
    column) maps to 1."""
    import torch
    from paper_1802_03773_amd import BlockAngularSolver
    m = np.where(np.arange(300) % 3 == 0, 0, 4 + np.arange(300) % 9)  # empty blocks included
    inst = gen.make_blockangular(91, K=300, m=m, n=3, nB=37, lam=1e-2, dtype=dtype)
    inst.A[inst.row_off[4]:inst.row_off[5], 1] = 0.0
    inst.B[:, 11] = 0.0
    d_ref = gen.column_norms_blockangular(inst.row_off, inst.n, inst.A, inst.B)
    J = np.zeros((inst.M, inst.N))
    for i in range(inst.K):
        J[inst.row_off[i]:inst.row_off[i + 1], 3 * i:3 * i + 3] = inst.A[inst.row_off[i]:inst.row_off[i + 1]]
    J[:, 3 * inst.K:] = inst.B
    d_dense = np.sqrt((J * J).sum(axis=0))
    d_dense[d_dense == 0.0] = 1.0
    assert np.abs(d_ref - d_dense).max() <= 1e-14 * d_dense.max()
    A, B, _, _ = to_device(inst)
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype=str(inst.dtype))
    d = s.colnorms(A, B).cpu().numpy()
    assert d[3 * 4 + 1] == 1.0 and d[3 * inst.K + 11] == 1.0 and d[0] == 1.0
    assert np.abs(d - d_dense).max() <= 1e-13 * d_dense.max()
