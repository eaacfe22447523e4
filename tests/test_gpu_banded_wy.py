"""GPU parity of the block-banded compact-WY factorisation (Section 4.4, qrk_set_banded_method)
against the oracle: the band of R and c up to row signs against the oracle's factor, p
unrefined and after float64-residual sweeps, batches, row patterns and window edge cases, the
2,048-problem workload sampled, agreement with the Givens kernels, the LM driver, and the
argument errors of the method switch."""
import numpy as np
import pytest

from oracle import banded, block_banded
from tests.gpu_util import log, p_err, sign_fix_rows
from workloads import generators as gen

pytestmark = pytest.mark.gpu

METHODS = ["blockwy", "blockwy-bf16x3"]
UNREF = {"blockwy": 1e-5, "blockwy-bf16x3": 5e-4}
FTOL = {"blockwy": 5e-5, "blockwy-bf16x3": 2e-3}


def _dev(insts):
    import torch
    rs = torch.from_numpy(np.stack([i.row_start for i in insts])).cuda().contiguous()
    vals = torch.from_numpy(np.stack([i.vals for i in insts])).cuda().contiguous()
    b = torch.from_numpy(np.stack([i.b for i in insts])).cuda().contiguous()
    d = torch.from_numpy(np.stack([i.d for i in insts])).cuda().contiguous()
    return rs, vals, b, d


def _solve(insts, method, sweeps=0):
    import torch
    from paper_1802_03773_amd import BandedSolver
    i0 = insts[0]
    s = BandedSolver(i0.M, i0.N, i0.w, dtype=str(i0.dtype), P=len(insts)).set_method(method)
    rs, vals, b, d = _dev(insts)
    s.factor(rs, vals, b, d, i0.lam)
    p = s.solve(sweeps=sweeps)
    torch.cuda.synchronize()
    return p.cpu().numpy().reshape(len(insts), i0.N), s.status(), s


def _check_factor(inst, solver, k, tol):
    Rb, c = [t.cpu().numpy().astype(np.float64) for t in solver.get_factor()]
    N, w = inst.N, inst.w
    Rb, c = Rb[k * N:(k + 1) * N], c[k * N:(k + 1) * N]
    R = np.zeros((N, N))
    for j in range(N):
        m = min(w, N - j)
        R[j, j:j + m] = Rb[j, :m]
    f = block_banded.factor(inst)
    Rg, cg = sign_fix_rows(R, c)
    Ro, co = sign_fix_rows(np.triu(f["R"]) * (np.triu(np.ones((N, N)), 0) - np.triu(np.ones((N, N)), w)), f["c"])
    scale = np.abs(Ro).max()
    assert np.abs(Rg - Ro).max() <= tol * scale
    assert np.abs(cg - co).max() <= tol * max(np.abs(co).max(), scale)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("w", [1, 2, 5, 12, 15])
def test_blockwy_small(w, method):
    log(f"blockwy N=60 w={w} {method}")
    inst = gen.make_banded(5700 + w, N=60, w=w, lam=1e-2, dtype=np.float32)
    p_ref, _, _ = banded.reference_solution(inst)
    p, st, solver = _solve([inst], method)
    assert st[0] == 0, st
    e = p_err(p[0], p_ref, inst.d)
    log(f"  unrefined {e:.2e}")
    assert e <= UNREF[method]
    _check_factor(inst, solver, 0, FTOL[method])
    p2, st, _ = _solve([inst], method, sweeps=2)
    assert p_err(p2[0], p_ref, inst.d) <= 1e-10


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("rows_per_col,w,N", [(1, 5, 90), (3, 12, 90), (1, 15, 64), (3, 13, 33), (2, 12, 256)])
def test_blockwy_patterns_batch(rows_per_col, w, N, method):
    """Row counts per column block of 16, 48 and 24-32 (several merges per block), batches of
    four problems, N a multiple of 16 or not."""
    log(f"blockwy patterns rows_per_col={rows_per_col} w={w} N={N} {method}")
    insts = [gen.make_banded(5800 + 10 * k + w + N, N=N, w=w, rows_per_col=rows_per_col, lam=1e-2,
                             dtype=np.float32) for k in range(4)]
    p0, st, solver = _solve(insts, method)
    assert st[0] == 0
    p2, _, _ = _solve(insts, method, sweeps=2)
    for k, inst in enumerate(insts):
        p_ref, _, _ = banded.reference_solution(inst)
        assert p_err(p0[k], p_ref, inst.d) <= UNREF[method]
        assert p_err(p2[k], p_ref, inst.d) <= 1e-10
    _check_factor(insts[3], solver, 3, FTOL[method])


def _custom(seed, N, w, rs, lam):
    rng = np.random.default_rng(seed)
    rs = np.asarray(rs, np.int32)
    vals = rng.standard_normal((rs.shape[0], w)).astype(np.float32)
    b = rng.standard_normal(rs.shape[0]).astype(np.float32)
    d = gen.column_norms_banded(N, w, rs, vals) if rs.shape[0] else np.ones(N)
    d = np.where(d > 0, d, 1.0)
    return gen.Banded(N, w, rs, vals, b, d, float(lam), np.dtype(np.float32))


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("case", ["N_eq_w", "tiny_N", "few_rows", "jumps", "one_start", "lam0"])
def test_blockwy_edge_shapes(case, method):
    """A single window (N = w), N below one column block, fewer rows than columns, starts that
    skip whole blocks, every row at one start, and lambda = 0 with full column rank."""
    w = 12 if case not in ("tiny_N",) else 5
    lam = 1e-2
    if case == "N_eq_w":
        N, rs = 12, [0] * 30
    elif case == "tiny_N":
        N, rs = 9, [min(i // 2, 4) for i in range(14)]
    elif case == "few_rows":
        N, rs = 80, [0, 3, 3, 20, 41, 68]
    elif case == "jumps":
        N, rs = 200, sorted([0, 0, 1, 30, 30, 31, 100, 100, 150, 170, 188, 188])
    elif case == "one_start":
        N, rs = 40, [10] * 25
    else:
        N, rs, lam = 50, [min(i // 3, 38) for i in range(150)], 0.0
    log(f"blockwy edge {case} {method}")
    insts = [_custom(5900 + k, N, w, rs, lam) for k in range(3)]
    p0, st, solver = _solve(insts, method)
    assert st[0] == 0
    p2, _, _ = _solve(insts, method, sweeps=2)
    for k, inst in enumerate(insts):
        p_ref, _, _ = banded.reference_solution(inst)
        # these J have fewer rows than columns or empty columns: cond([J; sqrt(lam) D]) reaches
        # 1e4, where the unrefined bound (stated at cond <= 1e3) scales with the condition number
        Aaug = np.vstack([banded.assemble(inst), np.sqrt(inst.lam) * np.diag(inst.d)])
        cond = np.linalg.cond(Aaug)
        e0 = p_err(p0[k], p_ref, inst.d)
        log(f"  problem {k}: cond {cond:.3g}, unrefined {e0:.2e}")
        assert e0 <= UNREF[method] * max(1.0, cond / 1e3)
        assert p_err(p2[k], p_ref, inst.d) <= 1e-10
    _check_factor(insts[1], solver, 1, FTOL[method])


def test_blockwy_agrees_with_givens():
    """The same R (up to row signs) and p as the Givens kernels on 64 problems."""
    import torch
    insts = [gen.make_banded(6000 + k, N=300, w=12, lam=1e-2, dtype=np.float32) for k in range(64)]
    pg, _, sg = _solve(insts, "givens")
    pw, _, sw = _solve(insts, "blockwy")
    assert np.max(np.abs(pg - pw)) <= 1e-5 * np.max(np.abs(pg))
    Rg, cg = [t.cpu().numpy().astype(np.float64) for t in sg.get_factor()]
    Rw, cw = [t.cpu().numpy().astype(np.float64) for t in sw.get_factor()]
    sgn = np.sign(Rg[:, 0]) * np.sign(Rw[:, 0])
    assert np.abs(Rg - Rw * sgn[:, None]).max() <= 5e-5 * np.abs(Rg).max()
    assert np.abs(cg - cw * sgn).max() <= 5e-5 * max(np.abs(cg).max(), np.abs(Rg).max())
    torch.cuda.synchronize()


@pytest.mark.parametrize("method", METHODS)
def test_blockwy_full_size_sampled(method):
    """2,048 problems of n = 2,048 (4,096 rows, 12 values per row): sampled problems vs oracle."""
    log(f"blockwy full size {method}: generating")
    insts = gen.banded_batch(300, P=2048)
    p0, st, solver = _solve(insts, method)
    assert st[0] == 0
    p1 = solver.solve(sweeps=1).cpu().numpy().reshape(2048, -1)
    for k in (0, 1023, 2047):
        log(f"blockwy full size: oracle problem {k}")
        p_ref, _, _ = banded.reference_solution(insts[k])
        e0, e1 = p_err(p0[k], p_ref, insts[k].d), p_err(p1[k], p_ref, insts[k].d)
        log(f"  errors {e0:.2e} / {e1:.2e}")
        assert e0 <= UNREF[method]
        assert e1 <= 1e-10


def test_blockwy_bad_row_start_is_reported():
    inst = gen.make_banded(5, N=40, w=4, dtype=np.float32)
    inst.row_start[10] = inst.row_start[9] - 3  # decreasing
    _, st, _ = _solve([inst], "blockwy")
    assert st[0] == 1  # QRK_EINVAL


def test_blockwy_lm_driver_matches_oracle():
    """The banded LM driver with the block-banded factor: float32 iterations against the
    Backtrack-LM oracle (accept decisions identical, costs to 1e-5)."""
    import torch
    from oracle import lm as olm
    from paper_1802_03773_amd import BandedSolver, LMDriver
    probs = [gen.lm_banded(6100 + k, N=200, w=12, c=0.1, dtype=np.float32)[:3] for k in range(3)]
    i0 = probs[0][0]
    s = BandedSolver(i0.M, i0.N, i0.w, dtype="float32", P=3).set_method("blockwy")
    rs = torch.from_numpy(np.concatenate([p[0].row_start for p in probs])).cuda()
    vals0 = torch.from_numpy(np.concatenate([p[0].vals for p in probs])).cuda()
    y = torch.from_numpy(np.concatenate([p[1] for p in probs])).cuda()
    drv = LMDriver(s, rs, vals0, y, 0.1, sweeps=2, max_log=16)
    x0 = torch.from_numpy(np.concatenate([p[2] for p in probs])).cuda()
    drv.reset(x0, torch.full((3,), 1e-2, dtype=torch.float64, device="cuda"))
    drv.run(6, graph=True)
    x, _, lg, done = drv.get()
    assert done == 6
    lg = lg.cpu().numpy()
    for q, (inst0, yq, x0q) in enumerate(probs):
        model = olm.BandedModel(inst0, yq.astype(np.float64), 0.1)
        _, _, lgo = olm.bd_lm(model, x0q, 1e-2, 6, store=np.float32)
        real = (lgo[:, 0] - lgo[:, 1]) > 1e-7 * lgo[:, 0]
        k = int(np.argmin(real)) if not real.all() else len(real)
        assert k >= 2
        np.testing.assert_allclose(lg[:k, q, :3], lgo[:k, :3], rtol=1e-5)
        assert np.array_equal(lg[:k, q, 3], lgo[:k, 3])


def test_blockwy_method_errors():
    from paper_1802_03773_amd import BandedSolver, QRKError
    with pytest.raises(QRKError):
        BandedSolver(40, 20, 4, dtype="float64").set_method("blockwy")
    with pytest.raises(QRKError):
        BandedSolver(40, 20, 16, dtype="float32").set_method("blockwy")
    BandedSolver(40, 20, 15, dtype="float32").set_method("blockwy-bf16x3").set_method("givens")
