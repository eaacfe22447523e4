"""GPU parity of the block-angular LM step (HIP path through the C ABI) against the
CPU oracle: the solution p, and the stored factor (R_i, S_i | c_i, R_B | c_B) up to row
signs.  Tolerances: float64 path 1e-12 vs the longdouble-refined reference; float32
unrefined 1e-5 at cond(J) <= 1e3; any path after refinement sweeps 1e-10."""
import numpy as np
import pytest

from oracle import refine, structured
from tests.gpu_util import p_err, gpu_solve_blockangular, log, rel_err, sign_fix_rows
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _check_factor(inst, solver, f, tol):
    Rblk, S, RB = [t.cpu().numpy().astype(np.float64) for t in solver.get_factor()]
    K, n, nB = inst.K, inst.n, inst.nB
    # per-block R_i and coupling rows S_i | c_i, up to the sign of each row
    for i in range(0, K, max(1, K // 64)):
        Rg, Sg = sign_fix_rows(Rblk[i], S[i])
        Ro, So = sign_fix_rows(f.R_blk[i], np.concatenate([f.S[i], f.c_blk[i][:, None]], axis=1))
        scale = max(np.abs(Ro).max(), 1e-300)
        assert np.abs(Rg - Ro).max() <= tol * scale, f"R_{i}"
        assert np.abs(Sg - So).max() <= tol * max(np.abs(So).max(), scale), f"S_{i}"
    if nB:
        Rg, cg = sign_fix_rows(RB[:nB, :nB], RB[:nB, nB])
        Ro, co = sign_fix_rows(f.R_B, f.c_B)
        assert np.abs(Rg - Ro).max() <= tol * np.abs(Ro).max()
        assert np.abs(cg - co).max() <= tol * max(np.abs(co).max(), np.abs(Ro).max())
    assert abs(abs(RB[nB, nB]) - f.resid) <= tol * max(1.0, f.resid) * 10


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_float64(seed):
    log(f"tiny float64 seed={seed}")
    inst = gen.tiny_blockangular(seed, dtype=np.float64)
    p_ref, f = refine.reference_solution(inst)
    p, st, solver, _ = gpu_solve_blockangular(inst, return_solver=True)
    assert st[0] == 0
    assert p_err(p, p_ref, inst.d) <= 1e-12
    _check_factor(inst, solver, f, 1e-12)


@pytest.mark.parametrize("seed", [0, 3])
def test_tiny_float32_unrefined_and_refined(seed):
    log(f"tiny float32 seed={seed}")
    inst = gen.tiny_blockangular(seed, dtype=np.float32)
    p_ref, f = refine.reference_solution(inst)
    p0, st, solver, _ = gpu_solve_blockangular(inst, return_solver=True)
    assert st[0] == 0
    assert p_err(p0, p_ref, inst.d) <= 1e-5
    _check_factor(inst, solver, f, 2e-5)
    p2, st = gpu_solve_blockangular(inst, sweeps=2)
    assert p_err(p2, p_ref, inst.d) <= 1e-10


SHAPES = [
    # (K, m (int or (lo, hi) ragged), n, nB, lam)
    (1, 30, 3, 6, 1e-2),
    (7, (0, 9), 2, 1, 1e-1),
    (33, (1, 12), 1, 0, 1e-2),
    (50, (3, 20), 3, 63, 1e-3),
    (61, (3, 20), 3, 64, 1e-2),
    (70, (0, 40), 4, 90, 1e-2),
    (45, (10, 56), 8, 127, 1.0),
    (200, 12, 3, 90, 1e-4),
]


def _ragged(seed, K, m):
    if isinstance(m, tuple):
        rng = np.random.default_rng(seed + 77)
        return rng.integers(m[0], m[1] + 1, size=K)
    return m


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape", SHAPES)
def test_shapes(shape, dtype):
    K, m, n, nB, lam = shape
    log(f"shape K={K} m={m} n={n} nB={nB} lam={lam} dtype={np.dtype(dtype).name}")
    inst = gen.make_blockangular(10 + K, K=K, m=_ragged(K, K, m), n=n, nB=nB, lam=lam, dtype=dtype)
    p_ref, f = refine.reference_solution(inst)
    p, st, solver, _ = gpu_solve_blockangular(inst, return_solver=True)
    assert st[0] == 0, st
    tol = 1e-11 if dtype == np.float64 else 1e-5
    assert p_err(p, p_ref, inst.d) <= tol
    _check_factor(inst, solver, f, 1e-11 if dtype == np.float64 else 5e-5)
    p2, st = gpu_solve_blockangular(inst, sweeps=2)
    assert p_err(p2, p_ref, inst.d) <= 1e-10


def test_tsqr_launch_shapes_agree():
    """Leaf counts and tree fan-ins change only the rounding of the result."""
    inst = gen.make_blockangular(5, K=400, m=12, n=3, nB=30, lam=1e-2, dtype=np.float64)
    p_ref, _ = refine.reference_solution(inst)
    for leaves, fanin in [(1, 2), (3, 2), (17, 4), (64, 8), (400, 16), (1024, 64)]:
        log(f"tsqr leaves={leaves} fanin={fanin}")
        p, st = gpu_solve_blockangular(inst, leaves=leaves, fanin=fanin)
        assert st[0] == 0
        assert p_err(p, p_ref, inst.d) <= 1e-12


@pytest.mark.parametrize("nB", [95, 100, 111, 112, 120, 127])
def test_wide_dense_part_multi_leaf_trees(nB):
    """7 and 8 column blocks of the dense part with forced multi-leaf reduction trees."""
    inst = gen.make_blockangular(40 + nB, K=60, m=(np.arange(60) % 9) + 8, n=3, nB=nB, lam=1e-2,
                                 dtype=np.float32)
    p_ref, _ = refine.reference_solution(inst)
    for leaves in [1, 2, 3, 5, 0]:
        log(f"nB={nB} leaves={leaves}")
        p, st = gpu_solve_blockangular(inst, leaves=leaves)
        assert st[0] == 0, st
        assert p_err(p, p_ref, inst.d) <= 1e-5


@pytest.mark.parametrize("mode", ["plain", "bf16x3"])
@pytest.mark.parametrize("nB", [5, 20, 40, 60, 75, 90])
def test_pipelined_tree_every_width(nB, mode):
    """Single float32 problems of 1..6 column blocks, whose leaf triangles are merged by the
    pipelined tree launch (each column block published above the diagonal first, then its
    diagonal block): even and odd leaf counts (a node without a sibling carries its triangle
    up a level), the factor R_B | c_B against the oracle up to row signs, and p."""
    K = 300
    inst = gen.make_blockangular(700 + nB, K=K, m=(np.arange(K) % 7) + 6, n=3, nB=nB, lam=1e-2,
                                 dtype=np.float32)
    p_ref, f = refine.reference_solution(inst)
    for leaves in [2, 3, 7, 16, 33]:
        log(f"pipelined tree nB={nB} mode={mode} leaves={leaves}")
        p, st, solver, _ = gpu_solve_blockangular(inst, mode=mode, leaves=leaves, return_solver=True)
        assert st[0] == 0, st
        assert p_err(p, p_ref, inst.d) <= 1e-5
        _check_factor(inst, solver, f, 5e-5)
        p2, st = gpu_solve_blockangular(inst, mode=mode, leaves=leaves, sweeps=2)
        assert p_err(p2, p_ref, inst.d) <= 1e-10


@pytest.mark.parametrize("lam", [1e-2, 0.0])
@pytest.mark.parametrize("nB", [47, 90, 127])
def test_few_rows_per_leaf(nB, lam):
    """Leaves of 33 and 12 rows: each leaf triangle starts from zero and has rank far below
    the column count, so the columns beyond that rank are reflected on roundoff that shrinks
    by about eps per leaf height and underflows to subnormal floats (lam = 0 starts leaf 0
    from zero as well)."""
    K = 40
    m = np.where(np.arange(K) % 2 == 0, 10, 56)
    inst = gen.make_blockangular(90 + nB, K=K, m=m, n=8, nB=nB, lam=lam, dtype=np.float32)
    p_ref, _ = refine.reference_solution(inst)
    for leaves in [1, 3, 40, 110, 0]:
        log(f"few rows per leaf nB={nB} lam={lam} leaves={leaves}")
        p, st = gpu_solve_blockangular(inst, leaves=leaves)
        assert st[0] == 0, st
        assert np.isfinite(p).all()
        e0 = p_err(p, p_ref, inst.d)
        log(f"  unrefined error {e0:.2e} (rel {rel_err(p, p_ref):.2e})")
        assert e0 <= 1e-5
        p1, st = gpu_solve_blockangular(inst, leaves=leaves, sweeps=2)
        assert p_err(p1, p_ref, inst.d) <= 1e-10


def test_lambda_zero_gauss_newton():
    inst = gen.make_blockangular(6, K=300, m=(np.arange(300) % 7) + 4, n=3, nB=20, lam=0.0,
                                 dtype=np.float64)
    log("lambda = 0")
    p_ref, _ = refine.reference_solution(inst)
    p, st = gpu_solve_blockangular(inst)
    assert st[0] == 0
    assert p_err(p, p_ref, inst.d) <= 1e-11


def test_singular_block_is_reported():
    """lam = 0 with a block of fewer rows than columns: R_i has a zero pivot."""
    log("singular status")
    m = np.full(20, 6)
    m[7] = 2
    inst = gen.make_blockangular(7, K=20, m=m, n=3, nB=4, lam=0.0, dtype=np.float64)
    _, st = gpu_solve_blockangular(inst)
    assert st[0] == 4  # QRK_ESINGULAR


def test_nonfinite_input_is_reported():
    log("non-finite status")
    inst = gen.make_blockangular(8, K=20, m=6, n=3, nB=4, lam=1e-2, dtype=np.float32)
    inst.B[13, 2] = np.nan
    _, st = gpu_solve_blockangular(inst)
    assert st[0] == 5  # QRK_ENONFINITE


def test_deterministic_repeat():
    log("determinism")
    inst = gen.make_blockangular(9, K=5000, m=12, n=3, nB=90, lam=1e-2, dtype=np.float32, scale_k=3.0)
    p1, _ = gpu_solve_blockangular(inst, sweeps=1)
    p2, _ = gpu_solve_blockangular(inst, sweeps=1)
    assert np.array_equal(p1, p2)


@pytest.mark.parametrize("lam", [1e-2, 0.0, 1e-4, 1.0])
def test_scale_workload_full_size(lam):
    """50,000 blocks of 12x3 with a 600,000 x 90 dense part (column scales 10^(3t)), in the
    launch configuration the benchmark times: unrefined <= 1e-5, one sweep <= 1e-10."""
    log(f"scale workload lam={lam}: generating")
    inst = gen.scale_blockangular(100, lam=lam)
    log("oracle")
    p_ref, f = refine.reference_solution(inst, sweeps=2)
    log("gpu")
    p0, st, solver, dev = gpu_solve_blockangular(inst, return_solver=True)
    assert st[0] == 0
    e0 = p_err(p0, p_ref, inst.d)
    log(f"unrefined rel err {e0:.3e}")
    assert e0 <= 1e-5
    p1 = solver.solve(sweeps=1).cpu().numpy()
    e1 = p_err(p1, p_ref, inst.d)
    log(f"1 sweep rel err {e1:.3e}")
    assert e1 <= 1e-10
    p2 = solver.solve(sweeps=2).cpu().numpy()
    assert p_err(p2, p_ref, inst.d) <= 1e-10


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_every_block_width(n, dtype):
    """Block widths 1 .. 8 with ragged blocks covering every per-block QR class: m_i < n
    (including empty blocks), m_i + n within 16, 32 and 64 rows, and dense parts in one and
    two column slots."""
    for nB in (5, 70):
        rng = np.random.default_rng(500 + 10 * n + nB)
        K = 48
        m = rng.integers(0, 56 - 0 + 1, size=K)
        m = np.minimum(m, 64 - n)
        m[:6] = [0, max(n - 1, 0), n, 16 - n, 32 - n, 64 - n if 64 - n <= 56 else 56]
        inst = gen.make_blockangular(600 + 10 * n + nB, K=K, m=m, n=n, nB=nB, lam=1e-2, dtype=dtype)
        log(f"n={n} nB={nB} {np.dtype(dtype).name} m range {m.min()}..{m.max()}")
        p_ref, _ = refine.reference_solution(inst)
        p, st = gpu_solve_blockangular(inst)
        assert st[0] == 0, st
        tol = 1e-11 if dtype == np.float64 else 1e-5
        assert p_err(p, p_ref, inst.d) <= tol
        p1, _ = gpu_solve_blockangular(inst, sweeps=2)
        assert p_err(p1, p_ref, inst.d) <= 1e-10
