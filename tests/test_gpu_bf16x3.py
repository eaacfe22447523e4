"""GPU parity of the BF16x3 mode (the dense-part trailing updates formed as three bf16
products with fp32 accumulation) against the oracle: the unrefined step carries roughly
2^-16 relative error per product, and float64-residual refinement brings it to <= 1e-10.
The bf16 split itself is pinned on the CPU (tests/test_oracle_extra.py); the matrix-core
accumulation order is parity unpinned (tolerances only)."""
import numpy as np
import pytest

from oracle import refine
from tests.gpu_util import gpu_solve_blockangular, log, rel_err
from workloads import generators as gen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [
    (100, 8, 3, 24, 1e-2),          # tiny workload shape
    (300, (4, 20), 3, 90, 1e-2),    # 6 column blocks
    (120, (8, 40), 3, 127, 1e-1),   # 8 column blocks
    (50, (3, 12), 2, 20, 1.0),      # two panels (one panel has no trailing update)
])
def test_bf16x3_unrefined_and_refined(shape):
    K, m, n, nB, lam = shape
    if isinstance(m, tuple):
        m = np.random.default_rng(K).integers(m[0], m[1] + 1, size=K)
    inst = gen.make_blockangular(600 + K, K=K, m=m, n=n, nB=nB, lam=lam, dtype=np.float32)
    p_ref, _ = refine.reference_solution(inst)
    pb, st = gpu_solve_blockangular(inst, mode="bf16x3")
    pp, _ = gpu_solve_blockangular(inst, mode="plain")
    assert st[0] == 0, st
    eb, ep = rel_err(pb, p_ref), rel_err(pp, p_ref)
    log(f"bf16x3 K={K} nB={nB}: unrefined {eb:.2e} (plain {ep:.2e})")
    assert eb <= 5e-4
    assert rel_err(pb, pp) > 1e-7  # the bf16 products are really used
    errs = [rel_err(gpu_solve_blockangular(inst, mode="bf16x3", sweeps=s)[0], p_ref) for s in (1, 2, 3)]
    log(f"  refined {errs}")
    assert min(errs) <= 1e-10


@pytest.mark.parametrize("k", [3.0, 4.0, 5.0])
def test_bf16x3_precision_workload_reaches_1e10(k):
    """Column scales 10^(k t): float32 and BF16x3 factors both reach 1e-10 within 3 sweeps."""
    inst = gen.precision_blockangular(400 + int(k), k, dtype=np.float32)
    p_ref, _ = refine.reference_solution(inst)
    for mode in ("plain", "bf16x3"):
        errs = [rel_err(gpu_solve_blockangular(inst, mode=mode, sweeps=s)[0], p_ref) for s in range(4)]
        log(f"k={k} {mode}: {['%.1e' % e for e in errs]}")
        assert min(errs[1:]) <= 1e-10, (mode, errs)


def test_bf16x3_full_scale_workload():
    """50,000 blocks of 12x3, dense part 600,000 x 90: refined BF16x3 reaches 1e-10."""
    inst = gen.scale_blockangular(100, lam=1e-2)
    p_ref, _ = refine.reference_solution(inst, sweeps=2)
    errs = [rel_err(gpu_solve_blockangular(inst, mode="bf16x3", sweeps=s)[0], p_ref) for s in range(4)]
    log(f"bf16x3 scale workload: {['%.1e' % e for e in errs]}")
    assert errs[0] <= 5e-4
    assert min(errs[1:]) <= 1e-10
