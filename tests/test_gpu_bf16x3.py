"""GPU parity of the BF16x3 mode (the dense-part trailing updates formed as three bf16
products with fp32 accumulation) against the oracle: the unrefined step carries roughly
2^-16 relative error per product, and float64-residual refinement brings it to <= 1e-10.
The device split (the kernels' own bf_split) is compared bit for bit with the oracle's
emulation, and the matrix-core tile product with the oracle's three-product sum; the
matrix-core accumulation order is parity unpinned (a rounding-level tolerance only)."""
import numpy as np
import pytest

from oracle import bf16, refine
from tests.gpu_util import p_err, gpu_solve_blockangular, log, rel_err
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
    eb, ep = p_err(pb, p_ref, inst.d), p_err(pp, p_ref, inst.d)
    log(f"bf16x3 K={K} nB={nB}: unrefined {eb:.2e} (plain {ep:.2e})")
    assert eb <= 5e-4
    assert rel_err(pb, pp) > 1e-7  # the bf16 products are really used
    errs = [p_err(gpu_solve_blockangular(inst, mode="bf16x3", sweeps=s)[0], p_ref, inst.d) for s in (1, 2, 3)]
    log(f"  refined {errs}")
    assert min(errs) <= 1e-10


@pytest.mark.parametrize("k", [3.0, 4.0, 5.0])
def test_bf16x3_precision_workload_reaches_1e10(k):
    """Column scales 10^(k t): float32 and BF16x3 factors both reach 1e-10 within 3 sweeps."""
    inst = gen.precision_blockangular(400 + int(k), k, dtype=np.float32)
    p_ref, _ = refine.reference_solution(inst)
    for mode in ("plain", "bf16x3"):
        errs = [p_err(gpu_solve_blockangular(inst, mode=mode, sweeps=s)[0], p_ref, inst.d) for s in range(4)]
        log(f"k={k} {mode}: {['%.1e' % e for e in errs]}")
        assert errs[3] <= 1e-10, (mode, errs)


def test_bf16x3_full_scale_workload():
    """50,000 blocks of 12x3, dense part 600,000 x 90: refined BF16x3 reaches 1e-10."""
    inst = gen.scale_blockangular(100, lam=1e-2)
    p_ref, _ = refine.reference_solution(inst, sweeps=2)
    errs = [p_err(gpu_solve_blockangular(inst, mode="bf16x3", sweeps=s)[0], p_ref, inst.d) for s in range(4)]
    log(f"bf16x3 scale workload: {['%.1e' % e for e in errs]}")
    assert errs[0] <= 5e-4
    assert errs[1] <= 1e-10  # the benchmark's sweep count


def _split_inputs():
    rng = np.random.default_rng(81)
    x = (rng.standard_normal(200_000) * 10.0 ** rng.uniform(-30, 30, 200_000)).astype(np.float32)
    # exact ties of the first rounding (low 16 bits 0x8000), both parities of bit 16
    top = rng.integers(0, 2**15, 4000).astype(np.uint32) << np.uint32(16)
    ties = (np.uint32(0x3F800000) ^ (top & np.uint32(0x007F0000))) | np.uint32(0x8000)
    # values whose remainder x - hi is itself a tie of the second rounding
    low = np.where(np.arange(top.size) % 2 == 0, np.uint32(0x0101), np.uint32(0x0103)).astype(np.uint32)
    rem = (np.uint32(0x40000000) | (top & np.uint32(0x007F0000)) | low).view(np.float32)
    return np.concatenate([x, ties.view(np.float32), rem, np.float32([0.0, -0.0, 1.0, -3.5])])


def test_device_bf16_split_bit_exact():
    """The dense-part kernels' split hi = bf16(x), lo = bf16(x - hi) (round to nearest even)
    against the oracle's bit-level emulation, bit for bit (normal-range values, ties included)."""
    import torch
    from paper_1802_03773_amd import qrkit
    x = _split_inputs()
    hi, lo = qrkit.check_bf16_split(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    hi_o, lo_o = bf16.split(x)
    assert np.array_equal(hi.cpu().numpy().view(np.uint32), hi_o.view(np.uint32))
    assert np.array_equal(lo.cpu().numpy().view(np.uint32), lo_o.view(np.uint32))


@pytest.mark.parametrize("k", [32, 64, 96, 512])
def test_device_bf16x3_tile_product(k):
    """A 16 x k by k x 16 product in the trailing updates' layout and order against the oracle's
    three-product emulation: every bf16 x bf16 product is exact in fp32, so the two differ only
    by fp32 accumulation order, at most 3k roundings of 2^-24 of sum |a||b| per entry; both are
    within the split's 2^-15 relative bound of the float64 product."""
    import torch
    from paper_1802_03773_amd import qrkit
    rng = np.random.default_rng(82 + k)
    A = (rng.standard_normal((16, k)) * 10.0 ** rng.uniform(-2, 2, (16, k))).astype(np.float32)
    B = (rng.standard_normal((k, 16)) * 10.0 ** rng.uniform(-2, 2, (k, 16))).astype(np.float32)
    C = qrkit.check_bf16x3_product(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
    torch.cuda.synchronize()
    C = C.cpu().numpy().astype(np.float64)
    Ce = bf16.bf16x3_matmul(A, B).astype(np.float64)
    absprod = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    assert np.all(np.abs(C - Ce) <= 3 * k * 2.0 ** -24 * absprod)
    C64 = A.astype(np.float64) @ B.astype(np.float64)
    assert np.all(np.abs(C - C64) <= 2.0 ** -15 * absprod)
    # a plain bf16 product (hi*hi only) would be off by about 2^-9: the lo terms are really used
    hA, _ = bf16.split(A)
    hB, _ = bf16.split(B)
    Chh = hA.astype(np.float64) @ hB.astype(np.float64)
    assert np.abs(C - C64).max() < 0.01 * np.abs(Chh - C64).max()
