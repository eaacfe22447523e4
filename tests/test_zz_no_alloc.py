"""qrk_solve_banded_noalloc (the banded step without any device allocation, its buffers carved
from one fixed scratch array per GPU) against the handle path it replaces (qrk_create_banded_batched
+ qrk_factor_banded + qrk_solve): two calls in a row, the second with a smaller input, each equal
to the handle path's p bit for bit (the same kernels on the same inputs) and within the parity
tolerances of the oracle's solution."""
import numpy as np
import pytest

from oracle import banded as obanded
from tests.gpu_util import log, p_err
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _dev(insts):
    import torch
    rs = torch.from_numpy(np.stack([i.row_start for i in insts])).cuda().contiguous()
    vals = torch.from_numpy(np.stack([i.vals for i in insts])).cuda().contiguous()
    b = torch.from_numpy(np.stack([i.b for i in insts])).cuda().contiguous()
    d = torch.from_numpy(np.stack([i.d for i in insts])).cuda().contiguous()
    return rs, vals, b, d


def _handle_path(insts, sweeps):
    import torch
    from paper_1802_03773_amd import BandedSolver
    i0 = insts[0]
    s = BandedSolver(i0.M, i0.N, i0.w, dtype=np.dtype(i0.dtype).name, P=len(insts))
    rs, vals, b, d = _dev(insts)
    s.factor(rs, vals, b, d, i0.lam)
    p = s.solve(sweeps=sweeps)
    torch.cuda.synchronize()
    return p.cpu().numpy()


def _noalloc(insts, sweeps):
    import torch
    from paper_1802_03773_amd import qrkit
    i0 = insts[0]
    rs, vals, b, d = _dev(insts)
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    p = qrkit.solve_banded_noalloc(rs, vals, b, d, i0.lam, i0.N, sweeps=sweeps, status=status)
    torch.cuda.synchronize()
    return p.cpu().numpy(), int(status.cpu()[0])


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_noalloc_matches_handle_path_twice(dtype):
    cases = [  # (P, N, w, sweeps): the second call is smaller than the first
        (6, 700, 12, 1),
        (2, 150, 7, 0),
    ]
    for k, (P, N, w, sweeps) in enumerate(cases):
        log(f"noalloc call {k}: P={P} N={N} w={w} sweeps={sweeps} {np.dtype(dtype).name}")
        insts = [gen.make_banded(3000 + 10 * k + q, N=N, w=w, lam=1e-2, dtype=dtype) for q in range(P)]
        p_na, st = _noalloc(insts, sweeps)
        assert st == 0
        p_h = _handle_path(insts, sweeps)
        assert np.array_equal(p_na, p_h)
        tol = 1e-10 if (sweeps > 0 or dtype == np.float64) else 1e-5
        for q in (0, P - 1):
            p_ref, _, _ = obanded.reference_solution(insts[q])
            assert p_err(p_na[q * N:(q + 1) * N], p_ref, insts[q].d) <= tol


def test_noalloc_wide_band_and_bad_row_start():
    """w = 20 (no sweep copy of the band) matches the handle path; a decreasing row start sets the
    bad-input bit in the status word written to the caller's buffer."""
    insts = [gen.make_banded(3100 + q, N=90, w=20, lam=5e-2, dtype=np.float32) for q in range(3)]
    p_na, st = _noalloc(insts, 2)
    assert st == 0
    assert np.array_equal(p_na, _handle_path(insts, 2))
    bad = gen.make_banded(3200, N=60, w=5, lam=1e-2, dtype=np.float32)
    bad.row_start[20] = bad.row_start[19] - 1
    _, st = _noalloc([bad], 0)
    assert st & 4


def test_noalloc_rejects_oversized_request():
    """A request beyond the fixed scratch array returns QRK_ETOOLARGE before enqueueing anything."""
    import torch
    from paper_1802_03773_amd import qrkit
    P, M, N, w = 512, 4096, 2048, 12
    rs = torch.zeros((P, M), dtype=torch.int32, device="cuda")
    vals = torch.zeros((P, M, w), dtype=torch.float32, device="cuda")
    b = torch.zeros((P, M), dtype=torch.float32, device="cuda")
    d = torch.ones((P, N), dtype=torch.float64, device="cuda")
    with pytest.raises(qrkit.QRKError) as ei:
        qrkit.solve_banded_noalloc(rs, vals, b, d, 1e-2, N)
    assert ei.value.status == qrkit.QRK_ETOOLARGE
