"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
function declared in include/qrkit.h, and rejects bad arguments before touching the
device."""
import ctypes

import numpy as np
import pytest

from paper_1802_03773_amd import qrkit

pytestmark = pytest.mark.skipif(not __import__("os").path.exists(qrkit.LIB_PATH),
                                reason="libqrkit.so not built")


def test_every_declared_symbol_is_exported():
    L = qrkit.lib()
    names = qrkit.header_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(qrkit._SIGS) == set(names)


def test_strerror():
    L = qrkit.lib()
    assert L.qrk_strerror(0) == b"success"
    assert L.qrk_strerror(1) == b"invalid argument"
    assert L.qrk_strerror(99) == b"unknown status"


def _create(K, n, nB, row_off, ldb, dtype=0, mode=0):
    L = qrkit.lib()
    h = ctypes.c_void_p()
    ro = np.ascontiguousarray(np.asarray(row_off, np.int64))
    st = L.qrk_create_blockangular(K, n, nB, ro.ctypes.data_as(qrkit._c_i64p), ldb, dtype, mode,
                                   ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("args", [
    (0, 3, 4, [0], 4),                      # K < 1
    (2, 0, 4, [0, 1, 2], 4),                # n < 1
    (2, 9, 4, [0, 1, 2], 4),                # n > 8
    (2, 3, -1, [0, 1, 2], 4),               # nB < 0
    (2, 3, 128, [0, 1, 2], 128),            # nB > 127
    (2, 3, 4, [0, 1, 2], 3),                # ldb < nB
    (2, 3, 4, [0, 1, 2], (1 << 20) + 1),    # ldb above the limit
    (2, 3, 4, [1, 2, 3], 4),                # row_off[0] != 0
    (2, 3, 4, [0, 5, 3], 4),                # negative block
    (2, 3, 4, [0, 57, 60], 4),              # block taller than the limit
])
def test_create_rejects_bad_shapes(args):
    st, h = _create(*args)
    assert st == qrkit.QRK_EINVAL and not h.value


def test_create_rejects_bad_dtype_mode():
    assert _create(2, 3, 4, [0, 2, 4], 4, dtype=5)[0] == qrkit.QRK_EINVAL
    assert _create(2, 3, 4, [0, 2, 4], 4, mode=7)[0] == qrkit.QRK_EINVAL
    # bf16x3 trailing updates exist only for float32 factors
    assert _create(2, 3, 4, [0, 2, 4], 4, dtype=1, mode=1)[0] == qrkit.QRK_EINVAL


def test_null_handle_calls_are_rejected():
    L = qrkit.lib()
    assert L.qrk_factor_blockangular(None, None, None, None, None, 0.1, None) == qrkit.QRK_EINVAL
    assert L.qrk_solve(None, None, 0, None) == qrkit.QRK_EINVAL
    assert L.qrk_status_get(None, None, None) == qrkit.QRK_EINVAL
    assert L.qrk_get_factor(None, None, None, None, None) == qrkit.QRK_EINVAL
    assert L.qrk_solve_adjoint(None, None, None, None, None, None, None, None, None) == qrkit.QRK_EINVAL
    assert L.qrk_set_tsqr_shape(None, 0, 0) == qrkit.QRK_EINVAL
    assert L.qrk_factor_lambda(None, 1e-2, None) == qrkit.QRK_EINVAL
    assert L.qrk_solve_rhs(None, None, None, 1, None) == qrkit.QRK_EINVAL
    assert L.qrk_workspace_bytes(None) == 0
    L.qrk_destroy(None)


def test_banded_create_rejects_bad_shapes():
    L = qrkit.lib()
    h = ctypes.c_void_p()
    for M, N, w in [(-1, 10, 3), (10, 0, 3), (10, 10, 0), (10, 10, 32), (10, 4, 5)]:
        assert L.qrk_create_banded(M, N, w, 0, ctypes.byref(h)) == qrkit.QRK_EINVAL


def _create_batched(P, n, K, nB, row_off, dtype=0, mode=0):
    L = qrkit.lib()
    h = ctypes.c_void_p()
    Ka = np.ascontiguousarray(np.asarray(K, np.int32))
    nBa = np.ascontiguousarray(np.asarray(nB, np.int32))
    ro = np.ascontiguousarray(np.asarray(row_off, np.int64))
    st = L.qrk_create_blockangular_batched(P, n, Ka.ctypes.data_as(qrkit._c_i32p), nBa.ctypes.data_as(qrkit._c_i32p),
                                           ro.ctypes.data_as(qrkit._c_i64p), dtype, mode, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("args", [
    (0, 3, [1], [4], [0, 2]),                       # P < 1
    (2, 0, [1, 1], [4, 4], [0, 2, 4]),              # n < 1
    (2, 3, [1, 0], [4, 4], [0, 2, 4]),              # a problem without blocks
    (2, 3, [1, 1], [4, 128], [0, 2, 4]),            # nB > 127
    (2, 3, [1, 1], [-1, 4], [0, 2, 4]),             # nB < 0
    (2, 3, [1, 1], [4, 4], [1, 2, 4]),              # row_off[0] != 0
    (2, 3, [1, 1], [4, 4], [0, 4, 2]),              # negative block
    (2, 3, [1, 1], [4, 4], [0, 60, 62]),            # block taller than the limit
])
def test_batched_create_rejects_bad_shapes(args):
    st, h = _create_batched(*args)
    assert st == qrkit.QRK_EINVAL and not h.value


def test_batched_calls_reject_null_handle():
    L = qrkit.lib()
    assert L.qrk_factor_blockangular_batched(None, None, None, None, None, None, None) == qrkit.QRK_EINVAL
    assert L.qrk_status_get_problems(None, None, None) == qrkit.QRK_EINVAL
    assert L.qrk_autotune_blockangular(None, None, None) == qrkit.QRK_EINVAL
    assert _create_batched(2, 3, [1, 1], [4, 4], [0, 2, 4], dtype=1, mode=1)[0] == qrkit.QRK_EINVAL


def test_stack_batch_layout():
    """The batched layout: global row offsets, packed B per problem, stacked d."""
    from workloads import generators as gen
    insts = [gen.make_blockangular(s, K=k, m=5, n=2, nB=nb, lam=0.1, dtype=np.float32)
             for s, k, nb in [(1, 3, 4), (2, 2, 0), (3, 4, 7)]]
    st = gen.stack_batch(insts)
    assert list(st["K"]) == [3, 2, 4] and list(st["nB"]) == [4, 0, 7]
    assert st["row_off"].tolist() == list(range(0, 46, 5))
    assert st["B"].size == 15 * 4 + 20 * 7
    assert np.array_equal(st["B"][60:].reshape(20, 7), insts[2].B)
    assert st["d"].size == sum(i.N for i in insts)


def test_tune_cache_file_parsing(tmp_path):
    """qrk_tune_cache_file loads the autotuner's JSON cache: a file of the library's own layout
    (and a missing file) is accepted, a malformed one is refused; no device is touched."""
    L = qrkit.lib()
    good = tmp_path / "tune.json"
    good.write_text('{"version": 1, "entries": {\n  "gfx950/f32/bf16x3/P512/n3/rows67108864/L91/w3": '
                    '{"leaf_scale": 2, "leaf_queue": 1, "refine_scale": 0.5, "ms": 25.1}\n}}\n')
    assert L.qrk_tune_cache_file(str(good).encode()) == qrkit.QRK_OK
    assert L.qrk_tune_cache_file(str(tmp_path / "absent.json").encode()) == qrkit.QRK_OK
    bad = tmp_path / "bad.json"
    bad.write_text('{"version": 1, "entries": {"k": {"leaf_scale": 2}}}')
    assert L.qrk_tune_cache_file(str(bad).encode()) == qrkit.QRK_EINVAL
    assert L.qrk_tune_cache_file(None) == qrkit.QRK_OK


def test_solve_tol_rejects_bad_arguments():
    """qrk_solve_tol validates on the host: no handle or p, negative or too many sweeps, a
    negative or non-finite tolerance; and the new status has its message."""
    L = qrkit.lib()
    done = ctypes.c_int32(-1)
    assert L.qrk_solve_tol(None, None, 2, 1e-12, ctypes.byref(done), None) == qrkit.QRK_EINVAL
    assert L.qrk_strerror(qrkit.QRK_ENOTCONVERGED) == b"refinement sweeps exhausted above the requested tolerance"
    assert L.qrk_strerror(qrkit.QRK_ETOOLARGE).startswith(b"request exceeds")


def test_stored_q_entry_points_reject_null_handle():
    """qrk_set_keep_q, qrk_apply_qt and qrk_solve_qt validate on the host before any device work."""
    L = qrkit.lib()
    assert L.qrk_set_keep_q(None, 1) == qrkit.QRK_EINVAL
    assert L.qrk_set_keep_q(None, 0) == qrkit.QRK_EINVAL
    assert L.qrk_apply_qt(None, None, None, None) == qrkit.QRK_EINVAL
    assert L.qrk_solve_qt(None, None, None, 0, None) == qrkit.QRK_EINVAL


@pytest.mark.parametrize("ncol", [[3, 0, 2], [3, 9, 2], [1, 2, -1]])
def test_ncol_create_rejects_bad_widths(ncol):
    """qrk_create_blockangular_ncol: every block width in 1..8, checked on the host."""
    L = qrkit.lib()
    h = ctypes.c_void_p()
    ro = np.array([0, 4, 8, 12], dtype=np.int64)
    nc = np.asarray(ncol, dtype=np.int32)
    st = L.qrk_create_blockangular_ncol(3, nc.ctypes.data_as(qrkit._c_i32p), 5, ro.ctypes.data_as(qrkit._c_i64p), 5,
                                        0, 0, ctypes.byref(h))
    assert st == qrkit.QRK_EINVAL and not h.value
    assert L.qrk_create_blockangular_ncol(3, None, 5, ro.ctypes.data_as(qrkit._c_i64p), 5, 0, 0,
                                          ctypes.byref(h)) == qrkit.QRK_EINVAL
    assert L.qrk_create_blockangular_ncol(3, nc.ctypes.data_as(qrkit._c_i32p), 5, ro.ctypes.data_as(qrkit._c_i64p),
                                          5, 0, 0, None) == qrkit.QRK_EINVAL


@pytest.mark.parametrize("ncam,cw", [(0, 9), (3, 0), (15, 9), (128, 1), (-1, 4)])
def test_cam_create_rejects_bad_cameras(ncam, cw):
    """qrk_create_blockangular_cam: ncam >= 1, cw >= 1 and ncam * cw <= 127, checked on the host."""
    L = qrkit.lib()
    h = ctypes.c_void_p()
    ro = np.array([0, 4, 8, 12], dtype=np.int64)
    st = L.qrk_create_blockangular_cam(3, 3, ncam, cw, ro.ctypes.data_as(qrkit._c_i64p), 0, 0, ctypes.byref(h))
    assert st == qrkit.QRK_EINVAL and not h.value
    assert L.qrk_create_blockangular_cam(3, 3, 4, 9, ro.ctypes.data_as(qrkit._c_i64p), 0, 0,
                                         None) == qrkit.QRK_EINVAL


def test_cam_entry_points_reject_null_handle():
    L = qrkit.lib()
    assert L.qrk_factor_blockangular_cam(None, None, None, None, None, None, 1e-2, None) == qrkit.QRK_EINVAL
    assert L.qrk_colnorms_blockangular_cam(None, None, None, None, None, None) == qrkit.QRK_EINVAL
