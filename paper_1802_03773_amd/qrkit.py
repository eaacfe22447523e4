"""Python binding of libqrkit.so (ctypes; argument marshalling only).

Every step of the LM step solve runs in the library's HIP kernels; torch supplies
device memory and the current HIP stream.  There is no CPU fallback: if the library
is missing or no gfx950 device is present, the calls raise.

Names follow the C ABI of include/qrkit.h:
    factor_blockangular / factor_banded   -> compute(A) and Q^T b  (paper Section 5.1)
    Factor.solve                          -> R.solve(Q^T b), plus refinement sweeps
    Factor.solve_adjoint                  -> gradients of a loss of p
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libqrkit.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "qrkit.h")

(QRK_OK, QRK_EINVAL, QRK_ENOMEM, QRK_EHIP, QRK_ESINGULAR, QRK_ENONFINITE, QRK_ENODEVICE, QRK_ETOOLARGE,
 QRK_ENOTCONVERGED) = range(9)
NOALLOC_SCRATCH_BYTES = 32 << 20
QRK_F32, QRK_F64 = 0, 1
QRK_PLAIN, QRK_BF16X3 = 0, 1
MAX_BLOCK_COLS, MAX_BLOCK_ROWS, MAX_DENSE_COLS, MAX_BAND = 8, 56, 127, 31

_c_i32, _c_i64, _c_dbl, _c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_i32p = ctypes.POINTER(ctypes.c_int32)

_SIGS = {
    "qrk_create_blockangular": (_c_i32, [_c_i32, _c_i32, _c_i32, _c_i64p, _c_i64, _c_i32, _c_i32,
                                         ctypes.POINTER(_c_vp)]),
    "qrk_create_blockangular_ncol": (_c_i32, [_c_i32, _c_i32p, _c_i32, _c_i64p, _c_i64, _c_i32, _c_i32,
                                              ctypes.POINTER(_c_vp)]),
    "qrk_factor_blockangular": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_dbl, _c_vp]),
    "qrk_create_blockangular_cam": (_c_i32, [_c_i32, _c_i32, _c_i32, _c_i32, _c_i64p, _c_i32, _c_i32,
                                             ctypes.POINTER(_c_vp)]),
    "qrk_factor_blockangular_cam": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_dbl, _c_vp]),
    "qrk_colnorms_blockangular_cam": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp]),
    "qrk_discover_blockangular": (_c_i32, [_c_i64, _c_i64, _c_i64p, _c_i32p, _c_i32, _c_i32p, _c_i64p, _c_i32p,
                                           _c_i32p, _c_i64p, _c_i32p]),
    "qrk_discover_banded": (_c_i32, [_c_i64, _c_i64, _c_i64p, _c_i32p, _c_i64p, _c_i32p, _c_i32p]),
    "qrk_factor_lambda": (_c_i32, [_c_vp, _c_dbl, _c_vp]),
    "qrk_create_blockangular_batched": (_c_i32, [_c_i32, _c_i32, _c_i32p, _c_i32p, _c_i64p, _c_i32, _c_i32,
                                                 ctypes.POINTER(_c_vp)]),
    "qrk_factor_blockangular_batched": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp]),
    "qrk_status_get_problems": (_c_i32, [_c_vp, _c_i32p, _c_vp]),
    "qrk_autotune_blockangular": (_c_i32, [_c_vp, ctypes.POINTER(_c_dbl), _c_vp]),
    "qrk_tune_get": (_c_i32, [_c_vp, ctypes.POINTER(_c_dbl), _c_i32p, ctypes.POINTER(_c_dbl)]),
    "qrk_tune_cache_file": (_c_i32, [ctypes.c_char_p]),
    "qrk_lm_create_blockangular": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_dbl, _c_i32, _c_i32,
                                            ctypes.POINTER(_c_vp)]),
    "qrk_lm_create_banded": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_dbl, _c_i32, _c_i32, ctypes.POINTER(_c_vp)]),
    "qrk_lm_reset": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp]),
    "qrk_lm_run": (_c_i32, [_c_vp, _c_i32, _c_i32, _c_vp]),
    "qrk_lm_get": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_i32p, _c_vp]),
    "qrk_lm_destroy": (None, [_c_vp]),
    "qrk_create_banded": (_c_i32, [_c_i64, _c_i64, _c_i32, _c_i32, ctypes.POINTER(_c_vp)]),
    "qrk_create_banded_batched": (_c_i32, [_c_i32, _c_i64, _c_i64, _c_i32, _c_i32, ctypes.POINTER(_c_vp)]),
    "qrk_factor_banded": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_dbl, _c_vp]),
    "qrk_set_banded_method": (_c_i32, [_c_vp, _c_i32]),
    "qrk_solve": (_c_i32, [_c_vp, _c_vp, _c_i32, _c_vp]),
    "qrk_solve_rhs": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i32, _c_vp]),
    "qrk_solve_tol": (_c_i32, [_c_vp, _c_vp, _c_i32, _c_dbl, _c_i32p, _c_vp]),
    "qrk_factor_vcat": (_c_i32, [_c_vp, _c_vp, _c_vp]),
    "qrk_set_keep_q": (_c_i32, [_c_vp, _c_i32]),
    "qrk_apply_qt": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp]),
    "qrk_solve_qt": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i32, _c_vp]),
    "qrk_solve_adjoint": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp]),
    "qrk_colnorms_blockangular": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp]),
    "qrk_get_factor": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp]),
    "qrk_status_get": (_c_i32, [_c_vp, _c_i32p, _c_vp]),
    "qrk_set_tsqr_shape": (_c_i32, [_c_vp, _c_i32, _c_i32]),
    "qrk_workspace_bytes": (_c_i64, [_c_vp]),
    "qrk_profile_enable": (_c_i32, [_c_vp, _c_i32]),
    "qrk_profile_read": (_c_i32, [_c_vp, ctypes.POINTER(_c_dbl), _c_i32p, _c_i32]),
    "qrk_check_bf16_split": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i64, _c_vp]),
    "qrk_check_bf16x3_product": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i32, _c_vp]),
    "qrk_solve_banded_noalloc": (_c_i32, [_c_i32, _c_i64, _c_i64, _c_i32, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp,
                                          _c_dbl, _c_vp, _c_i32, _c_vp, _c_vp]),
    "qrk_destroy": (None, [_c_vp]),
    "qrk_strerror": (ctypes.c_char_p, [_c_i32]),
}

_LIB = None


def header_functions() -> list[str]:
    """Names of every function declared in include/qrkit.h."""
    with open(HEADER_PATH) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qrk_[a-z0-9_]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    """Load libqrkit.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1802_03773_amd.build`")
        # torch's GPU runtime is brought up before the library's first HIP call: started the other
        # way round, torch found no GPU in the same process
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


class QRKError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        msg = lib().qrk_strerror(int(status)).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


def _check(status: int, what: str):
    if status != QRK_OK:
        raise QRKError(status, what)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype, name, numel=None):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _torch_dtype(qdtype):
    torch = _torch()
    return torch.float32 if qdtype == QRK_F32 else torch.float64


class Factor:
    """A qrkit handle plus the borrowed inputs of its last factor call."""

    def __init__(self, handle, kind: str, dtype: int, N: int):
        self._h = handle
        self.kind = kind
        self.qdtype = dtype
        self.N = N
        self._keep = ()

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h is not None and _LIB is not None:
            _LIB.qrk_destroy(h)

    def solve(self, sweeps: int = 0, out=None, stream=None):
        """Back-substitution (plus `sweeps` float64-residual refinement sweeps); p float64 [N]."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(lib().qrk_solve(self._h, _dev_ptr(out, torch.float64, "p", self.N), int(sweeps),
                               _stream_ptr(stream)), "qrk_solve")
        return out

    def solve_tol(self, max_sweeps: int = 3, rel_tol: float = 1e-12, out=None, stream=None):
        """Back-substitution, then refinement sweeps until ||delta|| <= rel_tol ||p|| for every
        problem or max_sweeps ran out.  Returns (p float64, sweeps run, converged)."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64, device="cuda")
        done = _c_i32(0)
        st = lib().qrk_solve_tol(self._h, _dev_ptr(out, torch.float64, "p", self.N), int(max_sweeps),
                                 float(rel_tol), ctypes.byref(done), _stream_ptr(stream))
        if st not in (QRK_OK, QRK_ENOTCONVERGED):
            _check(st, "qrk_solve_tol")
        return out, int(done.value), st == QRK_OK

    def solve_rhs(self, b, sweeps: int = 4, out=None, stream=None):
        """The step for a new right-hand side b (same J, d, lambda as the last factor), by
        `sweeps` corrected semi-normal sweeps from p = 0 with the stored R; p float64 [N].
        Four sweeps reach 1e-10 for float32 factors at cond(J) <= 1e3."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(lib().qrk_solve_rhs(self._h, _dev_ptr(b, _torch_dtype(self.qdtype), "b", self._rhs_rows()),
                                   _dev_ptr(out, torch.float64, "p", self.N), int(sweeps), _stream_ptr(stream)),
               "qrk_solve_rhs")
        return out

    def set_keep_q(self, keep: bool = True):
        """Keep Q at the following factor calls (float32 block-angular handles whose blocks all
        have m_i >= n): the per-block reflectors and the dense part's compact-WY panels, which
        apply_qt and solve_qt use."""
        _check(lib().qrk_set_keep_q(self._h, 1 if keep else 0), "qrk_set_keep_q")

    def apply_qt(self, b, out=None, stream=None):
        """The first N entries of Q^T [b; 0] with the stored Q of the last factor call: c_i of
        every block, then c_B (laid out like p); float64 [N]."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(lib().qrk_apply_qt(self._h, _dev_ptr(b, _torch_dtype(self.qdtype), "b", self._rhs_rows()),
                                  _dev_ptr(out, torch.float64, "c", self.N), _stream_ptr(stream)),
               "qrk_apply_qt")
        return out

    def solve_qt(self, b, sweeps: int = 0, out=None, stream=None):
        """The step for a new right-hand side b with the stored Q: p = R^{-1} (Q^T b) (the first N
        entries), then `sweeps` (0..8) refinement sweeps for b; p float64 [N]."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(lib().qrk_solve_qt(self._h, _dev_ptr(b, _torch_dtype(self.qdtype), "b", self._rhs_rows()),
                                  _dev_ptr(out, torch.float64, "p", self.N), int(sweeps), _stream_ptr(stream)),
               "qrk_solve_qt")
        return out

    def _rhs_rows(self) -> int:
        return int(self.P) * int(self.M) if self.kind == "banded" else int(self.M)

    def status(self, stream=None) -> tuple[int, int]:
        detail = ctypes.c_int32(0)
        st = lib().qrk_status_get(self._h, ctypes.byref(detail), _stream_ptr(stream))
        return int(st), int(detail.value)

    def raise_on_status(self, stream=None):
        st, _ = self.status(stream)
        _check(st, "device status")

    def workspace_bytes(self) -> int:
        return int(lib().qrk_workspace_bytes(self._h))

    PHASES = ("block_qr", "dense_leaves", "dense_tree", "backsub", "refine", "banded")

    def profile_enable(self, max_calls: int):
        _check(lib().qrk_profile_enable(self._h, int(max_calls)), "qrk_profile_enable")

    def profile_read(self) -> dict:
        """{phase: (milliseconds summed, launches)} since enable or the previous read."""
        n = len(self.PHASES)
        ms = (_c_dbl * n)()
        cnt = (_c_i32 * n)()
        _check(lib().qrk_profile_read(self._h, ms, cnt, n), "qrk_profile_read")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(self.PHASES)}


class BlockAngularSolver(Factor):
    """Solver for J = [blkdiag(A_1..A_K) | B] (K blocks of n columns, nB dense columns)."""

    def __init__(self, row_off, n: int, nB: int, ldb: Optional[int] = None, dtype="float32",
                 mode: str = "plain"):
        row_off = np.ascontiguousarray(np.asarray(row_off, dtype=np.int64))
        K = int(row_off.shape[0] - 1)
        qd = QRK_F32 if str(dtype).endswith("float32") else QRK_F64
        qm = {"plain": QRK_PLAIN, "bf16x3": QRK_BF16X3}[mode]
        ldb = nB if ldb is None else int(ldb)
        h = _c_vp()
        st = lib().qrk_create_blockangular(K, int(n), int(nB), row_off.ctypes.data_as(_c_i64p), ldb,
                                           qd, qm, ctypes.byref(h))
        _check(st, "qrk_create_blockangular")
        super().__init__(h, "blockangular", qd, K * int(n) + int(nB))
        self.K, self.n, self.nB, self.ldb, self.M = K, int(n), int(nB), ldb, int(row_off[-1])
        self.row_off = row_off
        self.mode = mode

    def factor_vcat(self, other: "BlockAngularSolver", stream=None):
        """Vertical concatenation (Section 4.5): this handle's factor becomes that of the problem with
        its rows and `other`'s (both factored, same K, n, nB, dtype); `other` and its inputs must stay
        alive until this handle's next factor call, since solves refine against both."""
        _check(lib().qrk_factor_vcat(self._h, other._h, _stream_ptr(stream)), "qrk_factor_vcat")
        self._keep = tuple(self._keep) + (other,)

    def _a_len(self) -> int:
        return self.M * self.n

    def set_tsqr_shape(self, leaves: int = 0, fanin: int = 0):
        _check(lib().qrk_set_tsqr_shape(self._h, int(leaves), int(fanin)), "qrk_set_tsqr_shape")

    def autotune(self, stream=None) -> float:
        """Time a few dense-part leaf shapes on the last factor call's inputs; keep the best."""
        scale = _c_dbl(0.0)
        _check(lib().qrk_autotune_blockangular(self._h, ctypes.byref(scale), _stream_ptr(stream)),
               "qrk_autotune_blockangular")
        return float(scale.value)

    def factor(self, A, B, b, d, lam: float, stream=None):
        torch = _torch()
        td = _torch_dtype(self.qdtype)
        pa = _dev_ptr(A, td, "A", self._a_len())
        pB = _dev_ptr(B, td, "B", self.M * self.ldb) if self.nB > 0 else (
            _dev_ptr(B, td, "B") if B is not None else None)
        pb = _dev_ptr(b, td, "b", self.M)
        pd = _dev_ptr(d, torch.float64, "d", self.N)
        _check(lib().qrk_factor_blockangular(self._h, pa, pB, pb, pd, float(lam), _stream_ptr(stream)),
               "qrk_factor_blockangular")
        self._keep = (A, B, b, d)
        self.lam = float(lam)
        return self

    def factor_lambda(self, lam: float, stream=None):
        """Moré's two-stage damping: after factor(..., lam=0), factor [R; sqrt(lam) D] from the
        kept factor of J (qrk_factor_lambda); solve() then solves the damped problem."""
        _check(lib().qrk_factor_lambda(self._h, float(lam), _stream_ptr(stream)), "qrk_factor_lambda")
        self.lam = float(lam)
        return self

    def colnorms(self, A, B, out=None, stream=None):
        torch = _torch()
        td = _torch_dtype(self.qdtype)
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(lib().qrk_colnorms_blockangular(self._h, _dev_ptr(A, td, "A", self.M * self.n),
                                               _dev_ptr(B, td, "B") if B is not None else None,
                                               _dev_ptr(out, torch.float64, "d", self.N),
                                               _stream_ptr(stream)), "qrk_colnorms_blockangular")
        return out

    def get_factor(self, stream=None):
        """(Rblk [K,n,n], S [K,n,nB+1], RB [nB+1,nB+1]) copies of the stored factor."""
        torch = _torch()
        td = _torch_dtype(self.qdtype)
        L = self.nB + 1
        Rblk = torch.empty((self.K, self.n, self.n), dtype=td, device="cuda")
        S = torch.empty((self.K, self.n, L), dtype=td, device="cuda")
        RB = torch.empty((L, L), dtype=td, device="cuda")
        _check(lib().qrk_get_factor(self._h, _dev_ptr(Rblk, td, "Rblk"), _dev_ptr(S, td, "S"),
                                    _dev_ptr(RB, td, "RB"), _stream_ptr(stream)), "qrk_get_factor")
        return Rblk, S, RB

    def solve_adjoint(self, p, g, want=("dA", "dB", "db", "dlam", "dd"), stream=None):
        torch = _torch()
        td = _torch_dtype(self.qdtype)
        out = {}
        if "dA" in want:
            out["dA"] = torch.empty((self.M, self.n), dtype=td, device="cuda")
        if "dB" in want and self.nB > 0:
            out["dB"] = torch.zeros((self.M, self.ldb), dtype=td, device="cuda")
        if "db" in want:
            out["db"] = torch.empty(self.M, dtype=td, device="cuda")
        if "dlam" in want:
            out["dlam"] = torch.empty(1, dtype=torch.float64, device="cuda")
        if "dd" in want:
            out["dd"] = torch.empty(self.N, dtype=torch.float64, device="cuda")

        def ptr(k, dt):
            return _dev_ptr(out[k], dt, k) if k in out else None

        _check(lib().qrk_solve_adjoint(self._h, _dev_ptr(p, torch.float64, "p", self.N),
                                       _dev_ptr(g, torch.float64, "g", self.N), ptr("dA", td),
                                       ptr("dB", td), ptr("db", td), ptr("dlam", torch.float64),
                                       ptr("dd", torch.float64), _stream_ptr(stream)),
               "qrk_solve_adjoint")
        return out



class BlockAngularNcolSolver(BlockAngularSolver):
    """Block-angular J whose block i has its own column count ncol[i] (1..8): A holds block
    i's rows row-major with ncol[i] values each, block after block; d and p hold block i's
    unknowns, then the dense part's (qrk_create_blockangular_ncol).  factor() needs lam > 0;
    get_factor() returns the factor at max(ncol) columns per block."""

    def __init__(self, row_off, ncol, nB: int, ldb: Optional[int] = None, dtype="float32",
                 mode: str = "plain"):
        row_off = np.ascontiguousarray(np.asarray(row_off, dtype=np.int64))
        ncol = np.ascontiguousarray(np.asarray(ncol, dtype=np.int32))
        K = int(row_off.shape[0] - 1)
        if ncol.shape != (K,):
            raise ValueError(f"ncol has shape {ncol.shape}, needs ({K},)")
        qd = QRK_F32 if str(dtype).endswith("float32") else QRK_F64
        qm = {"plain": QRK_PLAIN, "bf16x3": QRK_BF16X3}[mode]
        ldb = nB if ldb is None else int(ldb)
        h = _c_vp()
        st = lib().qrk_create_blockangular_ncol(K, ncol.ctypes.data_as(_c_i32p), int(nB),
                                                row_off.ctypes.data_as(_c_i64p), ldb, qd, qm, ctypes.byref(h))
        _check(st, "qrk_create_blockangular_ncol")
        Factor.__init__(self, h, "blockangular", qd, int(ncol.sum()) + int(nB))
        self.K, self.n, self.nB, self.ldb, self.M = K, int(ncol.max()), int(nB), ldb, int(row_off[-1])
        self.row_off = row_off
        self.ncol = ncol
        self.mode = mode

    def _a_len(self) -> int:
        return int((np.diff(self.row_off) * self.ncol).sum())

class BlockAngularCamSolver(BlockAngularSolver):
    """Block-angular J whose nB = ncam * cw coupled columns are cameras of cw columns, every row
    on at most one camera (qrk_create_blockangular_cam): B is passed compressed as Bv [M, cw]
    (each row's values) and cam int32 [M] (each row's camera; outside [0, ncam): none)."""

    def __init__(self, row_off, n: int, ncam: int, cw: int, dtype="float32", mode: str = "plain"):
        row_off = np.ascontiguousarray(np.asarray(row_off, dtype=np.int64))
        K = int(row_off.shape[0] - 1)
        qd = QRK_F32 if str(dtype).endswith("float32") else QRK_F64
        qm = {"plain": QRK_PLAIN, "bf16x3": QRK_BF16X3}[mode]
        h = _c_vp()
        _check(lib().qrk_create_blockangular_cam(K, int(n), int(ncam), int(cw), row_off.ctypes.data_as(_c_i64p),
                                                 qd, qm, ctypes.byref(h)), "qrk_create_blockangular_cam")
        nB = int(ncam) * int(cw)
        Factor.__init__(self, h, "blockangular", qd, K * int(n) + nB)
        self.K, self.n, self.nB, self.ldb, self.M = K, int(n), nB, int(cw), int(row_off[-1])
        self.ncam, self.cw = int(ncam), int(cw)
        self.row_off = row_off
        self.mode = mode

    def factor(self, A, Bv, cam, b, d, lam: float, stream=None):
        torch = _torch()
        td = _torch_dtype(self.qdtype)
        _check(lib().qrk_factor_blockangular_cam(self._h, _dev_ptr(A, td, "A", self.M * self.n),
                                                 _dev_ptr(Bv, td, "Bv", self.M * self.cw),
                                                 _dev_ptr(cam, torch.int32, "cam", self.M),
                                                 _dev_ptr(b, td, "b", self.M), _dev_ptr(d, torch.float64, "d", self.N),
                                                 float(lam), _stream_ptr(stream)), "qrk_factor_blockangular_cam")
        self._keep = (A, Bv, cam, b, d)
        self.lam = float(lam)
        return self

    def colnorms(self, A, Bv, cam, out=None, stream=None):
        torch = _torch()
        td = _torch_dtype(self.qdtype)
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(lib().qrk_colnorms_blockangular_cam(self._h, _dev_ptr(A, td, "A", self.M * self.n),
                                                   _dev_ptr(Bv, td, "Bv", self.M * self.cw),
                                                   _dev_ptr(cam, torch.int32, "cam", self.M),
                                                   _dev_ptr(out, torch.float64, "d", self.N), _stream_ptr(stream)),
               "qrk_colnorms_blockangular_cam")
        return out


class BlockAngularBatch(Factor):
    """P independent block-angular problems with the same block width n, factored and solved
    in the same launches.  Problem p: K[p] blocks, nB[p] dense columns.  Stacked arrays,
    problem after problem: A [M_tot, n], b [M_tot]; B flat, problem p's M_p x nB[p] rows
    packed with row stride nB[p]; d and p [sum_p N_p]; lam [P] float64 on the device."""

    def __init__(self, K, nB, row_off, n: int, dtype="float32", mode: str = "plain"):
        K = np.ascontiguousarray(np.asarray(K, dtype=np.int32))
        nB = np.ascontiguousarray(np.asarray(nB, dtype=np.int32))
        row_off = np.ascontiguousarray(np.asarray(row_off, dtype=np.int64))
        if K.shape != nB.shape or row_off.shape[0] != int(K.sum()) + 1:
            raise ValueError("K, nB and row_off do not describe the same batch")
        qd = QRK_F32 if str(dtype).endswith("float32") else QRK_F64
        qm = {"plain": QRK_PLAIN, "bf16x3": QRK_BF16X3}[mode]
        h = _c_vp()
        _check(lib().qrk_create_blockangular_batched(int(K.shape[0]), int(n), K.ctypes.data_as(_c_i32p),
                                                     nB.ctypes.data_as(_c_i32p), row_off.ctypes.data_as(_c_i64p),
                                                     qd, qm, ctypes.byref(h)), "qrk_create_blockangular_batched")
        self.P, self.n = int(K.shape[0]), int(n)
        self.K, self.nB, self.row_off = K, nB, row_off
        koff = np.concatenate([[0], np.cumsum(K)])
        self.M_p = row_off[koff[1:]] - row_off[koff[:-1]]
        self.N_p = K.astype(np.int64) * self.n + nB
        self.M = int(row_off[-1])
        self.B_elems = int(np.sum(self.M_p * nB))
        super().__init__(h, "blockangular_batch", qd, int(self.N_p.sum()))
        self.mode = mode

    def factor(self, A, B, b, d, lam, stream=None):
        torch = _torch()
        td = _torch_dtype(self.qdtype)
        pB = _dev_ptr(B, td, "B", self.B_elems) if self.B_elems > 0 else (
            _dev_ptr(B, td, "B") if B is not None else None)
        _check(lib().qrk_factor_blockangular_batched(
            self._h, _dev_ptr(A, td, "A", self.M * self.n), pB, _dev_ptr(b, td, "b", self.M),
            _dev_ptr(d, torch.float64, "d", self.N), _dev_ptr(lam, torch.float64, "lam", self.P),
            _stream_ptr(stream)), "qrk_factor_blockangular_batched")
        self._keep = (A, B, b, d, lam)
        return self

    def autotune(self, stream=None) -> float:
        scale = _c_dbl(0.0)
        _check(lib().qrk_autotune_blockangular(self._h, ctypes.byref(scale), _stream_ptr(stream)),
               "qrk_autotune_blockangular")
        return float(scale.value)

    def status_problems(self, stream=None) -> np.ndarray:
        bits = np.zeros(self.P, dtype=np.int32)
        _check(lib().qrk_status_get_problems(self._h, bits.ctypes.data_as(_c_i32p), _stream_ptr(stream)),
               "qrk_status_get_problems")
        return bits


class BandedSolver(Factor):
    """Solver for banded J (M x N, w values per row at nondecreasing starts); P problems of the
    same shape may be stacked in one handle (arrays [P, ...])."""

    def __init__(self, M: int, N: int, w: int, dtype="float32", P: int = 1):
        qd = QRK_F32 if str(dtype).endswith("float32") else QRK_F64
        h = _c_vp()
        if P == 1:
            _check(lib().qrk_create_banded(int(M), int(N), int(w), qd, ctypes.byref(h)), "qrk_create_banded")
        else:
            _check(lib().qrk_create_banded_batched(int(P), int(M), int(N), int(w), qd, ctypes.byref(h)),
                   "qrk_create_banded_batched")
        super().__init__(h, "banded", qd, int(P) * int(N))
        self.M, self.w, self.P, self.Nper = int(M), int(w), int(P), int(N)
        self.method = "givens"

    METHODS = {"givens": 0, "blockwy": 1, "blockwy-bf16x3": 2}

    def set_method(self, method: str):
        """Factorisation of the next factor call: "givens" (rotations row by row), "blockwy"
        (block-banded compact-WY steps on the matrix cores, Section 4.4) or "blockwy-bf16x3"."""
        _check(lib().qrk_set_banded_method(self._h, self.METHODS[method]), "qrk_set_banded_method")
        self.method = method
        return self

    def factor(self, row_start, vals, b, d, lam: float, stream=None):
        torch = _torch()
        td = _torch_dtype(self.qdtype)
        PM = self.P * self.M
        _check(lib().qrk_factor_banded(self._h, _dev_ptr(row_start, torch.int32, "row_start", PM),
                                       _dev_ptr(vals, td, "vals", PM * self.w),
                                       _dev_ptr(b, td, "b", PM), _dev_ptr(d, torch.float64, "d", self.N),
                                       float(lam), _stream_ptr(stream)), "qrk_factor_banded")
        self._keep = (row_start, vals, b, d)
        self.lam = float(lam)
        return self

    def get_factor(self, stream=None):
        """(R band [P*N, w] with row j = R[j, j..j+w-1], c [P*N])."""
        torch = _torch()
        td = _torch_dtype(self.qdtype)
        R = torch.empty((self.N, self.w), dtype=td, device="cuda")
        c = torch.empty(self.N, dtype=td, device="cuda")
        _check(lib().qrk_get_factor(self._h, _dev_ptr(R, td, "R"), _dev_ptr(c, td, "c"), None,
                                    _stream_ptr(stream)), "qrk_get_factor")
        return R, c

    def solve_adjoint(self, p, g, stream=None):
        torch = _torch()
        td = _torch_dtype(self.qdtype)
        PM = self.P * self.M
        out = dict(dvals=torch.empty((PM, self.w), dtype=td, device="cuda"),
                   db=torch.empty(PM, dtype=td, device="cuda"),
                   dlam=torch.empty(self.P, dtype=torch.float64, device="cuda"),
                   dd=torch.empty(self.N, dtype=torch.float64, device="cuda"))
        _check(lib().qrk_solve_adjoint(self._h, _dev_ptr(p, torch.float64, "p", self.N),
                                       _dev_ptr(g, torch.float64, "g", self.N),
                                       _dev_ptr(out["dvals"], td, "dvals"), None,
                                       _dev_ptr(out["db"], td, "db"),
                                       _dev_ptr(out["dlam"], torch.float64, "dlam"),
                                       _dev_ptr(out["dd"], torch.float64, "dd"), _stream_ptr(stream)),
               "qrk_solve_adjoint")
        return out


def factor_blockangular(row_off, A, B, b, d, lam, n: int, dtype="float32", mode="plain", stream=None):
    """Convenience: create a block-angular solver and factor one instance."""
    nB = 0 if B is None else int(B.shape[1])
    s = BlockAngularSolver(row_off, n, nB, dtype=dtype, mode=mode)
    return s.factor(A, B, b, d, lam, stream=stream)


def factor_banded(row_start, vals, b, d, lam, N: int, dtype="float32", stream=None):
    M, w = int(vals.shape[0]), int(vals.shape[1])
    s = BandedSolver(M, N, w, dtype=dtype)
    return s.factor(row_start, vals, b, d, lam, stream=stream)


class LMDriver:
    """Backtrack-LM iterations on f(x) = J0 phi(x) - y (phi(t) = t + c t^3) over every problem of
    a block-angular solver or batch or a banded solver, run by the library (optionally as a
    replayed HIP graph)."""

    def __init__(self, solver, A0, B0, y, c: float, sweeps: int = 1, max_log: int = 64):
        """Block-angular solver or batch: A0, B0 (None without a dense part), y.  Banded solver:
        A0 is row_start [P*M] int32 and B0 is vals0 [P*M, w]."""
        torch = _torch()
        td = _torch_dtype(solver.qdtype)
        self.solver, self.P = solver, int(getattr(solver, "P", 1))
        self.max_log = int(max_log)
        h = _c_vp()
        if isinstance(solver, BandedSolver):
            _check(lib().qrk_lm_create_banded(solver.handle, _dev_ptr(A0, torch.int32, "row_start"),
                                              _dev_ptr(B0, td, "vals0"), _dev_ptr(y, td, "y"), float(c),
                                              int(sweeps), self.max_log, ctypes.byref(h)), "qrk_lm_create_banded")
        else:
            _check(lib().qrk_lm_create_blockangular(solver.handle, _dev_ptr(A0, td, "A0"),
                                                    _dev_ptr(B0, td, "B0") if B0 is not None else None,
                                                    _dev_ptr(y, td, "y"), float(c), int(sweeps), self.max_log,
                                                    ctypes.byref(h)), "qrk_lm_create_blockangular")
        self._lm = h
        self._keep = (A0, B0, y)
        self.N = solver.N

    def __del__(self):
        h, self._lm = getattr(self, "_lm", None), None
        if h is not None and _LIB is not None:
            _LIB.qrk_lm_destroy(h)

    def reset(self, x0, lam0, stream=None):
        torch = _torch()
        self._x0 = x0.to(torch.float64).contiguous()
        self._lam0 = lam0.to(torch.float64).contiguous()
        _check(lib().qrk_lm_reset(self._lm, _dev_ptr(self._x0, torch.float64, "x0", self.N),
                                  _dev_ptr(self._lam0, torch.float64, "lam0", self.P), _stream_ptr(stream)),
               "qrk_lm_reset")

    def run(self, iters: int, graph: bool = False, stream=None):
        _check(lib().qrk_lm_run(self._lm, int(iters), int(bool(graph)), _stream_ptr(stream)), "qrk_lm_run")

    def get(self, stream=None):
        """(x [N], lam [P], log [max_log, P, 4] = F, F_new, lam after, accepted; iterations run)."""
        torch = _torch()
        x = torch.empty(self.N, dtype=torch.float64, device="cuda")
        lam = torch.empty(self.P, dtype=torch.float64, device="cuda")
        log = torch.empty((max(self.max_log, 1), self.P, 4), dtype=torch.float64, device="cuda")
        it = _c_i32(0)
        _check(lib().qrk_lm_get(self._lm, _dev_ptr(x, torch.float64, "x"), _dev_ptr(lam, torch.float64, "lam"),
                                _dev_ptr(log, torch.float64, "log"), ctypes.byref(it), _stream_ptr(stream)),
               "qrk_lm_get")
        return x, lam, log[:self.max_log], int(it.value)


def check_bf16_split(x, stream=None):
    """(hi, lo) of every float32 element of x by the dense-part kernels' BF16x3 split
    (qrk_check_bf16_split)."""
    torch = _torch()
    n = x.numel()
    hi = torch.empty_like(x)
    lo = torch.empty_like(x)
    _check(lib().qrk_check_bf16_split(_dev_ptr(x, torch.float32, "x"), _dev_ptr(hi, torch.float32, "hi"),
                                      _dev_ptr(lo, torch.float32, "lo"), n, _stream_ptr(stream)),
           "qrk_check_bf16_split")
    return hi, lo


def check_bf16x3_product(A, B, stream=None):
    """C = A B (A 16 x k, B k x 16, float32) by the dense-part kernels' BF16x3 matrix-core
    product (qrk_check_bf16x3_product)."""
    torch = _torch()
    k = A.shape[1]
    if A.shape != (16, k) or B.shape != (k, 16):
        raise ValueError("A must be 16 x k and B k x 16")
    C = torch.empty((16, 16), dtype=torch.float32, device=A.device)
    _check(lib().qrk_check_bf16x3_product(_dev_ptr(A, torch.float32, "A"), _dev_ptr(B, torch.float32, "B"),
                                          _dev_ptr(C, torch.float32, "C"), k, _stream_ptr(stream)),
           "qrk_check_bf16x3_product")
    return C


def solve_banded_noalloc(row_start, vals, b, d, lam: float, N: int, sweeps: int = 0, p=None, status=None,
                         stream=None):
    """The banded step of factor_banded + solve in one call that allocates no device memory
    (qrk_solve_banded_noalloc).  row_start [P, M] int32, vals [P, M, w], b [P, M], d [P, N]
    float64; p [P * N] float64 and status [1] int32 may be given (device tensors)."""
    torch = _torch()
    P, M = int(row_start.shape[0]), int(row_start.shape[1])
    w = int(vals.shape[-1])
    qd = QRK_F32 if vals.dtype == torch.float32 else QRK_F64
    td = _torch_dtype(qd)
    if p is None:
        p = torch.empty(P * int(N), dtype=torch.float64, device=vals.device)
    _check(lib().qrk_solve_banded_noalloc(
        P, M, int(N), w, qd, _dev_ptr(row_start, torch.int32, "row_start", P * M), _dev_ptr(vals, td, "vals", P * M * w),
        _dev_ptr(b, td, "b", P * M), _dev_ptr(d, torch.float64, "d", P * int(N)), float(lam),
        _dev_ptr(p, torch.float64, "p", P * int(N)), int(sweeps),
        _dev_ptr(status, torch.int32, "status", 1) if status is not None else None, _stream_ptr(stream)),
        "qrk_solve_banded_noalloc")
    return p


def set_tune_cache(path):
    """Autotuner cache file for the process (None: none); loads the choices it holds."""
    _check(lib().qrk_tune_cache_file(None if path is None else str(path).encode()), "qrk_tune_cache_file")


def tune_choice(solver) -> dict:
    """The launch-shape knobs a block-angular solver or batch uses."""
    ls, lq, rs = _c_dbl(0.0), _c_i32(0), _c_dbl(0.0)
    _check(lib().qrk_tune_get(solver.handle, ctypes.byref(ls), ctypes.byref(lq), ctypes.byref(rs)), "qrk_tune_get")
    return {"leaf_scale": float(ls.value), "leaf_queue": int(lq.value), "refine_scale": float(rs.value)}


def _csr(row_ptr, col_idx):
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    ci = np.ascontiguousarray(np.asarray(col_idx, dtype=np.int32))
    return rp, ci


def discover_blockangular(row_ptr, col_idx, N: int, dense_cols) -> dict:
    """Row and column permutations that bring the sparse pattern (CSR row_ptr, col_idx; N
    columns) to block-angular form with the given dense columns last (Section 4.3,
    qrk_discover_blockangular): dict(row_perm, col_perm, ncol, row_off, K), host numpy arrays."""
    rp, ci = _csr(row_ptr, col_idx)
    M = int(rp.shape[0] - 1)
    dc = np.ascontiguousarray(np.asarray(dense_cols, dtype=np.int32))
    row_perm = np.empty(M, dtype=np.int64)
    col_perm = np.empty(int(N), dtype=np.int32)
    ncol = np.empty(int(N), dtype=np.int32)
    row_off = np.empty(M + 1, dtype=np.int64)
    K = _c_i32(0)
    _check(lib().qrk_discover_blockangular(M, int(N), rp.ctypes.data_as(_c_i64p), ci.ctypes.data_as(_c_i32p),
                                           int(dc.shape[0]), dc.ctypes.data_as(_c_i32p),
                                           row_perm.ctypes.data_as(_c_i64p), col_perm.ctypes.data_as(_c_i32p),
                                           ncol.ctypes.data_as(_c_i32p), row_off.ctypes.data_as(_c_i64p),
                                           ctypes.byref(K)), "qrk_discover_blockangular")
    k = int(K.value)
    return dict(row_perm=row_perm, col_perm=col_perm, ncol=ncol[:k].copy(), row_off=row_off[:k + 1].copy(), K=k)


def discover_banded(row_ptr, col_idx, N: int) -> dict:
    """The row order that makes the sparse pattern banded (rows by first column, Section 4.3,
    qrk_discover_banded): dict(row_perm, row_start, w), host numpy arrays."""
    rp, ci = _csr(row_ptr, col_idx)
    M = int(rp.shape[0] - 1)
    row_perm = np.empty(M, dtype=np.int64)
    row_start = np.empty(M, dtype=np.int32)
    w = _c_i32(0)
    _check(lib().qrk_discover_banded(M, int(N), rp.ctypes.data_as(_c_i64p), ci.ctypes.data_as(_c_i32p),
                                     row_perm.ctypes.data_as(_c_i64p), row_start.ctypes.data_as(_c_i32p),
                                     ctypes.byref(w)), "qrk_discover_banded")
    return dict(row_perm=row_perm, row_start=row_start, w=int(w.value))
