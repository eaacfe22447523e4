"""Seeded synthetic instances for the structured-QR Levenberg-Marquardt step.

This module only *draws* problem instances; it contains none of the solver's
arithmetic.  Both the CPU oracle (``oracle/``) and the GPU path (through its
Python binding) consume the same instances, so the two sides see bit-identical
inputs.

Problem (Section 1, Eqs. 1-2 of the paper): given J, b, a positive diagonal D
and a damping lambda >= 0, the LM step p solves
    min_p || [J; sqrt(lambda) D] p - [b; 0] ||_2 .

Block-angular J (Section 4.2, horizontal concatenation of a block-diagonal part
and a dense part, Section 4.1):
    J = [ blkdiag(A_1, ..., A_K) | B ],
block i owns the rows [row_off[i], row_off[i+1]) of J; every block has the same
column count ``n`` (1..8); A is stored as one M x n row-major array (row r of A
belongs to the block that owns row r), B as M x nB row-major, b as an M-vector.
The unknowns are ordered p = [p_1, ..., p_K, p_B]; N = K*n + nB.

D = diag(d) with d_j = ||J e_j||_2 (Section 5.2, Backtrack LM: D = diag(J^T J)^(1/2)),
and d_j = 1 for an all-zero column.  d is part of the instance definition: it
is computed here once, in float64, from the values of J as stored.

Banded J (Section 4.4 problem class): row i has w consecutive nonzeros at
columns s_i .. s_i+w-1 with s_i = min(floor(i/2), N-w) for the 2N x N shape.

Draw order for block-angular instances: A, then B, then b, then the column
scale permutation, then the target p* (adjoint workloads).  Generator:
numpy PCG64 seeded with the given integer.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import Optional

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class BlockAngular:
    """One block-angular LM-step instance (arrays are host numpy arrays)."""

    row_off: np.ndarray  # int64 [K+1]
    n: int               # columns per block
    A: np.ndarray        # [M, n]   dtype
    B: np.ndarray        # [M, nB]  dtype
    b: np.ndarray        # [M]      dtype
    d: np.ndarray        # [N]      float64, > 0
    lam: float
    dtype: np.dtype

    @property
    def K(self) -> int:
        return int(self.row_off.shape[0] - 1)

    @property
    def M(self) -> int:
        return int(self.row_off[-1])

    @property
    def nB(self) -> int:
        return int(self.B.shape[1])

    @property
    def N(self) -> int:
        return self.K * self.n + self.nB

    def block_of_row(self) -> np.ndarray:
        """Block index of every row (int64 [M])."""
        counts = np.diff(self.row_off)
        return np.repeat(np.arange(self.K, dtype=np.int64), counts)

    def sha256(self) -> str:
        h = hashlib.sha256()
        for arr in (self.row_off, self.A, self.B, self.b, self.d):
            h.update(np.ascontiguousarray(arr).tobytes())
        h.update(np.float64(self.lam).tobytes())
        return h.hexdigest()

    def with_lambda(self, lam: float) -> "BlockAngular":
        return dataclasses.replace(self, lam=float(lam))

    def as_dtype(self, dtype) -> "BlockAngular":
        """The same instance stored in another dtype (d is recomputed from the
        stored values so that it is exactly the column norms of the stored J)."""
        dtype = np.dtype(dtype)
        A = self.A.astype(dtype)
        B = self.B.astype(dtype)
        b = self.b.astype(dtype)
        d = column_norms_blockangular(self.row_off, self.n, A, B)
        return BlockAngular(self.row_off.copy(), self.n, A, B, b, d, self.lam, dtype)

    def sub_blocks(self, k0: int, k1: int) -> "BlockAngular":
        """Blocks k0..k1-1 with their rows of B and b (its own d)."""
        r0, r1 = int(self.row_off[k0]), int(self.row_off[k1])
        row_off = self.row_off[k0:k1 + 1] - r0
        A = self.A[r0:r1].copy()
        B = self.B[r0:r1].copy()
        b = self.b[r0:r1].copy()
        d = column_norms_blockangular(row_off, self.n, A, B)
        return BlockAngular(row_off, self.n, A, B, b, d, self.lam, self.dtype)


def column_norms_blockangular(row_off, n, A, B) -> np.ndarray:
    """d_j = ||J e_j||_2 in float64 from the stored values; 1 where the column is zero."""
    K = row_off.shape[0] - 1
    A64 = A.astype(np.float64)
    B64 = B.astype(np.float64)
    counts = np.diff(row_off)
    blk = np.repeat(np.arange(K, dtype=np.int64), counts)
    dA = np.zeros((K, n), dtype=np.float64)
    np.add.at(dA, blk, A64 * A64)
    dB = (B64 * B64).sum(axis=0) if B64.shape[1] else np.zeros(0)
    d = np.sqrt(np.concatenate([dA.reshape(-1), dB]))
    d[d == 0.0] = 1.0
    return d


def _column_scales(rng: np.random.Generator, N: int, k: float) -> np.ndarray:
    """s = 10^(k t), t = linspace(0, 1, N) under a seeded permutation."""
    t = np.linspace(0.0, 1.0, N)
    perm = rng.permutation(N)
    return 10.0 ** (k * t[perm])


def make_blockangular(seed: int, K: int, m, n: int, nB: int, lam: float,
                      dtype=np.float64, scale_k: Optional[float] = None) -> BlockAngular:
    """Gaussian block-angular instance.

    m: an int (every block has m rows) or an int array of length K.
    scale_k: if given, all N columns are multiplied by 10^(k t) with t a seeded
    permutation of linspace(0, 1, N) (so cond(J) is about 10^k).
    The instance is defined by its values rounded to ``dtype``.
    """
    rng = _rng(seed)
    m_arr = np.full(K, int(m), dtype=np.int64) if np.isscalar(m) else np.asarray(m, np.int64)
    assert m_arr.shape == (K,)
    row_off = np.zeros(K + 1, dtype=np.int64)
    np.cumsum(m_arr, out=row_off[1:])
    M = int(row_off[-1])
    A = rng.standard_normal((M, n))
    B = rng.standard_normal((M, nB))
    b = rng.standard_normal(M)
    if scale_k is not None:
        s = _column_scales(rng, K * n + nB, float(scale_k))
        blk = np.repeat(np.arange(K), m_arr)
        sA = s[:K * n].reshape(K, n)
        A *= sA[blk]
        B *= s[K * n:][None, :]
    dtype = np.dtype(dtype)
    A = A.astype(dtype)
    B = B.astype(dtype)
    b = b.astype(dtype)
    d = column_norms_blockangular(row_off, n, A, B)
    return BlockAngular(row_off, n, A, B, b, d, float(lam), dtype)


@dataclasses.dataclass
class BlockAngularNcol:
    """Block-angular instance whose block i has its own column count ncol[i]."""

    row_off: np.ndarray  # int64 [K+1]
    ncol: np.ndarray     # int32 [K]
    A: np.ndarray        # [sum_i m_i ncol_i] dtype: block i's rows, ncol_i values each
    B: np.ndarray        # [M, nB] dtype
    b: np.ndarray        # [M]     dtype
    d: np.ndarray        # [N]     float64, > 0 (block i's unknowns, then the dense part's)
    lam: float
    dtype: np.dtype

    @property
    def K(self) -> int:
        return int(self.row_off.shape[0] - 1)

    @property
    def M(self) -> int:
        return int(self.row_off[-1])

    @property
    def nB(self) -> int:
        return int(self.B.shape[1])

    @property
    def N(self) -> int:
        return int(self.ncol.sum()) + self.nB

    def a_off(self) -> np.ndarray:
        """First value of block i in A (int64 [K+1])."""
        out = np.zeros(self.K + 1, dtype=np.int64)
        np.cumsum(np.diff(self.row_off) * self.ncol, out=out[1:])
        return out

    def p_off(self) -> np.ndarray:
        """First unknown of block i (int64 [K+1])."""
        out = np.zeros(self.K + 1, dtype=np.int64)
        np.cumsum(self.ncol, out=out[1:])
        return out


def make_blockangular_ncol(seed: int, K: int, m, ncol, nB: int, lam: float,
                           dtype=np.float64) -> BlockAngularNcol:
    """Gaussian block-angular instance with per-block column counts (m, ncol: ints or int
    arrays of length K); d is the column norms of the stored values (1 for a zero column)."""
    rng = _rng(seed)
    m_arr = np.full(K, int(m), dtype=np.int64) if np.isscalar(m) else np.asarray(m, np.int64)
    n_arr = np.full(K, int(ncol), dtype=np.int32) if np.isscalar(ncol) else np.asarray(ncol, np.int32)
    assert m_arr.shape == (K,) and n_arr.shape == (K,)
    row_off = np.zeros(K + 1, dtype=np.int64)
    np.cumsum(m_arr, out=row_off[1:])
    M = int(row_off[-1])
    dtype = np.dtype(dtype)
    A = rng.standard_normal(int((m_arr * n_arr).sum())).astype(dtype)
    B = rng.standard_normal((M, nB)).astype(dtype)
    b = rng.standard_normal(M).astype(dtype)
    dA = []
    pos = 0
    for i in range(K):
        blk = A[pos:pos + m_arr[i] * n_arr[i]].astype(np.float64).reshape(m_arr[i], n_arr[i])
        dA.append(np.sqrt((blk * blk).sum(axis=0)))
        pos += m_arr[i] * n_arr[i]
    B64 = B.astype(np.float64)
    d = np.concatenate(dA + [np.sqrt((B64 * B64).sum(axis=0))])
    d[d == 0.0] = 1.0
    return BlockAngularNcol(row_off, n_arr, A, B, b, d, float(lam), dtype)


@dataclasses.dataclass
class BlockAngularCam:
    """Block-angular instance whose coupled columns are camera blocks (the bundle-adjustment
    Jacobian of the experiments in Section 6.2, a horizontal concatenation as in Section 4.2:
    point blocks of n columns, then ncam cameras of cw parameters each).

    Row r of J touches its point block and at most one camera: its coupled entries are
    Bv[r, :] in the columns cam[r]*cw .. cam[r]*cw + cw - 1 of B and zero elsewhere; a row with
    cam[r] outside [0, ncam) touches no camera (its Bv row is ignored).  The unknowns are
    p = [p_1, ..., p_K, p_cam_0, ..., p_cam_{ncam-1}]; N = K*n + ncam*cw.
    """

    row_off: np.ndarray  # int64 [K+1]
    n: int               # columns per point block
    A: np.ndarray        # [M, n]  dtype
    Bv: np.ndarray       # [M, cw] dtype: each row's values in its camera's columns
    cam: np.ndarray      # int32 [M]: camera of each row
    ncam: int
    b: np.ndarray        # [M] dtype
    d: np.ndarray        # [N] float64, > 0
    lam: float
    dtype: np.dtype

    @property
    def K(self) -> int:
        return int(self.row_off.shape[0] - 1)

    @property
    def M(self) -> int:
        return int(self.row_off[-1])

    @property
    def cw(self) -> int:
        return int(self.Bv.shape[1])

    @property
    def nB(self) -> int:
        return self.ncam * self.cw

    @property
    def N(self) -> int:
        return self.K * self.n + self.nB

    def with_lambda(self, lam: float) -> "BlockAngularCam":
        return dataclasses.replace(self, lam=float(lam))


def column_norms_cam(row_off, n, A, Bv, cam, ncam) -> np.ndarray:
    """d_j = ||J e_j||_2 of a camera-block instance in float64; 1 where the column is zero."""
    K = row_off.shape[0] - 1
    cw = Bv.shape[1]
    A64 = A.astype(np.float64)
    B64 = Bv.astype(np.float64)
    blk = np.repeat(np.arange(K, dtype=np.int64), np.diff(row_off))
    dA = np.zeros((K, n), dtype=np.float64)
    np.add.at(dA, blk, A64 * A64)
    dC = np.zeros((ncam, cw), dtype=np.float64)
    seen = (cam >= 0) & (cam < ncam)
    np.add.at(dC, cam[seen].astype(np.int64), B64[seen] * B64[seen])
    d = np.sqrt(np.concatenate([dA.reshape(-1), dC.reshape(-1)]))
    d[d == 0.0] = 1.0
    return d


def make_blockangular_cam(seed: int, K: int, obs, ncam: int, cw: int = 9, n: int = 3, lam: float = 1e-2,
                          prior_rows: int = 0, dtype=np.float64) -> BlockAngularCam:
    """Gaussian camera-block instance shaped like bundle adjustment: point i is seen by obs_i
    distinct cameras (obs: an int or an int array of length K, each <= ncam), drawn uniformly;
    each observation gives two rows (its x and y residuals) on that camera; prior_rows extra
    rows per point touch no camera (cam = -1, their Bv rows random and ignored).
    Draw order: observations' cameras, A, Bv, b."""
    rng = _rng(seed)
    o_arr = np.full(K, int(obs), dtype=np.int64) if np.isscalar(obs) else np.asarray(obs, np.int64)
    assert o_arr.shape == (K,) and int(o_arr.max(initial=0)) <= ncam
    m_arr = 2 * o_arr + int(prior_rows)
    row_off = np.zeros(K + 1, dtype=np.int64)
    np.cumsum(m_arr, out=row_off[1:])
    M = int(row_off[-1])
    cam = np.empty(M, dtype=np.int32)
    for i in range(K):
        cams = rng.choice(ncam, size=int(o_arr[i]), replace=False)
        r0 = int(row_off[i])
        cam[r0:r0 + 2 * o_arr[i]] = np.repeat(cams, 2)
        cam[r0 + 2 * o_arr[i]:int(row_off[i + 1])] = -1
    dtype = np.dtype(dtype)
    A = rng.standard_normal((M, n)).astype(dtype)
    Bv = rng.standard_normal((M, cw)).astype(dtype)
    b = rng.standard_normal(M).astype(dtype)
    d = column_norms_cam(row_off, n, A, Bv, cam, ncam)
    return BlockAngularCam(row_off, n, A, Bv, cam, int(ncam), b, d, float(lam), dtype)


# ---------------------------------------------------------------------------
# Named workloads (shapes of the measured configurations)
# ---------------------------------------------------------------------------

def tiny_blockangular(seed: int = 0, dtype=np.float64, lam: float = 1e-2) -> BlockAngular:
    """100 blocks of 8x3, dense part 800x24, entries N(0,1), lambda = 1e-2."""
    return make_blockangular(seed, K=100, m=8, n=3, nB=24, lam=lam, dtype=dtype)


def scale_blockangular(seed: int = 100, lam: float = 1e-2, dtype=np.float32,
                       K: int = 50_000, m: int = 12, nB: int = 90,
                       scale_k: Optional[float] = 3.0) -> BlockAngular:
    """50,000 blocks of 12x3, dense part 600,000x90, column scales 10^(3t)."""
    return make_blockangular(seed, K=K, m=m, n=3, nB=nB, lam=lam, dtype=dtype, scale_k=scale_k)


def precision_blockangular(seed: int, k: float, dtype=np.float32, lam: float = 1e-2) -> BlockAngular:
    """Tiny-workload shapes with column scales 10^(k t), k in {3, 4, 5}."""
    return make_blockangular(seed, K=100, m=8, n=3, nB=24, lam=lam, dtype=dtype, scale_k=k)


def precision_rotated(seed: int, k: float, lam: float = 1e-4, dtype=np.float32) -> BlockAngular:
    """Tiny-workload shapes with B <- B diag(10^(k t_B)) H: t_B a seeded permutation of
    linspace(0, 1, 24), H a Haar-distributed orthogonal 24 x 24 matrix (QR of a Gaussian with the
    signs of R's diagonal folded into Q), so the spread of scales is rotated across B's columns
    and neither column scaling nor a small damping removes it; d is the column norms."""
    inst = make_blockangular(seed, K=100, m=8, n=3, nB=24, lam=lam, dtype=np.float64)
    rng = _rng(seed + 7919)
    nB = inst.nB
    s = _column_scales(rng, nB, float(k))
    G = rng.standard_normal((nB, nB))
    Q, R = np.linalg.qr(G)
    H = Q * np.sign(np.diag(R))[None, :]
    B = (inst.B * s[None, :]) @ H
    dtype = np.dtype(dtype)
    A = inst.A.astype(dtype)
    B = B.astype(dtype)
    b = inst.b.astype(dtype)
    d = column_norms_blockangular(inst.row_off, inst.n, A, B)
    return BlockAngular(inst.row_off, inst.n, A, B, b, d, float(lam), dtype)


def adjoint_blockangular(seed: int = 500, dtype=np.float32, K: int = 10_000, nB: int = 60,
                         lam: float = 1e-2):
    """10,000 blocks of 12x3, dense part 120,000x60, lambda = 1e-2; also returns p* ~ N(0,1)."""
    rng = _rng(seed)
    M = K * 12
    A = rng.standard_normal((M, 3))
    B = rng.standard_normal((M, nB))
    b = rng.standard_normal(M)
    p_star = rng.standard_normal(K * 3 + nB)
    row_off = np.arange(0, M + 1, 12, dtype=np.int64)
    dtype = np.dtype(dtype)
    A, B, b = A.astype(dtype), B.astype(dtype), b.astype(dtype)
    d = column_norms_blockangular(row_off, 3, A, B)
    return BlockAngular(row_off, 3, A, B, b, d, float(lam), dtype), p_star


def ragged_batch(seed: int = 200, P: int = 512, kmin: int = 500, kmax: int = 8000,
                 mmin: int = 4, mmax: int = 40, nB_choices=(6, 30, 90),
                 dtype=np.float32, lam: float = 1e-2):
    """P independent block-angular problems: K_p ~ U{kmin..kmax}, m_i ~ U{mmin, mmin+2, .., mmax},
    3 columns per block, nB_p uniform over nB_choices, N(0,1) entries."""
    rng = _rng(seed)
    out = []
    m_vals = np.arange(mmin, mmax + 1, 2, dtype=np.int64)
    for p in range(P):
        K = int(rng.integers(kmin, kmax + 1))
        m = m_vals[rng.integers(0, m_vals.shape[0], size=K)]
        nB = int(nB_choices[int(rng.integers(0, len(nB_choices)))])
        sub_seed = int(rng.integers(0, 2**63 - 1))
        out.append(make_blockangular(sub_seed, K=K, m=m, n=3, nB=nB, lam=lam, dtype=dtype))
    return out


def stack_rows(insts) -> BlockAngular:
    """The instance whose least-squares rows are those of all `insts` (same K, n, n_B, d), block i's
    rows of each instance in turn; the damping (lam) is the first instance's.  Input construction
    only: the row order of a least-squares problem does not change its solution."""
    first = insts[0]
    K, n, nB = first.K, first.n, first.nB
    assert all(i.K == K and i.n == n and i.nB == nB for i in insts)
    row_off = np.zeros(K + 1, np.int64)
    rows = []
    for k in range(K):
        for inst in insts:
            rows.append((inst, int(inst.row_off[k]), int(inst.row_off[k + 1])))
        row_off[k + 1] = row_off[k] + sum(int(i.row_off[k + 1] - i.row_off[k]) for i in insts)
    A = np.concatenate([inst.A[a:e] for inst, a, e in rows] or [first.A[:0]], axis=0)
    B = np.concatenate([inst.B[a:e] for inst, a, e in rows] or [first.B[:0]], axis=0)
    b = np.concatenate([inst.b[a:e] for inst, a, e in rows] or [first.b[:0]], axis=0)
    return BlockAngular(row_off, n, np.ascontiguousarray(A), np.ascontiguousarray(B), np.ascontiguousarray(b),
                        first.d.copy(), first.lam, first.dtype)


def stack_batch(insts):
    """Stack block-angular problems (same n and dtype) into the batched layout: K [P], nB [P],
    global row offsets [sum K + 1], A [M_tot, n], B flat (each problem's M_p x nB_p rows packed
    with row stride nB_p), b [M_tot], d [sum N_p] and lam [P].  Pure data layout."""
    n = insts[0].n
    K = np.array([i.K for i in insts], dtype=np.int32)
    nB = np.array([i.nB for i in insts], dtype=np.int32)
    row_off = [np.zeros(1, dtype=np.int64)]
    base = 0
    for i in insts:
        row_off.append(i.row_off[1:] + base)
        base += i.M
    B = [np.ascontiguousarray(i.B[:, :i.nB]).reshape(-1) for i in insts]
    return dict(n=n, K=K, nB=nB, row_off=np.concatenate(row_off),
                A=np.concatenate([i.A for i in insts], axis=0),
                B=np.concatenate(B) if B else np.zeros(0, dtype=insts[0].A.dtype),
                b=np.concatenate([i.b for i in insts]), d=np.concatenate([i.d for i in insts]),
                lam=np.array([i.lam for i in insts], dtype=np.float64))


@dataclasses.dataclass
class Banded:
    """Banded J: row i holds w values at columns row_start[i] .. row_start[i]+w-1."""

    N: int
    w: int
    row_start: np.ndarray  # int32 [M], nondecreasing, <= N - w
    vals: np.ndarray       # [M, w] dtype
    b: np.ndarray          # [M]
    d: np.ndarray          # [N] float64
    lam: float
    dtype: np.dtype

    @property
    def M(self) -> int:
        return int(self.row_start.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        for arr in (self.row_start, self.vals, self.b, self.d):
            h.update(np.ascontiguousarray(arr).tobytes())
        h.update(np.float64(self.lam).tobytes())
        return h.hexdigest()


def column_norms_banded(N, w, row_start, vals) -> np.ndarray:
    v64 = vals.astype(np.float64)
    d2 = np.zeros(N, dtype=np.float64)
    cols = row_start.astype(np.int64)[:, None] + np.arange(w)[None, :]
    np.add.at(d2, cols.reshape(-1), (v64 * v64).reshape(-1))
    d = np.sqrt(d2)
    d[d == 0.0] = 1.0
    return d


def make_banded(seed: int, N: int = 2048, w: int = 12, rows_per_col: int = 2,
                lam: float = 1e-2, dtype=np.float32) -> Banded:
    """M = rows_per_col*N rows, w nonzeros per row at s_i = min(floor(i/rows_per_col), N-w)."""
    rng = _rng(seed)
    M = rows_per_col * N
    row_start = np.minimum(np.arange(M) // rows_per_col, N - w).astype(np.int32)
    vals = rng.standard_normal((M, w))
    b = rng.standard_normal(M)
    dtype = np.dtype(dtype)
    vals = vals.astype(dtype)
    b = b.astype(dtype)
    d = column_norms_banded(N, w, row_start, vals)
    return Banded(N, w, row_start, vals, b, d, float(lam), dtype)


def banded_batch(seed: int = 300, P: int = 2048, N: int = 2048, w: int = 12,
                 dtype=np.float32, lam: float = 1e-2):
    rng = _rng(seed)
    seeds = rng.integers(0, 2**63 - 1, size=P)
    return [make_banded(int(s), N=N, w=w, lam=lam, dtype=dtype) for s in seeds]


def lm_blockangular(seed: int = 310, K: int = 200, m=12, n: int = 3, nB: int = 30, c: float = 0.1,
                    noise: float = 0.01, x_noise: float = 0.1, dtype=np.float32):
    """Synthetic LM workload on a block-angular J0: x_true ~ N(0,1), y = J0 (x_true + c x_true^3)
    + noise N(0,1), start x0 = x_true + x_noise N(0,1).  Returns (inst0, y, x0, x_true); inst0
    holds A0, B0 (its b, d, lam are unused)."""
    inst0 = make_blockangular(seed, K=K, m=m, n=n, nB=nB, lam=0.0, dtype=dtype)
    rng = _rng(seed + 1)
    x_true = rng.standard_normal(inst0.N)
    u = x_true + c * x_true ** 3
    blk = np.repeat(np.arange(K), np.diff(inst0.row_off))
    ub = u[:K * n].reshape(K, n)
    y = (inst0.A.astype(np.float64) * ub[blk]).sum(axis=1)
    if nB:
        y = y + inst0.B.astype(np.float64) @ u[K * n:]
    y = (y + noise * rng.standard_normal(inst0.M)).astype(dtype)
    x0 = x_true + x_noise * rng.standard_normal(inst0.N)
    return inst0, y, x0, x_true


def lm_banded(seed: int = 320, N: int = 2048, w: int = 12, c: float = 0.1, noise: float = 0.01,
              x_noise: float = 0.1, dtype=np.float32):
    """The same synthetic LM workload on a banded J0 (make_banded's pattern)."""
    inst0 = make_banded(seed, N=N, w=w, lam=0.0, dtype=dtype)
    rng = _rng(seed + 1)
    x_true = rng.standard_normal(N)
    u = x_true + c * x_true ** 3
    cols = inst0.row_start.astype(np.int64)[:, None] + np.arange(w)[None, :]
    y = (inst0.vals.astype(np.float64) * u[cols]).sum(axis=1)
    y = (y + noise * rng.standard_normal(inst0.M)).astype(dtype)
    x0 = x_true + x_noise * rng.standard_normal(N)
    return inst0, y, x0, x_true
