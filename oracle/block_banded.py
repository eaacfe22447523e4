"""Block-banded QR with the compressed WY form per step (paper Section 4.4, Eq. blockBandedYTY).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The problem is the banded step of oracle.banded: row i of J holds w values at columns
s_i .. s_i + w - 1 (s_i nondecreasing), the damping rows sqrt(lam) D sit under J, and the
right-hand side b rides along as one more column.  Section 4.4 factors the banded matrix as a
sequence of small dense steps, each with Householder vectors local to the rows that the step
touches, applied in the compressed WY form of Section 2,

    Q_k = I + Y_k T_k Y_k^T,    Q_k^T A_k = A_k + Y_k (T_k^T (Y_k^T A_k)),

(Y_k lower trapezoidal, T_k upper triangular), and A' = Q_{K-1}^T ... Q_0^T A.

Columns are taken in blocks of r.  A row whose first nonzero lies in block k ends in block k or
k+1 (w <= r + 1).  Step k works on the dense block A_k over the columns of blocks k and k+1 and
the right-hand side, whose rows are
  * the r rows carried from step k-1: a triangle in block k's columns (for k = 0 the damping
    rows of block 0),
  * the damping rows of block k+1 (zero except sqrt(lam) d_j on column j),
  * the rows of J whose first nonzero lies in block k,
and factors its first 2r columns (r for the last block).  The Householder vectors of a step are
thus local to the carried rows, the next block's damping rows and the block's own rows (the
paper's vectors of length n_k + n_{k+1}).  Afterwards the first r rows of Q_k^T A_k are R's
rows for block k (columns of blocks k and k+1) with their entries of c = Q^T b, the next r rows
are the triangle carried into step k+1, and the rows below are zero but for the right-hand side,
whose squares add to the squared residual norm.

Reading taken where Section 4.4 is silent: how rows left over after a step reach the next one.
Factoring two column blocks per step keeps the carried rows at r (a triangle) instead of letting
them grow by the block's row count at every step.

R is unique up to row signs, so it equals the R of any other QR of [J; sqrt(lam) D] (pinned
against oracle.banded / oracle.dense and LAPACK in tests/test_oracle_block_banded.py); its upper
bandwidth is w - 1 in exact arithmetic.
"""
from __future__ import annotations

import numpy as np

from . import dense


def compressed_wy(A: np.ndarray, ncols: int):
    """Householder QR of the first `ncols` columns of A (textbook reflectors, Section 2),
    returned as the compressed WY factors of Q = H_0 H_1 ... = I + Y T Y^T.

    Returns (Y [m, ncols], T [ncols, ncols] upper triangular).  With H_j = I - tau_j v_j v_j^T,
    T is built column by column: T_jj = -tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] (Y[:, 0:j]^T v_j),
    which is the sign of the paper's I + Y T Y^T (LAPACK's I - V T V^T with T negated)."""
    W = np.array(A, dtype=np.float64, copy=True)
    m = W.shape[0]
    k = min(m, ncols)
    Y = np.zeros((m, ncols))
    T = np.zeros((ncols, ncols))
    for j in range(k):
        v, tau, beta = dense.householder_vector(W[j:, j])
        y = np.zeros(m)
        y[j:] = v
        if tau != 0.0:
            W[j:, j:] -= tau * np.outer(v, v @ W[j:, j:])
        W[j, j] = beta
        W[j + 1:, j] = 0.0
        Y[:, j] = y
        T[j, j] = -tau
        if j:
            T[:j, j] = -tau * (T[:j, :j] @ (Y[:, :j].T @ y))
    return Y, T


def apply_wy_transposed(Y: np.ndarray, T: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Q^T A = A + Y (T^T (Y^T A)) for Q = I + Y T Y^T (the step of Eq. blockBandedYTY)."""
    return A + Y @ (T.T @ (Y.T @ A))


def factor(inst, r: int = 16):
    """Block-banded factorisation of [J | b; sqrt(lam) D | 0] of a banded instance (w <= r + 1).

    Returns dict(R [N, N] upper triangular (the rows of every step, entries outside the
    computed columns zero), c [N], resid (the residual norm), steps (the (Y, T) of each step))."""
    N, w, M = inst.N, inst.w, inst.M
    if w > r + 1:
        raise ValueError("block width r must be at least w - 1")
    s = np.asarray(inst.row_start, np.int64)
    vals = inst.vals.astype(np.float64)
    b = inst.b.astype(np.float64)
    dl = np.sqrt(inst.lam) * np.asarray(inst.d, np.float64)
    nblk = (N + r - 1) // r
    R = np.zeros((N, N))
    c = np.zeros(N)
    resid2 = 0.0
    steps = []
    # carried rows: r x (r + 1), columns of the current block and the right-hand side
    c0 = min(r, N)
    carry = np.zeros((r, r + 1))
    carry[np.arange(c0), np.arange(c0)] = dl[:c0]
    for k in range(nblk):
        lo = k * r
        nk = min(r, N - lo)                  # columns of block k
        nn = min(r, max(N - lo - r, 0))      # columns of block k+1
        width = nk + nn
        rows = []
        # the carried triangle (block k's columns) and the right-hand side
        top = np.zeros((r, width + 1))
        top[:, :nk] = carry[:, :nk]
        top[:, width] = carry[:, r]
        rows.append(top)
        # the damping rows of block k+1
        if nn:
            damp = np.zeros((nn, width + 1))
            damp[np.arange(nn), nk + np.arange(nn)] = dl[lo + r:lo + r + nn]
            rows.append(damp)
        # the rows of J whose first nonzero lies in block k
        mine = np.nonzero((s >= lo) & (s < lo + r))[0]
        if mine.size:
            new = np.zeros((mine.size, width + 1))
            for t, i in enumerate(mine):
                new[t, s[i] - lo + np.arange(w)] = vals[i]
                new[t, width] = b[i]
            rows.append(new)
        Ak = np.vstack(rows)
        Y, T = compressed_wy(Ak, width)
        Ak = apply_wy_transposed(Y, T, Ak)
        steps.append((Y, T))
        R[lo:lo + nk, lo:lo + width] = np.triu(Ak[:nk, :width])
        c[lo:lo + nk] = Ak[:nk, width]
        carry = np.zeros((r, r + 1))
        if nn:
            carry[:nn, :nn] = np.triu(Ak[nk:nk + nn, nk:width])
            carry[:nn, r] = Ak[nk:nk + nn, width]
        resid2 += float(np.sum(Ak[nk + nn:, width] ** 2))
    return dict(R=R, c=c, resid=float(np.sqrt(resid2)), steps=steps)


def solve(inst, r: int = 16):
    """p = R^{-1} c from the block-banded factor."""
    f = factor(inst, r)
    return dense.back_substitute(f["R"], f["c"]), f
