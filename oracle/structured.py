"""O2: structured block-angular oracle (LAPACK steps, float64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Section 4.2 (horizontal concatenation) with the block-diagonal part of
Section 4.1, applied to the damped system of Eq. 2 with the damping rows
permuted next to their blocks (Section 5.2, Backtrack LM: P_r [J; sqrt(lam) D]):

  augmented block i:  [A_i; sqrt(lam) D_i]  ((m_i+n) x n),
  its coupled rows:   [B_i; 0 | b_i; 0]      ((m_i+n) x (nB+1)),
  dense damping rows: [sqrt(lam) D_B | 0]    (nB x (nB+1)).

Step 1 (Section 4.1): Q_i R_i = qr([A_i; sqrt(lam) D_i]) for every block.
Step 2 (Section 4.2): Q_i^T applied to the coupled rows; the top n rows are the
        coupling rows S_i | c_i of R (the "Q_1^T A_2" block), the other m_i rows
        are the block's share of Q_1^perp^T A_2.
Step 3 (Section 4.2): Q'R' = qr(stack of all reduced rows and the dense damping
        rows), giving R_B | c_B and the residual norm.
Step 4: back-substitution through the structured R
        [[blkdiag(R_i), S], [0, R_B]] p = [c_blk; c_B].

numpy.linalg.qr (LAPACK geqrf/orgqr) serves as the QR step; numpy.matmul
serves as the product step.  No blocking or reordering beyond the section's
own order.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class BlockAngularFactor:
    R_blk: np.ndarray   # [K, n, n]   upper triangular per block
    S: np.ndarray       # [K, n, nB]  coupling rows
    c_blk: np.ndarray   # [K, n]      Q_i^T b_i, top n entries
    R_B: np.ndarray     # [nB, nB]
    c_B: np.ndarray     # [nB]
    resid: float        # || [J; sqrt(lam) D] p - [b; 0] ||


def factor_blockangular(inst) -> BlockAngularFactor:
    K, n, nB = inst.K, inst.n, inst.nB
    lam = float(inst.lam)
    sq = np.sqrt(lam)
    d = np.asarray(inst.d, np.float64)
    A = inst.A.astype(np.float64)
    C = np.concatenate([inst.B.astype(np.float64), inst.b.astype(np.float64)[:, None]], axis=1)
    m_all = np.diff(inst.row_off)
    R_blk = np.zeros((K, n, n))
    S = np.zeros((K, n, nB))
    c_blk = np.zeros((K, n))
    reduced = []
    for m in np.unique(m_all):
        idx = np.nonzero(m_all == m)[0]
        G = idx.shape[0]
        rows = inst.row_off[idx][:, None] + np.arange(m)[None, :]          # [G, m]
        Ai = A[rows]                                                       # [G, m, n]
        Di = np.zeros((G, n, n))
        di = d[(idx[:, None] * n + np.arange(n)[None, :])]                 # [G, n]
        Di[:, np.arange(n), np.arange(n)] = sq * di
        Aaug = np.concatenate([Ai, Di], axis=1)                            # [G, m+n, n]
        Caug = np.concatenate([C[rows], np.zeros((G, n, nB + 1))], axis=1)  # [G, m+n, nB+1]
        Q, Rr = np.linalg.qr(Aaug, mode="complete")                        # Q [G, m+n, m+n]
        QtC = np.matmul(np.swapaxes(Q, 1, 2), Caug)
        R_blk[idx] = Rr[:, :n, :]
        S[idx] = QtC[:, :n, :nB]
        c_blk[idx] = QtC[:, :n, nB]
        reduced.append(QtC[:, n:, :].reshape(-1, nB + 1))
    dB = np.zeros((nB, nB + 1))
    dB[np.arange(nB), np.arange(nB)] = sq * d[K * n:]
    stack = np.concatenate(reduced + [dB], axis=0)
    if nB == 0:
        return BlockAngularFactor(R_blk, S, c_blk, np.zeros((0, 0)), np.zeros(0),
                                  float(np.linalg.norm(stack[:, 0])))
    Rr = np.linalg.qr(stack, mode="r")
    if Rr.shape[0] < nB + 1:  # fewer stacked rows than columns: pad with zero rows
        Rr = np.vstack([Rr, np.zeros((nB + 1 - Rr.shape[0], nB + 1))])
    return BlockAngularFactor(R_blk, S, c_blk, Rr[:nB, :nB].copy(), Rr[:nB, nB].copy(),
                              float(abs(Rr[nB, nB])))


def factor_two_stage(inst, lam: float) -> BlockAngularFactor:
    """Moré's two-stage factor (Section 5.2, Eq. LMTwoStep): J = Q R first (the structured
    factor above with lambda = 0), then [R; sqrt(lam) D] = Q' R'.  The damping rows of each
    block go next to its R_i, so the second QR is the same horizontal-concatenation step on R's
    rows: block i is [R_i; sqrt(lam) D_i] with coupled rows [S_i | c_i; 0 | 0], and the dense
    part is the QR of the blocks' reduced rows stacked with the rows of [R_B | c_B], the
    residual row [0 | resid] and [sqrt(lam) D_B | 0]."""
    K, n, nB = inst.K, inst.n, inst.nB
    base = factor_blockangular(dataclasses.replace(inst, lam=0.0))
    sq = np.sqrt(float(lam))
    d = np.asarray(inst.d, np.float64)
    Di = np.zeros((K, n, n))
    Di[:, np.arange(n), np.arange(n)] = sq * d[:K * n].reshape(K, n)
    Aaug = np.concatenate([base.R_blk, Di], axis=1)                                   # [K, 2n, n]
    C = np.concatenate([base.S, base.c_blk[:, :, None]], axis=2)                      # [K, n, nB+1]
    Caug = np.concatenate([C, np.zeros((K, n, nB + 1))], axis=1)                      # [K, 2n, nB+1]
    Q, Rr = np.linalg.qr(Aaug, mode="complete")
    QtC = np.matmul(np.swapaxes(Q, 1, 2), Caug)
    R_blk, S, c_blk = Rr[:, :n, :], QtC[:, :n, :nB], QtC[:, :n, nB]
    reduced = QtC[:, n:, :].reshape(-1, nB + 1)
    RBc = np.zeros((nB + 1, nB + 1))
    RBc[:nB, :nB] = base.R_B
    RBc[:nB, nB] = base.c_B
    RBc[nB, nB] = base.resid
    dB = np.zeros((nB, nB + 1))
    dB[np.arange(nB), np.arange(nB)] = sq * d[K * n:]
    stack = np.concatenate([reduced, RBc, dB], axis=0)
    R2 = np.linalg.qr(stack, mode="r")
    return BlockAngularFactor(R_blk.copy(), S.copy(), c_blk.copy(), R2[:nB, :nB].copy(), R2[:nB, nB].copy(),
                              float(abs(R2[nB, nB])))


def factor_vcat(f1: BlockAngularFactor, f2: BlockAngularFactor) -> BlockAngularFactor:
    """Vertical concatenation (Section 4.5, Eq. vcatDecomp) of two factored problems over the same
    columns: [A1; A2] = blkdiag(Q1, Q2) [R1; R2].  [R1; R2] is not triangular; a row permutation P
    interleaves the two block by block, so that P [R1; R2] is block-angular again: block i is
    [R1_i; R2_i] (2n x n) with coupled rows [S1_i | c1_i; S2_i | c2_i], and the dense part holds
    the rows of [R1_B | c1_B] and [R2_B | c2_B] with their residual rows [0 | resid].  The same
    structured QR (Sections 4.1 and 4.2) then gives Q3 [R3; 0], the factor of [A1; A2]."""
    K, n = f1.R_blk.shape[0], f1.R_blk.shape[1]
    nB = f1.R_B.shape[0]
    Aaug = np.concatenate([f1.R_blk, f2.R_blk], axis=1)                                 # [K, 2n, n]
    C1 = np.concatenate([f1.S, f1.c_blk[:, :, None]], axis=2)                           # [K, n, nB+1]
    C2 = np.concatenate([f2.S, f2.c_blk[:, :, None]], axis=2)
    Caug = np.concatenate([C1, C2], axis=1)                                             # [K, 2n, nB+1]
    Q, Rr = np.linalg.qr(Aaug, mode="complete")
    QtC = np.matmul(np.swapaxes(Q, 1, 2), Caug)
    R_blk, S, c_blk = Rr[:, :n, :], QtC[:, :n, :nB], QtC[:, :n, nB]
    reduced = QtC[:, n:, :].reshape(-1, nB + 1)
    tri = []
    for f in (f1, f2):
        RBc = np.zeros((nB + 1, nB + 1))
        RBc[:nB, :nB] = f.R_B
        RBc[:nB, nB] = f.c_B
        RBc[nB, nB] = f.resid
        tri.append(RBc)
    stack = np.concatenate([reduced] + tri, axis=0)
    R3 = np.linalg.qr(stack, mode="r")
    return BlockAngularFactor(R_blk.copy(), S.copy(), c_blk.copy(), R3[:nB, :nB].copy(), R3[:nB, nB].copy(),
                              float(abs(R3[nB, nB])))


def _backsub_batched(R: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Solve R_k x_k = c_k for a stack of small upper-triangular R_k."""
    K, n, _ = R.shape
    x = np.zeros((K, n))
    for i in range(n - 1, -1, -1):
        x[:, i] = (c[:, i] - np.einsum("kj,kj->k", R[:, i, i + 1:], x[:, i + 1:])) / R[:, i, i]
    return x


def _fwdsub_T_batched(R: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Solve R_k^T y_k = g_k for a stack of small upper-triangular R_k."""
    K, n, _ = R.shape
    y = np.zeros((K, n))
    for i in range(n):
        y[:, i] = (g[:, i] - np.einsum("kj,kj->k", R[:, :i, i], y[:, :i])) / R[:, i, i]
    return y


def _backsub(R, c):
    n = R.shape[0]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (c[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x


def _fwdsub_T(R, g):
    n = R.shape[0]
    y = np.zeros(n)
    for i in range(n):
        y[i] = (g[i] - R[:i, i] @ y[:i]) / R[i, i]
    return y


def check_nonsingular(f: BlockAngularFactor):
    diags = [np.abs(np.diagonal(f.R_blk, axis1=1, axis2=2)).reshape(-1), np.abs(np.diag(f.R_B))]
    dg = np.concatenate(diags)
    if dg.size and dg.min() <= dg.size * np.finfo(np.float64).eps * dg.max():
        from .dense import SingularError
        raise SingularError("structured R has a (numerically) zero pivot")


def solve_factor(f: BlockAngularFactor) -> np.ndarray:
    """Back-substitution through [[blkdiag(R_i), S], [0, R_B]] p = [c_blk; c_B]."""
    check_nonsingular(f)
    pB = _backsub(f.R_B, f.c_B)
    rhs = f.c_blk - np.einsum("knj,j->kn", f.S, pB)
    p_blk = _backsub_batched(f.R_blk, rhs)
    return np.concatenate([p_blk.reshape(-1), pB])


def solve_RtR(f: BlockAngularFactor, g: np.ndarray) -> np.ndarray:
    """delta = (R^T R)^{-1} g with the structured R (two triangular solves)."""
    K, n, nB = f.S.shape[0], f.S.shape[1], f.S.shape[2]
    g = np.asarray(g, np.float64)
    g_blk = g[:K * n].reshape(K, n)
    g_B = g[K * n:]
    # R^T y = g :  R_i^T y_i = g_i ;  R_B^T y_B = g_B - sum_i S_i^T y_i
    y_blk = _fwdsub_T_batched(f.R_blk, g_blk)
    y_B = _fwdsub_T(f.R_B, g_B - np.einsum("knj,kn->j", f.S, y_blk))
    # R delta = y :  R_B delta_B = y_B ;  R_i delta_i = y_i - S_i delta_B
    dB = _backsub(f.R_B, y_B)
    d_blk = _backsub_batched(f.R_blk, y_blk - np.einsum("knj,j->kn", f.S, dB))
    return np.concatenate([d_blk.reshape(-1), dB])


def solve_blockangular(inst):
    """O2 end to end: returns (p, factor)."""
    f = factor_blockangular(inst)
    return solve_factor(f), f
