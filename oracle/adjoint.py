"""Gradient of a loss of the LM step with respect to its inputs.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The step is p = M^{-1} J^T b with M = J^T J + lam D^2 (paper, Section 1, Eq. 1).
Differentiating M p = J^T b gives
    M dp = dJ^T r + J^T db - J^T dJ p - dlam D^2 p - 2 lam D dD p,   r = b - J p.
For a loss L(p) with g = dL/dp and u = M^{-1} g (two triangular solves with the
stored R, since R^T R = M):
    dL/db      = J u
    dL/dJ_ab   = r_a u_b - (J u)_a p_b       (only structural nonzeros are kept)
    dL/dlam    = -u^T D^2 p
    dL/dd_j    = -2 lam u_j d_j p_j          (d treated as an independent input)
"""
from __future__ import annotations

import numpy as np

from . import refine, structured


def adjoint_blockangular(inst, factor, p, g):
    """Closed-form gradients for a block-angular instance (float64).

    Returns dict(dA [M,n], dB [M,nB], db [M], dlam, dd [N], u [N]).
    """
    K, n = inst.K, inst.n
    p = np.asarray(p, np.float64)
    u = structured.solve_RtR(factor, np.asarray(g, np.float64))
    r = inst.b.astype(np.float64) - refine.apply_J(inst, p, np.float64)
    Ju = refine.apply_J(inst, u, np.float64)
    blk = inst.block_of_row()
    u_blk = u[:K * n].reshape(K, n)
    p_blk = p[:K * n].reshape(K, n)
    dA = r[:, None] * u_blk[blk] - Ju[:, None] * p_blk[blk]
    dB = np.outer(r, u[K * n:]) - np.outer(Ju, p[K * n:])
    d = np.asarray(inst.d, np.float64)
    dlam = float(-np.sum(u * d * d * p))
    dd = -2.0 * inst.lam * u * d * p
    return dict(dA=dA, dB=dB, db=Ju, dlam=dlam, dd=dd, u=u)


def adjoint_dense(J, b, d, lam, p, g, R):
    """The same closed form for a dense J with its R (R^T R = J^T J + lam D^2)."""
    from .dense import back_substitute, forward_substitute_transposed
    J = np.asarray(J, np.float64)
    u = back_substitute(R, forward_substitute_transposed(R, np.asarray(g, np.float64)))
    r = np.asarray(b, np.float64) - J @ p
    Ju = J @ u
    dJ = np.outer(r, u) - np.outer(Ju, p)
    d = np.asarray(d, np.float64)
    return dict(dJ=dJ, db=Ju, dlam=float(-np.sum(u * d * d * p)), dd=-2.0 * lam * u * d * p, u=u)
