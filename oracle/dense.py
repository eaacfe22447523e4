"""O1: dense Householder oracle for the damped least-squares step.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper's statement of the step (Section 1, Eq. 2): the LM update p
is the least-squares solution of [J; sqrt(lam) D] p = [b; 0], solved by a QR
decomposition (Section 2: Householder matrices H = I - 2 v v^T applied in turn
to zero the subdiagonal of each column, R = H_{N-1} ... H_0 A, and Q kept only
implicitly by applying the reflectors to the right-hand side).

Conventions (the paper states none; these are the readings taken):
  * reflector for x = A[j:, j]: alpha = x_0, sigma = ||x_{1:}||^2;
    sigma == 0 -> tau = 0 (no reflection, the diagonal keeps its sign);
    otherwise beta = -sign(alpha) sqrt(alpha^2 + sigma) with sign(0) = +1,
    tau = (beta - alpha) / beta, v = [1, x_{1:} / (alpha - beta)],
    H = I - tau v v^T  (equivalent to I - 2 u u^T with u = v / ||v||).
  * R diagonals may be negative; comparisons normalise row signs.
"""
from __future__ import annotations

import numpy as np

from workloads.generators import BlockAngular


class SingularError(np.linalg.LinAlgError):
    pass


def householder_vector(x: np.ndarray):
    """Return (v, tau, beta) with (I - tau v v^T) x = beta e_1."""
    x = np.asarray(x, dtype=np.float64)
    alpha = float(x[0])
    sigma = float(np.dot(x[1:], x[1:]))
    v = np.zeros_like(x)
    v[0] = 1.0
    if sigma == 0.0:
        return v, 0.0, alpha
    norm = np.sqrt(alpha * alpha + sigma)
    beta = -norm if alpha >= 0.0 else norm
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def householder_qr(A: np.ndarray, Y: np.ndarray | None = None):
    """Householder QR of A (m x n, m >= n is not required).

    Returns (R, QtY, reflectors) where R is min(m,n) x n upper triangular,
    QtY = Q^T Y (all m rows, if Y is given) and reflectors is a list of
    (j, v, tau) so that Q^T = H_{k-1} ... H_0.
    """
    A = np.array(A, dtype=np.float64, copy=True)
    m, n = A.shape
    if Y is not None:
        Y = np.array(Y, dtype=np.float64, copy=True)
        squeeze = Y.ndim == 1
        if squeeze:
            Y = Y[:, None]
    refl = []
    for j in range(min(m, n)):
        v, tau, beta = householder_vector(A[j:, j])
        if tau != 0.0:
            # A[j:, j:] <- (I - tau v v^T) A[j:, j:]
            A[j:, j:] -= tau * np.outer(v, v @ A[j:, j:])
            if Y is not None:
                Y[j:, :] -= tau * np.outer(v, v @ Y[j:, :])
        A[j, j] = beta
        A[j + 1:, j] = 0.0
        refl.append((j, v, tau))
    k = min(m, n)
    R = np.triu(A[:k, :])
    if Y is None:
        return R, None, refl
    QtY = Y[:, 0] if squeeze else Y
    return R, QtY, refl


def apply_qt(refl, Y: np.ndarray) -> np.ndarray:
    """Q^T Y from stored reflectors."""
    Y = np.array(Y, dtype=np.float64, copy=True)
    for j, v, tau in refl:
        Y[j:] -= tau * np.outer(v, v @ Y[j:]) if Y.ndim == 2 else tau * v * (v @ Y[j:])
    return Y


def apply_q(refl, Y: np.ndarray) -> np.ndarray:
    """Q Y from stored reflectors (Q = H_0 ... H_{k-1})."""
    Y = np.array(Y, dtype=np.float64, copy=True)
    for j, v, tau in reversed(refl):
        Y[j:] -= tau * np.outer(v, v @ Y[j:]) if Y.ndim == 2 else tau * v * (v @ Y[j:])
    return Y


def back_substitute(R: np.ndarray, c: np.ndarray, check: bool = True) -> np.ndarray:
    """Solve R p = c for upper-triangular R (plain row-by-row substitution)."""
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    if check:
        diag = np.abs(np.diag(R))
        if n and diag.min() <= n * np.finfo(np.float64).eps * diag.max():
            raise SingularError("R has a (numerically) zero pivot")
    c = np.asarray(c, dtype=np.float64)
    p = np.zeros_like(c)
    for i in range(n - 1, -1, -1):
        p[i] = (c[i] - R[i, i + 1:] @ p[i + 1:]) / R[i, i]
    return p


def forward_substitute_transposed(R: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Solve R^T y = g for upper-triangular R."""
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    y = np.zeros(n, dtype=np.float64)
    for i in range(n):
        y[i] = (g[i] - R[:i, i] @ y[:i]) / R[i, i]
    return y


def solve_augmented(J: np.ndarray, b: np.ndarray, d: np.ndarray, lam: float):
    """Solve min ||[J; sqrt(lam) diag(d)] p - [b; 0]|| by O1.

    Returns dict(p, R, c, resid, refl).
    """
    J = np.asarray(J, dtype=np.float64)
    M, N = J.shape
    Aaug = np.vstack([J, np.sqrt(lam) * np.diag(np.asarray(d, np.float64))])
    y = np.concatenate([np.asarray(b, np.float64), np.zeros(N)])
    R, Qty, refl = householder_qr(Aaug, y)
    R = R[:N, :N]
    c = Qty[:N]
    resid = float(np.linalg.norm(Qty[N:]))
    p = back_substitute(R, c)
    return dict(p=p, R=R, c=c, resid=resid, refl=refl)


def assemble_blockangular(inst) -> np.ndarray:
    """Dense J (M x N) of a block-angular instance (float64 of the stored values)."""
    K, n, M, nB = inst.K, inst.n, inst.M, inst.nB
    J = np.zeros((M, K * n + nB), dtype=np.float64)
    A = inst.A.astype(np.float64)
    for i in range(K):
        r0, r1 = int(inst.row_off[i]), int(inst.row_off[i + 1])
        J[r0:r1, i * n:(i + 1) * n] = A[r0:r1]
    J[:, K * n:] = inst.B.astype(np.float64)
    return J


def assemble_blockangular_ncol(inst) -> np.ndarray:
    """Dense J (M x N) of a block-angular instance whose block i has its own n_i columns
    (Section 4.1 lets every diagonal block be m_i x n_i): block i's values are its rows
    row-major, n_i per row, block after block; its columns follow those of the blocks before
    it, the dense part's columns come last."""
    K, M, nB = inst.K, inst.M, inst.nB
    N = int(np.sum(inst.ncol)) + nB
    J = np.zeros((M, N), dtype=np.float64)
    A = inst.A.astype(np.float64)
    pos, col = 0, 0
    for i in range(K):
        r0, r1 = int(inst.row_off[i]), int(inst.row_off[i + 1])
        ni = int(inst.ncol[i])
        J[r0:r1, col:col + ni] = A[pos:pos + (r1 - r0) * ni].reshape(r1 - r0, ni)
        pos += (r1 - r0) * ni
        col += ni
    J[:, col:] = inst.B.astype(np.float64)
    return J


def camera_columns(inst) -> np.ndarray:
    """Dense B (M x ncam*cw, float64) of a camera-block instance: row r's cw values go to the
    columns of its camera cam[r] (cameras in order, cw columns each); a row whose camera is
    outside [0, ncam) touches no camera (the bundle-adjustment Jacobian of Section 6.2: every
    observation depends on one point and one camera)."""
    M, ncam, cw = inst.M, inst.ncam, inst.cw
    B = np.zeros((M, ncam * cw), dtype=np.float64)
    Bv = inst.Bv.astype(np.float64)
    for r in range(M):
        c = int(inst.cam[r])
        if 0 <= c < ncam:
            B[r, c * cw:(c + 1) * cw] = Bv[r]
    return B


def blockangular_from_cam(inst):
    """The camera-block instance as a block-angular instance with its B stored dense (the
    values are moved, not rounded, so the stored J is the same)."""
    B = camera_columns(inst).astype(inst.dtype)
    return BlockAngular(inst.row_off.copy(), inst.n, inst.A.copy(), B, inst.b.copy(), inst.d.copy(), inst.lam,
                        inst.dtype)


def solve_blockangular_dense(inst):
    """O1 on an assembled block-angular instance."""
    J = assemble_blockangular(inst)
    return solve_augmented(J, inst.b.astype(np.float64), inst.d, inst.lam)


def sign_normalise(R: np.ndarray, *rows_alongside):
    """Flip rows so that diag(R) >= 0; the same flips are applied to the extra arrays."""
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    out = [R * s[:, None]]
    for X in rows_alongside:
        X = np.asarray(X, dtype=np.float64)
        out.append(X * (s[:, None] if X.ndim == 2 else s))
    return out if rows_alongside else out[0]
