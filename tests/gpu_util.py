"""Helpers for the GPU parity tests: move seeded instances to the device and run the
HIP path through the C ABI binding; compare with the oracle."""
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_device(inst):
    import torch
    td = torch.float32 if inst.dtype == np.float32 else torch.float64
    A = torch.from_numpy(np.ascontiguousarray(inst.A)).to("cuda")
    B = torch.from_numpy(np.ascontiguousarray(inst.B)).to("cuda") if inst.nB else None
    b = torch.from_numpy(np.ascontiguousarray(inst.b)).to("cuda")
    d = torch.from_numpy(np.ascontiguousarray(inst.d)).to("cuda")
    assert A.dtype == td
    return A, B, b, d


def gpu_solve_blockangular(inst, sweeps=0, mode="plain", leaves=0, fanin=0, return_solver=False):
    import torch
    from paper_1802_03773_amd import BlockAngularSolver
    A, B, b, d = to_device(inst)
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype=str(inst.dtype), mode=mode)
    if leaves or fanin:
        s.set_tsqr_shape(leaves, fanin)
    s.factor(A, B, b, d, inst.lam)
    p = s.solve(sweeps=sweeps)
    torch.cuda.synchronize()
    st = s.status()
    out = p.cpu().numpy()
    if return_solver:
        return out, st, s, (A, B, b, d)
    return out, st


def rel_err(p, p_ref):
    p = np.asarray(p, np.float64)
    p_ref = np.asarray(p_ref, np.float64)
    return float(np.linalg.norm(p - p_ref) / np.linalg.norm(p_ref))


def scaled_err(p, p_ref, d):
    """Largest componentwise error with each unknown weighted by its column scale d_j
    (the column 2-norm of J): max_j d_j |p_j - p_ref_j| / max_j d_j |p_ref_j|.  Under
    column scalings of 10^(k t) the unknowns with large scales are tiny, so the 2-norm error
    alone could miss them; weighted by d they count as much as the others."""
    p = np.asarray(p, np.float64)
    p_ref = np.asarray(p_ref, np.float64)
    d = np.asarray(d, np.float64)
    return float(np.max(d * np.abs(p - p_ref)) / np.max(d * np.abs(p_ref)))


def p_err(p, p_ref, d):
    """The larger of the relative 2-norm error and the column-scaled componentwise error;
    a parity bound on p holds for both measures."""
    return max(rel_err(p, p_ref), scaled_err(p, p_ref, d))


def sign_fix_rows(R, *extra):
    """Flip rows of R (and of the extra arrays) so that diag(R) >= 0."""
    R = np.asarray(R, np.float64)
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    out = [R * s[:, None]]
    for X in extra:
        X = np.asarray(X, np.float64)
        out.append(X * (s[:, None] if X.ndim == 2 else s))
    return out
