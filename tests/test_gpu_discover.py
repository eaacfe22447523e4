"""Structure discovery end to end (Section 4.3): a block-angular J and a banded J whose rows (and,
block-angular, columns) were shuffled are brought back to their structures by
qrk_discover_blockangular / qrk_discover_banded, gathered into the solvers' layouts, solved on the
GPU, and the step mapped back to the shuffled unknowns is compared with the damped least-squares
solution of the shuffled problem (LAPACK on the dense matrix).  Float32, unrefined 1e-5 at cond <=
1e3 (scaled by cond / 1e3 above), 1e-10 after two sweeps."""
import numpy as np
import pytest

from oracle import dense
from tests.gpu_util import log, p_err
from workloads import generators as gen

pytestmark = pytest.mark.gpu


def _csr_of(J):
    nz = J != 0
    row_ptr = np.zeros(J.shape[0] + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(nz.sum(axis=1))
    col_idx = np.nonzero(nz)[1].astype(np.int32)
    return row_ptr, col_idx


def _lstsq(J, b, d, lam):
    Aaug = np.vstack([J, np.sqrt(lam) * np.diag(d)])
    rhs = np.concatenate([b, np.zeros(J.shape[1])])
    p, *_ = np.linalg.lstsq(Aaug, rhs, rcond=None)
    return p, np.linalg.cond(Aaug)


def test_discovered_blockangular_solves_the_shuffled_problem():
    import torch
    from paper_1802_03773_amd import BlockAngularNcolSolver, discover_blockangular
    inst = gen.make_blockangular_ncol(61, K=250, m=(np.arange(250) % 8) + 2, ncol=(np.arange(250) * 3) % 8 + 1,
                                      nB=20, lam=1e-2, dtype=np.float32)
    J = dense.assemble_blockangular_ncol(inst)
    rng = np.random.default_rng(62)
    pr, pc = rng.permutation(inst.M), rng.permutation(inst.N)
    Js, bs, ds = J[pr][:, pc], inst.b.astype(np.float64)[pr], inst.d[pc]
    nd = int(inst.p_off()[inst.K])
    dense_new = np.argsort(pc)[nd:]                  # where the coupled columns went
    rp, ci = _csr_of(Js)
    st = discover_blockangular(rp, ci, inst.N, dense_new)
    K, ncol, row_off, rperm, cperm = st["K"], st["ncol"], st["row_off"], st["row_perm"], st["col_perm"]
    co = np.concatenate([[0], np.cumsum(ncol)])
    A = np.concatenate([Js[np.ix_(rperm[row_off[k]:row_off[k + 1]], cperm[co[k]:co[k + 1]])].reshape(-1)
                        for k in range(K)]).astype(np.float32)
    B = Js[np.ix_(rperm, cperm[co[K]:])].astype(np.float32)
    b = bs[rperm].astype(np.float32)
    d = ds[cperm]
    s = BlockAngularNcolSolver(row_off, ncol, B.shape[1])
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (A, B, b, d)]
    s.factor(*dev, inst.lam)
    p_ref, cond = _lstsq(Js, bs, ds, inst.lam)
    out = {}
    for sw in (0, 2):
        pp = s.solve(sweeps=sw).cpu().numpy()
        p = np.empty_like(pp)
        p[cperm] = pp                                # back to the shuffled problem's unknowns
        out[sw] = p_err(p, p_ref, ds)
    torch.cuda.synchronize()
    log(f"discovered block-angular ({K} blocks, cond {cond:.3g}): unrefined {out[0]:.2e}, two sweeps {out[2]:.2e}")
    assert K == inst.K and s.status()[0] == 0
    assert out[0] <= 1e-5 * max(1.0, cond / 1e3)
    assert out[2] <= 1e-10


def test_discovered_banded_solves_the_shuffled_problem():
    import torch
    from paper_1802_03773_amd import BandedSolver, discover_banded
    inst = gen.make_banded(71, N=600, w=12, dtype=np.float32)
    M, N, w = 2 * 600, 600, 12
    J = np.zeros((M, N))
    for i in range(M):
        J[i, inst.row_start[i]:inst.row_start[i] + w] = inst.vals[i]
    rng = np.random.default_rng(72)
    pr = rng.permutation(M)
    Js, bs = J[pr], inst.b.astype(np.float64)[pr]
    rp, ci = _csr_of(Js)
    st = discover_banded(rp, ci, N)
    rperm, starts = st["row_perm"], st["row_start"]
    assert st["w"] == w
    vals = np.stack([Js[rperm[k], starts[k]:starts[k] + w] for k in range(M)]).astype(np.float32)
    b = bs[rperm].astype(np.float32)
    s = BandedSolver(M, N, w)
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (starts, vals, b, inst.d)]
    s.factor(*dev, inst.lam)
    p_ref, cond = _lstsq(Js, bs, inst.d, inst.lam)
    e0 = p_err(s.solve(sweeps=0).cpu().numpy(), p_ref, inst.d)
    e2 = p_err(s.solve(sweeps=2).cpu().numpy(), p_ref, inst.d)
    torch.cuda.synchronize()
    log(f"discovered banded (cond {cond:.3g}): unrefined {e0:.2e}, two sweeps {e2:.2e}")
    assert s.status()[0] == 0
    assert e0 <= 1e-5 * max(1.0, cond / 1e3)
    assert e2 <= 1e-10
