"""Pins of the oracle's block-angular J with per-block column counts (Section 4.1: block i is
m_i x n_i).  The ragged assembly agrees with the uniform one when every n_i = n; the damped
least-squares solution of the ragged problem (LAPACK on the dense matrix) satisfies the normal
equations; and the structured oracle on the problem widened to n = max n_i (zero columns past
n_i, damping value 1 for them) gives the same solution on the real unknowns and exact zeros on
the added ones, which is how the GPU path runs such a problem.  Planted mistake: added columns
without damping make the widened problem singular."""
import numpy as np
import pytest

from oracle import dense, structured
from workloads import generators as gen


def _instance(seed, K=40, nB=7, lam=1e-2):
    return gen.make_blockangular_ncol(seed, K=K, m=(np.arange(K) % 7) + 2, ncol=(np.arange(K) * 5) % 8 + 1,
                                      nB=nB, lam=lam, dtype=np.float64)


def _lstsq(inst):
    J = dense.assemble_blockangular_ncol(inst)
    Aaug = np.vstack([J, np.sqrt(inst.lam) * np.diag(inst.d)])
    rhs = np.concatenate([inst.b.astype(np.float64), np.zeros(inst.N)])
    p, *_ = np.linalg.lstsq(Aaug, rhs, rcond=None)
    return J, p


def _widened(inst, dpad=1.0):
    """The instance at n = max n_i: zero columns past n_i, damping value dpad for them."""
    K, n = inst.K, int(inst.ncol.max())
    ao, po = inst.a_off(), inst.p_off()
    A = np.zeros((inst.M, n), dtype=inst.dtype)
    d = np.full(K * n + inst.nB, float(dpad))
    for i in range(K):
        r0, r1, ni = int(inst.row_off[i]), int(inst.row_off[i + 1]), int(inst.ncol[i])
        A[r0:r1, :ni] = inst.A[ao[i]:ao[i + 1]].reshape(r1 - r0, ni)
        d[i * n:i * n + ni] = inst.d[po[i]:po[i] + ni]
    d[K * n:] = inst.d[po[K]:]
    return gen.BlockAngular(inst.row_off.copy(), n, A, inst.B, inst.b, d, inst.lam, inst.dtype)


def test_uniform_widths_match_the_uniform_assembly():
    inst = gen.make_blockangular_ncol(3, K=25, m=(np.arange(25) % 5) + 3, ncol=3, nB=6, lam=1e-2)
    uni = gen.BlockAngular(inst.row_off, 3, inst.A.reshape(inst.M, 3), inst.B, inst.b, inst.d, inst.lam,
                           inst.dtype)
    assert np.array_equal(dense.assemble_blockangular_ncol(inst), dense.assemble_blockangular(uni))
    # and the generator's d is the column norms of that matrix
    J = dense.assemble_blockangular_ncol(inst)
    assert np.allclose(inst.d, np.linalg.norm(J, axis=0), rtol=1e-14)


def test_block_columns_land_where_the_layout_says():
    inst = _instance(5)
    J = dense.assemble_blockangular_ncol(inst)
    ao, po = inst.a_off(), inst.p_off()
    for i in (0, 1, 17, inst.K - 1):
        r0, r1, ni = int(inst.row_off[i]), int(inst.row_off[i + 1]), int(inst.ncol[i])
        blk = inst.A[ao[i]:ao[i + 1]].reshape(r1 - r0, ni)
        assert np.array_equal(J[r0:r1, po[i]:po[i] + ni], blk)
        others = np.delete(J[r0:r1, :po[inst.K]], np.arange(po[i], po[i] + ni), axis=1)
        assert not others.any()


def test_solution_satisfies_the_normal_equations():
    inst = _instance(11)
    J, p = _lstsq(inst)
    lhs = J.T @ J @ p + inst.lam * inst.d ** 2 * p
    rhs = J.T @ inst.b.astype(np.float64)
    assert np.abs(lhs - rhs).max() <= 1e-11 * np.abs(rhs).max()


@pytest.mark.parametrize("nB", [0, 7, 30])
@pytest.mark.parametrize("lam", [1e-2, 1.0])
def test_widened_structured_oracle_gives_the_ragged_solution(nB, lam):
    inst = _instance(21 + nB, nB=nB, lam=lam)
    _, p_ref = _lstsq(inst)
    wide = _widened(inst)
    p_w, _ = structured.solve_blockangular(wide)
    n, po = wide.n, inst.p_off()
    got = np.concatenate([p_w[i * n:i * n + int(inst.ncol[i])] for i in range(inst.K)] + [p_w[inst.K * n:]])
    assert np.abs(got - p_ref).max() <= 1e-10 * np.abs(p_ref).max()
    added = np.concatenate([p_w[i * n + int(inst.ncol[i]):(i + 1) * n] for i in range(inst.K)])
    assert added.size and np.all(added == 0.0)
    assert po[inst.K] + nB == inst.N


def test_planted_mistake_undamped_widening_is_singular():
    inst = _instance(31)
    with pytest.raises(np.linalg.LinAlgError):
        structured.solve_blockangular(_widened(inst, dpad=0.0))
