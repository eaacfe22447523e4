"""The rotated stress variant of the precision problems: the tiny-workload shapes with B <- B
diag(10^(k t_B)) H (H Haar-orthogonal), k in {3, 4, 5}, so the spread of scales is not along B's
columns and column scaling does not remove it; lambda 1e-4 (the damping rows with d = column norms
keep cond after column equilibration near 300) and lambda 0 (cond_eq 1.2e3, 1e4, 1.3e5).  The
float32 factor, plain and BF16x3, then float64-residual refinement sweeps, against the oracle's
refined solution: with damping every case reaches 1e-10 in three sweeps; without it the sweeps
needed grow with cond_eq (each sweep contracts the error by about eps_factor cond_eq), and the
counts asserted here have a margin of at least 30x over the measured errors."""
import numpy as np
import pytest

from oracle import refine
from tests.gpu_util import log, p_err
from workloads import generators as gen

pytestmark = pytest.mark.gpu

# sweeps after which the error is <= 1e-10 at lambda = 0
SWEEPS_UNDAMPED = {("plain", 3): 3, ("plain", 4): 4, ("plain", 5): 5,
                   ("bf16x3", 3): 3, ("bf16x3", 4): 5, ("bf16x3", 5): 7}


@pytest.mark.parametrize("k", [3, 4, 5])
@pytest.mark.parametrize("lam", [1e-4, 0.0])
def test_rotated_precision_problem(k, lam):
    import torch
    from paper_1802_03773_amd import BlockAngularSolver
    inst = gen.precision_rotated(400 + k, k, lam=lam)
    p_ref, _ = refine.reference_solution(inst)
    A, B, b, d = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (inst.A, inst.B, inst.b, inst.d))
    for mode in ("plain", "bf16x3"):
        s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, dtype="float32", mode=mode)
        s.factor(A, B, b, d, lam)
        need = 3 if lam > 0 else SWEEPS_UNDAMPED[(mode, k)]
        errs = [p_err(s.solve(sweeps=sw).cpu().numpy(), p_ref, inst.d) for sw in range(need + 1)]
        torch.cuda.synchronize()
        log(f"rotated k={k} lambda={lam} {mode}: " + " ".join(f"{e:.1e}" for e in errs))
        assert s.status()[0] == 0
        assert all(np.isfinite(errs))
        assert errs[need] <= 1e-10
