"""The step solve (factor + solve with refinement sweeps) captured into a HIP graph through
torch.cuda.graph and replayed: every replay, with eager work and synchronisations between the
replays, gives p bit for bit equal to the eager step, and a replay after the inputs change in
place follows them (the graph holds the pointers, the handle re-reads the data)."""
import numpy as np
import pytest

from workloads import generators as gen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,sweeps", [("plain", 1), ("bf16x3", 2)])
def test_graph_replays_match_eager_step(mode, sweeps):
    import torch
    from paper_1802_03773_amd import BlockAngularSolver
    inst = gen.make_blockangular(901, K=2000, m=(np.arange(2000) % 7) + 6, n=3, nB=60, lam=1e-2, dtype=np.float32)
    A, B, b, d = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (inst.A, inst.B, inst.b, inst.d))
    s = BlockAngularSolver(inst.row_off, inst.n, inst.nB, mode=mode)
    p = torch.empty(inst.N, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up off the default stream before capture
        s.factor(A, B, b, d, inst.lam)
        s.solve(sweeps=sweeps, out=p)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = p.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.factor(A, B, b, d, inst.lam)
        s.solve(sweeps=sweeps, out=p)
    for r in range(4):
        p.fill_(float("nan"))
        x = torch.ones(1 << 20, device="cuda").cumsum(0)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(p, eager), f"replay {r}"
        assert float(x[-1]) == float(1 << 20)
    # new values in the same buffers: the replay solves the new problem, as an eager step does
    b.mul_(-2.0)
    g.replay()
    torch.cuda.synchronize()
    replayed = p.clone()
    s.factor(A, B, b, d, inst.lam)
    s.solve(sweeps=sweeps, out=p)
    torch.cuda.synchronize()
    assert torch.equal(replayed, p)
    assert torch.allclose(replayed, -2.0 * eager, rtol=1e-9, atol=0.0)
    assert s.status()[0] == 0
