"""Graph mode (options.graph = 1): the numeric setup and the two halves of a
PCG iteration are captured into HIP graphs once and replayed.  Every replay
must give bitwise the results of ordinary launches, with the program's own
eager work and synchronisations between the replays."""
import numpy as np
import pytest

import workloads as W
from oracle import bddc, pcg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def pk():
    import paper_2001_07289_amd as m
    return m


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_graph_replays_equal_eager(precision):
    p = W.config2_like(n=24, H=6, L=3, cfg=71)
    m = pk()
    prob = m.Problem.from_workload(p)
    rho0 = dev(p.rho)
    kw = dict(max_nrhs=3, precision=precision, rtol=1e-8)
    pe = m.Preconditioner(prob, rho0, graph=0, **kw)
    pg = m.Preconditioner(prob, rho0, graph=1, **kw)
    rng = W.rng(71, 0)
    b1 = dev(rng.uniform(-1, 1, p.n_free))
    b3 = dev(rng.uniform(-1, 1, 3 * p.n_free))
    for rep in range(4):
        rho = rho0 * (1.0 + 0.25 * rep)
        pe.refactor(rho)
        pg.refactor(rho)          # first call captures, later calls replay
        # eager work between replays
        y = pe.operator(b1)
        z = pg.apply(b1)
        torch.cuda.synchronize()
        assert torch.equal(z, pe.apply(b1)), rep
        for b in (b1, b3):
            xe, se = pe.solve(b)
            xg, sg = pg.solve(b)
            torch.cuda.synchronize()
            assert se["iters"] == sg["iters"], (rep, se["iters"], sg["iters"])
            assert torch.equal(xe, xg), rep
        assert float(torch.linalg.norm(y)) > 0


def test_graph_fixed_iterations_match_oracle():
    """Graph-mode iterates at the oracle's iteration count, to 1e-10."""
    p = W.config2_like(n=18, H=6, L=3, cfg=72)
    orc = bddc.from_problem(p)
    ref = pcg.solve(orc, p.f[0], rtol=1e-8)
    m = pk()
    prob = m.Problem.from_workload(p)
    pc = m.Preconditioner(prob, dev(p.rho), graph=1, fixed_iters=ref.iters)
    for _ in range(3):
        x, _ = pc.solve(dev(p.f[0]))
        err = float(np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x))
        assert err <= 1e-10, err


def test_coarse_factorization_overlap_orders_setups():
    """The coarse factorization runs on its own stream and the next
    application waits for it: back-to-back refactors, then a solve, equal a
    fresh setup with the last coefficient (bitwise), in ordinary mode."""
    p = W.config2_like(n=24, H=6, L=3, cfg=73)
    m = pk()
    prob = m.Problem.from_workload(p)
    rho0 = dev(p.rho)
    a = m.Preconditioner(prob, rho0 * 3.0)
    a.refactor(rho0 * 0.5)
    a.refactor(rho0)
    b = dev(p.f[0])
    xa, sa = a.solve(b)
    fresh = m.Preconditioner(prob, rho0)
    xf, sf = fresh.solve(b)
    torch.cuda.synchronize()
    assert sa["iters"] == sf["iters"]
    assert torch.equal(xa, xf)
    z1 = a.apply(b)
    a.refactor(rho0)
    assert torch.equal(a.apply(b), z1)
