"""GPU parity against the oracle on a reduced form of the batched uneven
workload: a 48^3 mesh cut by seeded planes into 4^3 boxes of 8^3 to 16^3
elements (the 16-element boxes have 289-node plane blocks, the largest the
register sweep holds), subobject lengths 2h / 4h / 8h drawn per axis
interval, channels of coefficient 1e6 aligned with the subobjects, and six
right-hand sides solved in lockstep by the many-RHS kernels.  Each column
at an equal iteration count to 1e-10, free-running iterations within 1 and
kappa within 1%, for ordinary launches and for replayed graphs."""
import numpy as np
import pytest

import workloads as W
from oracle import bddc, pcg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def uneven():
    p = W.config3(n=48, nrhs=6, count=4, cfg=30, n_channels_per_axis=2)
    orc = bddc.from_problem(p)
    refs = [pcg.solve(orc, p.f[k], rtol=1e-8) for k in range(6)]
    print(f"\n[uneven] 48^3, cuts {p.extra['sub_cuts']}, {orc.cls.n_coarse} coarse dofs, "
          f"oracle iterations {[r.iters for r in refs]}", flush=True)
    return p, orc, refs


@pytest.mark.parametrize("graph", [0, 1], ids=["eager", "graph"])
def test_uneven_many_rhs_match_oracle(uneven, graph):
    import paper_2001_07289_amd as m
    p, orc, refs = uneven
    prob = m.Problem.from_workload(p)
    F = dev(p.f.reshape(-1))
    kfix = max(r.iters for r in refs)
    pcf = m.Preconditioner(prob, dev(p.rho), max_nrhs=6, fixed_iters=kfix, graph=graph)
    X = pcf.solve(F)[0].cpu().numpy().reshape(6, -1)
    for k in range(6):
        rk = refs[k] if refs[k].iters == kfix else pcg.solve(orc, p.f[k], fixed_iters=kfix)
        assert relerr(X[k], rk.x) <= 1e-10, k
    pc = m.Preconditioner(prob, dev(p.rho), max_nrhs=6, graph=graph)
    X, st = pc.solve(F)
    X = X.cpu().numpy().reshape(6, -1)
    for k in range(6):
        assert abs(st["iters"][k] - refs[k].iters) <= 1, k
        assert abs(st["kappa"][k] - refs[k].kappa) <= 0.01 * refs[k].kappa, k
        rk = refs[k] if st["iters"][k] == refs[k].iters else pcg.solve(orc, p.f[k], fixed_iters=st["iters"][k])
        assert relerr(X[k], rk.x) <= 1e-10, k
