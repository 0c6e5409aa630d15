"""Table 1 of the paper (Section 5.1) on the GPU: PCG iterations to a 10^6
reduction of the residual for the Poisson problem with f = 1 on (10k)^3
hexahedra, 10^3 subdomains of k^3 cells, BDDC-SO(vef) with L/h = 4 and
BDDC(vef) (L = H).  The printed counts are the reference (within +-1, a tie
at the threshold); the coarse sizes must match exactly.  BDDC-SO at k = 24
(354,159 coarse unknowns) needs more device memory than one GPU holds with
this single-level coarse solver, so it is left out."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _golden(name):
    from conftest import golden_path
    out = {}
    for line in open(golden_path(name)):
        f = line.split("#")[0].split()
        if f:
            out[(f[0], int(f[1]))] = int(f[2])
    return out


def _solve(p, method):
    import paper_2001_07289_amd as m
    prob = m.Problem.from_workload(p)
    rho = torch.ones(p.n_elements, dtype=torch.float64, device="cuda")
    pc = m.Preconditioner(prob, rho, rtol=1e-6, maxit=100)
    b = torch.as_tensor(np.ascontiguousarray(p.f[0]), device="cuda")
    x, st = pc.solve(b)
    A_res = torch.linalg.norm(b - pc.operator(x)) / torch.linalg.norm(b)
    return prob.info()["n_coarse"], st, float(A_res)


@pytest.mark.parametrize("k", [4, 8, 16])
def test_bddc_so_vef(k):
    iters, sizes = _golden("table1_iters.txt"), _golden("table1.txt")
    p = W.table1_problem(k)
    nc, st, res = _solve(p, "BDDC-SO(vef)")
    print(f"BDDC-SO(vef) k={k}: coarse {nc}, iterations {st['iters'][0]}, kappa {st['kappa'][0]:.3f}")
    assert nc == sizes[("BDDC-SO(vef)", k)]
    assert res <= 1.0001e-6
    assert abs(st["iters"][0] - iters[("BDDC-SO(vef)", k)]) <= 1


@pytest.mark.parametrize("k", [8, 16, 24])
def test_bddc_vef(k):
    iters, sizes = _golden("table1_iters.txt"), _golden("table1.txt")
    p = W.table1_problem(k, L=k)
    nc, st, res = _solve(p, "BDDC(vef)")
    print(f"BDDC(vef) k={k}: coarse {nc}, iterations {st['iters'][0]}, kappa {st['kappa'][0]:.3f}")
    assert nc == sizes[("BDDC(vef)", k)]
    assert res <= 1.0001e-6
    assert abs(st["iters"][0] - iters[("BDDC(vef)", k)]) <= 1
