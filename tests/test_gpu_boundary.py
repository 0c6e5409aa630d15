"""GPU checks of the boundary conventions, through the C ABI: caller-owned
setup workspace, the log-coefficient map, and the factor generation that
keeps an adjoint solve tied to its own forward solve."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from oracle import adjoint

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def pk():
    import paper_2001_07289_amd as m
    return m


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def test_workspace_setup_equals_library_allocation():
    """The same setup in a PyTorch workspace and in library-allocated memory
    gives bitwise the same preconditioner; the workspace holds exactly the
    reported size."""
    p = W.config2_like(n=24, H=6, L=3, cfg=70)
    m = pk()
    prob = m.Problem.from_workload(p)
    a = m.Preconditioner(prob, dev(p.rho), workspace=True)
    b = m.Preconditioner(prob, dev(p.rho), workspace=False)
    assert a._ws.numel() == prob.workspace_size(a.options) == a.info()["device_bytes"]
    r = dev(W.rng(70, 0).standard_normal(p.n_free))
    assert torch.equal(a.apply(r), b.apply(r))
    xa, sa = a.solve(dev(p.f[0]))
    xb, sb = b.solve(dev(p.f[0]))
    assert torch.equal(xa, xb) and sa["iters"] == sb["iters"]


def test_workspace_too_small_or_misaligned_is_refused():
    p = W.config1()
    m = pk()
    B = m._binding
    lib = B.load()
    prob = m.Problem.from_workload(p)
    o = m.default_options()
    need = prob.workspace_size(o)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rho = dev(p.rho)
    out = C.c_void_p()
    st = lib.bddcso_setup(prob._h, C.c_void_p(rho.data_ptr()), C.byref(o), C.c_void_p(ws.data_ptr()), need - 1,
                          None, C.byref(out))
    assert B.STATUS[st] == "EINVAL" and "workspace too small" in lib.bddcso_last_error().decode()
    st = lib.bddcso_setup(prob._h, C.c_void_p(rho.data_ptr()), C.byref(o), C.c_void_p(ws.data_ptr() + 8), need - 8,
                          None, C.byref(out))
    assert B.STATUS[st] == "EINVAL" and "aligned" in lib.bddcso_last_error().decode()
    st = lib.bddcso_setup(prob._h, C.c_void_p(rho.data_ptr()), C.byref(o), C.c_void_p(ws.data_ptr()), need,
                          None, C.byref(out))
    assert st == 0
    lib.bddcso_precond_destroy(out)


def test_coef_from_log_matches_oracle():
    p = W.config5_like(n=16, H=4, L=2, cfg=71, name="adj16")
    m = pk()
    prob = m.Problem.from_workload(p)
    th = p.extra["theta"]
    rho = host(prob.coef_from_log(dev(th)))
    ref = adjoint.rho_of_theta(th, p.n_el)
    assert np.abs(rho - ref).max() <= 1e-14 * np.abs(ref).max()


def test_generation_counts_numeric_setups():
    p = W.config1()
    m = pk()
    pc = m.Preconditioner(m.Problem.from_workload(p), dev(p.rho))
    g0 = pc.generation
    pc.refactor(dev(p.rho))
    pc.refactor(dev(p.rho))
    assert pc.generation == g0 + 2


def test_interleaved_forwards_give_their_own_gradients():
    """Two forward solves on one preconditioner before either backward: each
    backward refactors from its own forward's coefficient, so both gradients
    equal those of separate forward/backward pairs."""
    p = W.config5_like(n=16, H=4, L=2, cfg=72, name="adj16")
    m = pk()
    prob = m.Problem.from_workload(p)
    pc = m.Preconditioner(prob, dev(np.ones(p.n_elements)), rtol=1e-12)
    f = dev(p.f[0])
    u_obs = dev(W.rng(72, 9).standard_normal(p.n_free) * 1e-2)
    th1 = p.extra["theta"]
    th2 = p.extra["theta_obs"]

    def grad_alone(th):
        t = dev(th).requires_grad_(True)
        u = m.BDDCSOSolve.apply(t, f, pc)
        (0.5 * torch.sum((u - u_obs) ** 2)).backward()
        return host(t.grad)

    g1, g2 = grad_alone(th1), grad_alone(th2)
    t1 = dev(th1).requires_grad_(True)
    t2 = dev(th2).requires_grad_(True)
    l1 = 0.5 * torch.sum((m.BDDCSOSolve.apply(t1, f, pc) - u_obs) ** 2)
    l2 = 0.5 * torch.sum((m.BDDCSOSolve.apply(t2, f, pc) - u_obs) ** 2)
    l1.backward()
    l2.backward()
    assert np.array_equal(host(t1.grad), g1)
    assert np.array_equal(host(t2.grad), g2)
    assert np.linalg.norm(g1 - g2) > 1e-3 * np.linalg.norm(g1)
