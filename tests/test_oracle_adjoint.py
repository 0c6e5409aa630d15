"""Pins of the oracle's gradient (CPU): adjointness of the filter and
central finite differences of the loss."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint


@pytest.mark.parametrize("n_el", [(5, 4), (4, 5, 3)])
def test_box_filter_transpose(n_el):
    rng = np.random.default_rng(2)
    n = int(np.prod(n_el))
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    assert np.isclose(adjoint.box_filter(x, n_el) @ y, x @ adjoint.box_filter_T(y, n_el), rtol=1e-12)
    assert np.allclose(adjoint.box_filter(np.full(n, 3.0), n_el), 3.0)


def test_box_filter_brute_force():
    n_el = (4, 3, 5)
    rng = np.random.default_rng(5)
    th = rng.standard_normal(60)
    out = adjoint.box_filter(th, n_el)
    t = th.reshape(5, 3, 4)
    for ez in range(5):
        for ey in range(3):
            for ex in range(4):
                vals = [t[z, y, x] for z in range(ez - 1, ez + 2) for y in range(ey - 1, ey + 2)
                        for x in range(ex - 1, ex + 2) if 0 <= z < 5 and 0 <= y < 3 and 0 <= x < 4]
                assert np.isclose(out[ex + 4 * (ey + 3 * ez)], np.mean(vals))


def test_gradient_central_differences():
    p = W.config5_like(n=6, H=3, L=3, cfg=23)
    theta = p.extra["theta"]
    u_obs, _ = adjoint.direct_solve(p.n_el, p.h, adjoint.rho_of_theta(p.extra["theta_obs"], p.n_el), p.f[0])
    L, g, _ = adjoint.loss_and_grad(theta, p.n_el, p.h, p.f[0], u_obs)
    dirs = W.fd_directions(23, 5, p.n_elements)
    for d in dirs:
        eps = 1e-5
        fd = (adjoint.loss(theta + eps * d, p.n_el, p.h, p.f[0], u_obs)
              - adjoint.loss(theta - eps * d, p.n_el, p.h, p.f[0], u_obs)) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-6 * max(abs(fd), 1e-12) + 1e-12


def test_element_grad_energy_identity():
    # sum_e -rho_e lambda_e^T K_e u_e = -lambda^T A u
    p = W.config5_like(n=5, H=5, L=5, cfg=24)
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.5, 2, p.n_elements)
    from oracle import q1
    A = q1.assemble(p.n_el, p.h, rho)
    u = rng.standard_normal(p.n_free)
    lam = rng.standard_normal(p.n_free)
    g = adjoint.element_grad(p.n_el, p.h, u, lam)
    assert np.isclose(rho @ g, -(lam @ (A @ u)), rtol=1e-12)
