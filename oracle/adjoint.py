"""Gradient of a least-squares loss through the solve (oracle; test
infrastructure).

Parameterisation (readings of the adjoint workload): theta is a raw
per-element log-coefficient; theta~ = F theta with F the 3x3x3 (3x3 in 2D)
box mean over the in-domain neighbours of each element, normalised by their
count; rho = exp(theta~).  The loss is L = 1/2 ||u - u_obs||^2 with
A(rho) u = f.

Calculus (A symmetric): lambda = A^{-1} (u - u_obs); dL/drho_e =
-lambda_e^T K^_e u_e with K^_e the unit-coefficient element matrix and
lambda_e, u_e the element's nodal values (zero at boundary nodes);
dL/dtheta~_e = rho_e dL/drho_e; dL/dtheta = F^T dL/dtheta~.

All solves here are direct sparse solves of the assembled matrix.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse.linalg as spla

from . import q1


def box_filter(theta: np.ndarray, n_el) -> np.ndarray:
    """Mean of theta over the in-domain (3^dim)-neighbourhood of each element."""
    dim = len(n_el)
    t = np.asarray(theta, dtype=float).reshape(tuple(reversed(n_el)))
    acc = np.zeros_like(t)
    cnt = np.zeros_like(t)
    for off in itertools.product((-1, 0, 1), repeat=dim):
        src = [slice(None)] * dim
        dst = [slice(None)] * dim
        ok = True
        for ax, o in enumerate(off):
            n = t.shape[ax]
            if o == -1:
                dst[ax], src[ax] = slice(1, n), slice(0, n - 1)
            elif o == 1:
                dst[ax], src[ax] = slice(0, n - 1), slice(1, n)
            if n == 1 and o != 0:
                ok = False
        if not ok:
            continue
        acc[tuple(dst)] += t[tuple(src)]
        cnt[tuple(dst)] += 1.0
    return (acc / cnt).reshape(-1)


def box_filter_T(g: np.ndarray, n_el) -> np.ndarray:
    """Transpose of ``box_filter``: sum over the neighbourhood of g_e / count_e."""
    dim = len(n_el)
    shape = tuple(reversed(n_el))
    ones = np.ones(int(np.prod(n_el)))
    # count_e = number of in-domain neighbours, from the filter of ones times count
    cnt = np.zeros(shape)
    t1 = ones.reshape(shape)
    for off in itertools.product((-1, 0, 1), repeat=dim):
        src = [slice(None)] * dim
        dst = [slice(None)] * dim
        for ax, o in enumerate(off):
            n = shape[ax]
            if o == -1:
                dst[ax], src[ax] = slice(1, n), slice(0, n - 1)
            elif o == 1:
                dst[ax], src[ax] = slice(0, n - 1), slice(1, n)
        cnt[tuple(dst)] += t1[tuple(src)]
    w = np.asarray(g, dtype=float).reshape(shape) / cnt
    out = np.zeros(shape)
    for off in itertools.product((-1, 0, 1), repeat=dim):
        src = [slice(None)] * dim
        dst = [slice(None)] * dim
        for ax, o in enumerate(off):
            n = shape[ax]
            if o == -1:
                dst[ax], src[ax] = slice(1, n), slice(0, n - 1)
            elif o == 1:
                dst[ax], src[ax] = slice(0, n - 1), slice(1, n)
        # out[src] += w[dst]: element src is a neighbour of element dst
        out[tuple(src)] += w[tuple(dst)]
    return out.reshape(-1)


def rho_of_theta(theta, n_el):
    return np.exp(box_filter(theta, n_el))


def direct_solve(n_el, h, rho, f):
    A = q1.assemble(n_el, h, rho).tocsc()
    return spla.spsolve(A, f), A


def element_grad(n_el, h, u, lam) -> np.ndarray:
    """-lambda_e^T K^_e u_e for every element (zero boundary values)."""
    g = q1.Grid(n_el)
    Ke = q1.element_matrix(g.dim, h)
    efn = g.element_free_nodes()
    ue = np.where(efn >= 0, u[np.maximum(efn, 0)], 0.0)
    le = np.where(efn >= 0, lam[np.maximum(efn, 0)], 0.0)
    return -np.einsum("ea,ab,eb->e", le, Ke, ue)


def loss_and_grad(theta, n_el, h, f, u_obs):
    """L(theta) and dL/dtheta by direct forward and adjoint solves."""
    rho = rho_of_theta(theta, n_el)
    u, A = direct_solve(n_el, h, rho, f)
    res = u - u_obs
    L = 0.5 * float(res @ res)
    lam = spla.spsolve(A, res)
    g_rho = element_grad(n_el, h, u, lam)
    g_theta_t = rho * g_rho
    return L, box_filter_T(g_theta_t, n_el), {"u": u, "lam": lam, "rho": rho}


def loss(theta, n_el, h, f, u_obs) -> float:
    rho = rho_of_theta(theta, n_el)
    u, _ = direct_solve(n_el, h, rho, f)
    res = u - u_obs
    return 0.5 * float(res @ res)
