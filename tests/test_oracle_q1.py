"""Pins of the oracle's Q1 element matrices and assembly (CPU)."""
import numpy as np
import pytest

import workloads as W
from oracle import q1


def test_element_matrix_2d_closed_form():
    # Bilinear square: diagonal 2/3, edge neighbours -1/6, diagonal neighbour -1/3.
    K = q1.element_matrix(2, 0.37)
    assert np.allclose(np.diag(K), 2.0 / 3.0)
    assert np.isclose(K[0, 1], -1.0 / 6.0) and np.isclose(K[0, 2], -1.0 / 6.0)
    assert np.isclose(K[0, 3], -1.0 / 3.0)
    assert np.allclose(K, K.T)


def test_element_matrix_3d_closed_form():
    # Trilinear cube of side h: h*{1/3 diagonal, 0 edge, -1/12 face diagonal, -1/12 body diagonal}.
    h = 0.25
    K = q1.element_matrix(3, h)
    off = q1.element_offsets(3)
    for a in range(8):
        for b in range(8):
            d = int(np.sum(off[a] != off[b]))
            expect = {0: 1.0 / 3.0, 1: 0.0, 2: -1.0 / 12.0, 3: -1.0 / 12.0}[d]
            assert np.isclose(K[a, b], h * expect), (a, b)


@pytest.mark.parametrize("dim", [2, 3])
def test_constants_in_kernel(dim):
    K = q1.element_matrix(dim, [0.1, 0.2, 0.3][:dim])
    assert np.allclose(K @ np.ones(2 ** dim), 0.0, atol=1e-14)
    ev = np.linalg.eigvalsh(K)
    assert ev[0] > -1e-14 and np.sum(ev > 1e-12) == 2 ** dim - 1


@pytest.mark.parametrize("n_el", [(7, 5), (5, 4, 6)])
def test_energy_matches_quadrature(n_el):
    # x^T A x equals the Gauss-quadrature energy of the interpolant (independent code path).
    rng = np.random.default_rng(3)
    g = q1.Grid(n_el)
    rho = rng.uniform(0.1, 10.0, g.n_elements)
    h = [1.0 / n for n in n_el]
    A = q1.assemble(n_el, h, rho)
    for _ in range(3):
        x = rng.standard_normal(g.n_free)
        assert np.isclose(x @ (A @ x), q1.energy_by_quadrature(n_el, h, rho, x), rtol=1e-12)


def test_3d_stencil_has_no_axis_coupling():
    # Trilinear Laplacian: no coupling between axis neighbours, whatever rho is.
    n_el = (6, 6, 6)
    g = q1.Grid(n_el)
    rho = np.random.default_rng(0).uniform(0.5, 2.0, g.n_elements)
    A = q1.assemble(n_el, [1 / 6] * 3, rho).tocsr()
    c = g.free_index(np.array([3, 3, 3]))
    for d in range(3):
        nb = np.array([3, 3, 3])
        nb[d] += 1
        assert A[c, g.free_index(nb)] == 0.0
    assert np.count_nonzero(A[c].toarray()) == 1 + 12 + 8


def test_assembly_symmetric_positive_definite():
    p = W.config1_like(n=8, H=4, L=2)
    A = q1.assemble(p.n_el, p.h, p.rho).toarray()
    assert np.allclose(A, A.T)
    assert np.linalg.eigvalsh(A)[0] > 0
