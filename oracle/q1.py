"""Q1 finite elements on a structured grid (oracle; test infrastructure).

Model problem, Section 2: -div(alpha grad u) = f with zero Dirichlet data on
the whole boundary; the bilinear form is a(u, v) = sum_e alpha_e int_e grad u .
grad v (Remark 4 for the per-element coefficient).  The paper's experiments
use hexahedra (Section 5), so the space is bi/trilinear Q1.

The element stiffness matrix of a Q1 box is the tensor sum of 1D stiffness
and mass matrices; that is its definition written out (the integral of the
gradient product factorises per axis).  Local element node (a, b[, c]) with
a, b, c in {0, 1} has index a + 2 b + 4 c (x fastest).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def stiffness_1d(h: float) -> np.ndarray:
    """int_0^h phi_a' phi_b' for the two linear hat functions."""
    return np.array([[1.0, -1.0], [-1.0, 1.0]]) / h


def mass_1d(h: float) -> np.ndarray:
    """int_0^h phi_a phi_b for the two linear hat functions."""
    return h * np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0


def element_matrix(dim: int, h) -> np.ndarray:
    """Unit-coefficient Q1 stiffness matrix of one box element.

    For a tensor-product basis phi(x)phi(y)phi(z) the integral of
    grad u . grad v is K_x (x) M_y (x) M_z + M_x (x) K_y (x) M_z
    + M_x (x) M_y (x) K_z.  ``np.kron`` puts its first factor slowest, so the
    z factor comes first to keep x fastest in the local numbering.
    """
    h = [float(v) for v in np.broadcast_to(np.asarray(h, dtype=float), (dim,))]
    K = [stiffness_1d(v) for v in h]
    M = [mass_1d(v) for v in h]
    if dim == 2:
        return np.kron(M[1], K[0]) + np.kron(K[1], M[0])
    if dim == 3:
        return (np.kron(M[2], np.kron(M[1], K[0])) + np.kron(M[2], np.kron(K[1], M[0]))
                + np.kron(K[2], np.kron(M[1], M[0])))
    raise ValueError("dim must be 2 or 3")


def element_offsets(dim: int) -> np.ndarray:
    """Grid offsets (dx, dy[, dz]) of the local element nodes, index a+2b+4c."""
    return np.array([[(l >> d) & 1 for d in range(dim)] for l in range(2 ** dim)])


class Grid:
    """Index bookkeeping for a structured mesh with Dirichlet boundary."""

    def __init__(self, n_el):
        self.n_el = tuple(int(n) for n in n_el)
        self.dim = len(self.n_el)
        self.n_nodes_axis = tuple(n + 1 for n in self.n_el)
        self.n_free_axis = tuple(n - 1 for n in self.n_el)
        self.n_elements = int(np.prod(self.n_el))
        self.n_free = int(np.prod(self.n_free_axis))

    def element_coords(self) -> np.ndarray:
        """[n_elements, dim] element grid coordinates (x fastest numbering)."""
        idx = np.arange(self.n_elements)
        out = np.empty((self.n_elements, self.dim), dtype=np.int64)
        for d in range(self.dim):
            out[:, d] = idx % self.n_el[d]
            idx = idx // self.n_el[d]
        return out

    def free_coords(self) -> np.ndarray:
        """[n_free, dim] grid coordinates (1..n-1) of the free nodes."""
        idx = np.arange(self.n_free)
        out = np.empty((self.n_free, self.dim), dtype=np.int64)
        for d in range(self.dim):
            out[:, d] = idx % self.n_free_axis[d] + 1
            idx = idx // self.n_free_axis[d]
        return out

    def free_index(self, coords: np.ndarray) -> np.ndarray:
        """Free-node index of grid coordinates, -1 for boundary nodes."""
        coords = np.asarray(coords)
        ok = np.ones(coords.shape[:-1], dtype=bool)
        idx = np.zeros(coords.shape[:-1], dtype=np.int64)
        stride = 1
        for d in range(self.dim):
            c = coords[..., d]
            ok &= (c >= 1) & (c <= self.n_el[d] - 1)
            idx += (c - 1) * stride
            stride *= self.n_free_axis[d]
        return np.where(ok, idx, -1)

    def element_free_nodes(self) -> np.ndarray:
        """[n_elements, 2^dim] free index of each element's nodes (-1 = boundary)."""
        ec = self.element_coords()
        off = element_offsets(self.dim)
        return self.free_index(ec[:, None, :] + off[None, :, :])

    def node_elements(self) -> np.ndarray:
        """[n_free, 2^dim] the elements around each free node.

        A free node is interior, so all 2^dim surrounding elements exist.
        Column l holds the element whose local node l is this node.
        """
        fc = self.free_coords()
        off = element_offsets(self.dim)
        ec = fc[:, None, :] - off[None, :, :]
        idx = np.zeros(ec.shape[:-1], dtype=np.int64)
        stride = 1
        for d in range(self.dim):
            idx += ec[..., d] * stride
            stride *= self.n_el[d]
        return idx


def assemble(n_el, h, rho, elements=None) -> sp.csr_matrix:
    """Global stiffness matrix over the free nodes: sum_e rho_e K_e.

    ``elements`` restricts the sum to a subset of elements (used for the
    local matrices K_i of Section 3); the result is still indexed by global
    free-node numbers.
    """
    g = Grid(n_el)
    Ke = element_matrix(g.dim, h)
    efn = g.element_free_nodes()
    rho = np.asarray(rho, dtype=np.float64)
    if elements is not None:
        efn = efn[elements]
        rho = rho[elements]
    nloc = Ke.shape[0]
    rows = np.repeat(efn, nloc, axis=1)                # [E, nloc*nloc], row = node a
    cols = np.tile(efn, (1, nloc))                     # col = node b
    vals = rho[:, None] * Ke.reshape(1, -1)
    keep = (rows >= 0) & (cols >= 0)
    A = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(g.n_free, g.n_free))
    return A.tocsr()


def energy_by_quadrature(n_el, h, rho, x: np.ndarray) -> float:
    """sum_e rho_e int_e |grad x_h|^2 with a 2^dim-point Gauss rule.

    Independent of ``element_matrix``: it evaluates gradients of the
    bilinear/trilinear shape functions at Gauss points.  Used to pin the
    assembled matrix through x^T A x.
    """
    g = Grid(n_el)
    dim = g.dim
    hv = np.broadcast_to(np.asarray(h, dtype=float), (dim,))
    efn = g.element_free_nodes()
    xe = np.where(efn >= 0, x[np.maximum(efn, 0)], 0.0)  # [E, 2^dim]
    off = element_offsets(dim)
    gp = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    total = np.zeros(g.n_elements)
    for q in np.ndindex(*(2,) * dim):
        xi = gp[list(q)]
        grad = np.zeros((g.n_elements, dim))
        for l in range(2 ** dim):
            for d in range(dim):
                dphi = 1.0 / hv[d] * (1.0 if off[l, d] else -1.0)
                for e in range(dim):
                    if e != d:
                        dphi *= xi[e] if off[l, e] else (1.0 - xi[e])
                grad[:, d] += dphi * xe[:, l]
        w = np.prod(hv) / 2 ** dim
        total += w * np.sum(grad * grad, axis=1)
    return float(np.dot(np.asarray(rho, dtype=float), total))
