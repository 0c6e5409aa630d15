"""The BDDC-SO preconditioner assembled from its definition (oracle; test
infrastructure; tiny meshes only).

Definition 1 with V1 = U_I, V2 = W~, Q1 = I, Q2 = (I - P) E (Section 3):

    B = R_I^T A_II^{-1} R_I + M A~^{-1} M^T,

with Z a basis of W~ (the null space of the jumps of every selected coarse
functional between the subdomains sharing its object), A~ = Z^T diag(K_i) Z,
M = (I - P) E Z, E the weighted average of eq. (W) / Remark 4, and (I - P)
the discrete-harmonic extension from Gamma: ((I-P)u)_Gamma = u_Gamma,
((I-P)u)_I = -A_II^{-1} A_I,Gamma u_Gamma.  Nothing here eliminates
vertices, builds coarse basis functions or a coarse matrix, so it pins the
step-by-step ``bddc`` module from a different direction.

The BDDC-A operator of Section 4 is built the same way on the fine partition
Theta^ (full continuity on Gamma^ minus Gamma, the selected subobjects on
Gamma, counting weights of eq. (W2)), for the bound of Theorem 3.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import q1
from .classify import classify, subsub_alpha, weight


def _local_dense(grid, Ke, rho, elements, nodes):
    efn = grid.element_free_nodes()[elements]
    n = len(nodes)
    K = np.zeros((n, n))
    pos = {int(v): k for k, v in enumerate(nodes)}
    for e, row in zip(elements, efn):
        loc = [pos.get(int(v), -1) if v >= 0 else -1 for v in row]
        for a, la in enumerate(loc):
            if la < 0:
                continue
            for b, lb in enumerate(loc):
                if lb >= 0:
                    K[la, lb] += rho[e] * Ke[a, b]
    return K


def bddc_dense(n_el, h, elem_sub, elem_subsub, rho, primal_mask=7, weighting=1,
               return_parts=False):
    grid = q1.Grid(n_el)
    N = grid.n_free
    rho = np.asarray(rho, dtype=float)
    elem_sub = np.asarray(elem_sub)
    cls = classify(n_el, elem_sub, elem_subsub, primal_mask)
    alpha = subsub_alpha(elem_subsub, rho, weighting)
    Ke = q1.element_matrix(grid.dim, h)
    A = q1.assemble(n_el, h, rho).toarray()

    # W = W_1 x ... x W_N: concatenated local node sets
    offs = [0]
    Ks = []
    for i in range(cls.n_sub):
        nodes = cls.sub_nodes[i]
        Ks.append(_local_dense(grid, Ke, rho, np.nonzero(elem_sub == i)[0], nodes))
        offs.append(offs[-1] + len(nodes))
    nW = offs[-1]
    Kblk = sla.block_diag(*Ks)

    def functional(o, i):
        """Row vector on W evaluating object o's coarse functional on w_i."""
        row = np.zeros(nW)
        nodes = cls.sub_nodes[i]
        onodes = cls.obj_nodes[o]
        li = np.searchsorted(nodes, onodes)
        row[offs[i] + li] = 1.0 / len(onodes)
        return row

    J = []
    for o in cls.coarse_objects:
        subs = cls.obj_subs[o]
        for s in subs[1:]:
            J.append(functional(o, subs[0]) - functional(o, s))
    J = np.array(J) if J else np.zeros((0, nW))
    Z = sla.null_space(J) if len(J) else np.eye(nW)
    At = Z.T @ Kblk @ Z

    E = np.zeros((N, nW))
    for i in range(cls.n_sub):
        for k, v in enumerate(cls.sub_nodes[i]):
            E[v, offs[i] + k] = weight(cls, alpha, v, i)
    I = np.nonzero(~cls.is_gamma)[0]
    G = np.nonzero(cls.is_gamma)[0]
    H = np.zeros((N, N))  # (I - P) on U
    H[G, G] = 1.0
    H[np.ix_(I, G)] = -np.linalg.solve(A[np.ix_(I, I)], A[np.ix_(I, G)])
    M = H @ E @ Z
    B = M @ np.linalg.solve(At, M.T)
    RI = np.zeros((len(I), N))
    RI[np.arange(len(I)), I] = 1.0
    B += RI.T @ np.linalg.solve(A[np.ix_(I, I)], RI)
    if return_parts:
        return B, {"A": A, "Z": Z, "E": E, "cls": cls, "Kblk": Kblk, "offs": offs, "H": H}
    return B


def bddc_a_dense(n_el, h, elem_sub, elem_subsub, rho, primal_mask=7):
    """BDDC-A (Section 4): BDDC on the subsubdomains, with the selected
    subobjects as coarse functionals on Gamma, every node of Gamma^ \\ Gamma
    fully continuous, and counting weights (eq. W2)."""
    grid = q1.Grid(n_el)
    N = grid.n_free
    rho = np.asarray(rho, dtype=float)
    elem_subsub = np.asarray(elem_subsub)
    cls = classify(n_el, elem_sub, elem_subsub, primal_mask)   # subobjects on Gamma
    fine = classify(n_el, elem_subsub, elem_subsub, 0)         # nodes of Gamma^
    n_ss = int(elem_subsub.max()) + 1
    Ke = q1.element_matrix(grid.dim, h)
    A = q1.assemble(n_el, h, rho).toarray()
    offs = [0]
    Ks = []
    for j in range(n_ss):
        nodes = fine.sub_nodes[j]
        Ks.append(_local_dense(grid, Ke, rho, np.nonzero(elem_subsub == j)[0], nodes))
        offs.append(offs[-1] + len(nodes))
    nW = offs[-1]
    Kblk = sla.block_diag(*Ks)

    def value_row(j, v, scale=1.0):
        row = np.zeros(nW)
        row[offs[j] + np.searchsorted(fine.sub_nodes[j], v)] = scale
        return row

    J = []
    # full continuity at every node of Gamma^ that is not on Gamma
    for v in np.nonzero(fine.is_gamma & ~cls.is_gamma)[0]:
        ss = fine.node_subs[v]
        for s in ss[1:]:
            J.append(value_row(ss[0], v) - value_row(s, v))
    # the selected subobjects on Gamma
    for o in cls.coarse_objects:
        onodes = cls.obj_nodes[o]
        key = cls.obj_key[o]
        rows = []
        for j in key:
            row = np.zeros(nW)
            row[offs[j] + np.searchsorted(fine.sub_nodes[j], onodes)] = 1.0 / len(onodes)
            rows.append(row)
        for rrow in rows[1:]:
            J.append(rows[0] - rrow)
    J = np.array(J)
    Z = sla.null_space(J)
    At = Z.T @ Kblk @ Z
    E = np.zeros((N, nW))
    for j in range(n_ss):
        for k, v in enumerate(fine.sub_nodes[j]):
            E[v, offs[j] + k] = 1.0 / len(fine.node_subs[v])
    I = np.nonzero(~fine.is_gamma)[0]
    G = np.nonzero(fine.is_gamma)[0]
    H = np.zeros((N, N))
    H[G, G] = 1.0
    H[np.ix_(I, G)] = -np.linalg.solve(A[np.ix_(I, I)], A[np.ix_(I, G)])
    M = H @ E @ Z
    B = M @ np.linalg.solve(At, M.T)
    RI = np.zeros((len(I), N))
    RI[np.arange(len(I)), I] = 1.0
    B += RI.T @ np.linalg.solve(A[np.ix_(I, I)], RI)
    return B
