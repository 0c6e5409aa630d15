"""BDDC-SO preconditioner, plain FP64 (oracle; test infrastructure).

Section 3 instantiates the multispace BDDC of Definition 1 with

    a = a^Theta,  V1 = U_I,  V2 = W~,  Q1 = I,  Q2 = (I - P) E,

where U_I are the functions vanishing on Gamma, P is the a^Theta-orthogonal
projection onto U_I, W~ is the subspace of W = W_1 x ... x W_N that is
continuous at the selected coarse degrees of freedom (values at, or averages
over, the selected subobjects), and E is the weighted average of eq. (W)
(Remark 4 with coefficients).  Definition 1 gives

    B r = v1 + (I - P) E v2,  a(v1, z) = <r, z> on U_I,
                               a^Theta(v2, z) = <r, (I - P) E z> on W~.

The steps below compute exactly this, one subdomain at a time:

 1. v1 = A_II^{-1} r_I (interior nodes belong to one subdomain).
 2. t = r_Gamma - A_Gamma,I v1, i.e. (I - P)^T r restricted to Gamma.
 3. g_i = D_i R_i t, i.e. E^T t (D_i = diag(delta_i) on Gamma_i, 1 inside).
 4.-7. v2 = argmin over W~ of 1/2 a^Theta(w, w) - <g, w>.  W~ splits
    a^Theta-orthogonally into the functions with all selected coarse
    functionals zero (independent per subdomain: a constrained Neumann
    problem) plus the span of the coarse basis Phi (energy-minimal local
    functions with unit coarse functional, Dohrmann's construction), so
    v2_i = v_Delta,i + Phi_i u_c with K_c u_c = sum_i R_ci^T Phi_i^T g_i and
    K_c = sum_i R_ci^T Phi_i^T K_i Phi_i R_ci.
 8. w = E v2 on Gamma.
 9.-10. z = v1 + (I - P) w: z_Gamma = w_Gamma and
    z_I = A_II^{-1} (r_I - A_I,Gamma w_Gamma).

Local constrained problems are solved through their full KKT systems
[K_i C_i^T; C_i 0] with every selected functional as a row of C_i (point
values and averages alike), by a sparse LU.  The coarse matrix is factored by
a dense Cholesky.  Both are library primitives used as single steps.

The averages are unweighted nodal means over an object's free nodes (the
paper only says "averages"; any fixed row scaling gives the same B).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import q1
from .classify import Classification, classify, subsub_alpha, weight


@dataclasses.dataclass
class Local:
    nodes: np.ndarray        # global free ids, sorted (local numbering)
    K: sp.csr_matrix         # local stiffness sum over this subdomain's elements
    interior: np.ndarray     # local indices of interior nodes
    gamma: np.ndarray        # local indices of Gamma nodes
    delta: np.ndarray        # weights on gamma (same order)
    coarse: np.ndarray       # global coarse ids of the local coarse dofs (ascending)
    C: sp.csr_matrix         # [n_c_local, n_local] selected functionals
    lu_II: object            # factorization of K_II
    lu_kkt: object           # factorization of [K C^T; C 0]
    Phi: np.ndarray          # [n_local, n_c_local] coarse basis
    Kc: np.ndarray           # [n_c_local, n_c_local] = Phi^T K Phi
    K_GI: sp.csr_matrix
    K_IG: sp.csr_matrix


def _local_matrix(grid: q1.Grid, Ke, rho, elements, nodes) -> sp.csr_matrix:
    efn = grid.element_free_nodes()[elements]
    loc = np.searchsorted(nodes, np.maximum(efn, 0))
    loc = np.where(efn >= 0, loc, -1)
    nl = Ke.shape[0]
    rows = np.repeat(loc, nl, axis=1)
    cols = np.tile(loc, (1, nl))
    vals = np.asarray(rho)[elements][:, None] * Ke.reshape(1, -1)
    keep = (rows >= 0) & (cols >= 0)
    n = len(nodes)
    return sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()


class BDDCSO:
    """Setup (local matrices, factorizations, coarse basis, coarse matrix) and
    application of the BDDC-SO preconditioner."""

    def __init__(self, n_el, h, elem_sub, elem_subsub, rho, primal_mask: int = 7,
                 weighting: int = 1, cls: Classification = None, local_only: bool = False):
        self.grid = q1.Grid(n_el)
        self.n_el = tuple(n_el)
        self.h = h
        self.rho = np.asarray(rho, dtype=np.float64)
        self.A = q1.assemble(n_el, h, self.rho)
        self.cls = cls if cls is not None else classify(n_el, elem_sub, elem_subsub, primal_mask)
        cls = self.cls
        self.alpha = subsub_alpha(elem_subsub, self.rho, weighting)
        Ke = q1.element_matrix(self.grid.dim, h)
        elem_sub = np.asarray(elem_sub)
        order = np.argsort(elem_sub, kind="stable")
        bounds = np.searchsorted(elem_sub[order], np.arange(cls.n_sub + 1))

        # which selected objects touch which subdomain
        coarse_of_obj = -np.ones(len(cls.obj_nodes), dtype=np.int64)
        coarse_of_obj[cls.coarse_objects] = np.arange(cls.n_coarse)
        sub_coarse: List[list] = [[] for _ in range(cls.n_sub)]
        for c, o in enumerate(cls.coarse_objects):
            for s in cls.obj_subs[o]:
                sub_coarse[s].append(c)

        self.sub_coarse = sub_coarse
        self._Ke = Ke
        self._elem_order = (order, bounds)
        self.locals: List[Local] = []
        if local_only:
            return
        # K_c = sum_i R_ci^T K_c,i R_ci, assembled sparse (each coarse dof
        # couples only to those of its subdomains) and factored exactly
        rows, cols, vals = [], [], []
        for i in range(cls.n_sub):
            L = self.local(i)
            r, c = np.meshgrid(L.coarse, L.coarse, indexing="ij")
            rows.append(r.reshape(-1))
            cols.append(c.reshape(-1))
            vals.append(L.Kc.reshape(-1))
            self.locals.append(L)
        nc = cls.n_coarse
        if nc:
            self.Kc = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                    shape=(nc, nc)).tocsc()
            self.Kc_solve = spla.factorized(self.Kc)
        else:
            self.Kc = sp.csc_matrix((0, 0))
            self.Kc_solve = None

    def local(self, i: int) -> Local:
        """Setup of subdomain i alone: K_i, K_II factor, constrained Neumann
        KKT factor, coarse basis Phi_i and Phi_i^T K_i Phi_i (Section 3)."""
        cls = self.cls
        order, bounds = self._elem_order
        nodes = cls.sub_nodes[i]
        elements = order[bounds[i]:bounds[i + 1]]
        K = _local_matrix(self.grid, self._Ke, self.rho, elements, nodes)
        gmask = cls.is_gamma[nodes]
        interior = np.nonzero(~gmask)[0]
        gamma = np.nonzero(gmask)[0]
        delta = np.array([weight(cls, self.alpha, nodes[k], i) for k in gamma])
        coarse = np.array(sorted(self.sub_coarse[i]), dtype=np.int64)
        # one row per selected functional: value at a node or mean over an object
        rows, cols, vals = [], [], []
        for a, c in enumerate(coarse):
            onodes = cls.obj_nodes[cls.coarse_objects[c]]
            li = np.searchsorted(nodes, onodes)
            rows.extend([a] * len(li))
            cols.extend(li.tolist())
            vals.extend([1.0 / len(li)] * len(li))
        nc = len(coarse)
        n = len(nodes)
        C = sp.coo_matrix((vals, (rows, cols)), shape=(nc, n)).tocsr()
        K_II = K[interior][:, interior].tocsc()
        lu_II = spla.splu(K_II) if len(interior) else None
        kkt = sp.bmat([[K, C.T], [C, None]]).tocsc()
        lu_kkt = spla.splu(kkt)
        # coarse basis: min energy with C Phi = I (one column per local coarse dof)
        rhs = np.zeros((n + nc, nc))
        rhs[n:, :] = np.eye(nc)
        Phi = lu_kkt.solve(rhs)[:n, :] if nc else np.zeros((n, 0))
        Kc_i = Phi.T @ (K @ Phi)
        return Local(nodes, K, interior, gamma, delta, coarse, C, lu_II, lu_kkt, Phi, Kc_i,
                     K[gamma][:, interior].tocsr(), K[interior][:, gamma].tocsr())

    # ------------------------------------------------------------------
    def apply(self, r: np.ndarray, return_parts: bool = False):
        """z = B r, Definition 1 with the Section 3 choices (steps 1-10)."""
        r = np.asarray(r, dtype=np.float64)
        N = self.grid.n_free
        cls = self.cls
        # steps 1-2
        t = np.where(cls.is_gamma, r, 0.0)
        v1 = np.zeros(N)
        for L in self.locals:
            if len(L.interior) == 0:
                continue
            yI = L.lu_II.solve(r[L.nodes[L.interior]])
            v1[L.nodes[L.interior]] = yI
            np.subtract.at(t, L.nodes[L.gamma], L.K_GI @ yI)
        # steps 3-5
        bc = np.zeros(cls.n_coarse)
        vdelta = []
        for L in self.locals:
            n = len(L.nodes)
            g = np.zeros(n)
            g[L.gamma] = L.delta * t[L.nodes[L.gamma]]
            sol = L.lu_kkt.solve(np.concatenate([g, np.zeros(len(L.coarse))]))
            vdelta.append(sol[:n])
            bc[L.coarse] += L.Phi.T @ g
        # step 6
        uc = self.Kc_solve(bc) if cls.n_coarse else bc
        # steps 7-8
        w = np.zeros(N)
        for L, vd in zip(self.locals, vdelta):
            v2 = vd + L.Phi @ uc[L.coarse]
            np.add.at(w, L.nodes[L.gamma], L.delta * v2[L.gamma])
        # steps 9-10
        z = np.where(cls.is_gamma, w, 0.0)
        for L in self.locals:
            if len(L.interior) == 0:
                continue
            rhs = r[L.nodes[L.interior]] - L.K_IG @ w[L.nodes[L.gamma]]
            z[L.nodes[L.interior]] = L.lu_II.solve(rhs)
        if return_parts:
            return z, {"t": t, "bc": bc, "uc": uc, "w": w, "v1": v1}
        return z

    def dense(self) -> np.ndarray:
        """B as a dense matrix (tiny problems): B applied to the unit vectors."""
        N = self.grid.n_free
        return np.column_stack([self.apply(np.eye(N)[:, k]) for k in range(N)])


def from_problem(p, **kw) -> BDDCSO:
    return BDDCSO(p.n_el, p.h, p.elem_sub, p.elem_subsub, p.rho,
                  primal_mask=kw.pop("primal_mask", p.primal_mask),
                  weighting=kw.pop("weighting", p.weighting), **kw)
