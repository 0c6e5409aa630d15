"""Interface classification into subobjects (oracle; test infrastructure).

Section 3: the partition Theta = {Omega_i} has interface Gamma; a finer
partition Theta^ = {Omega^_j} (the subsubdomains) splits subdomain faces and
edges into subfaces, subedges and the vertices between them.  Remark 2 on
classification in Section 3 groups each interface degree of freedom by the
list of subsubdomains that contain it.  This module does exactly that:

* a free node belongs to subdomain i (resp. subsubdomain j) when one of its
  surrounding elements does;
* Gamma = free nodes that belong to two or more subdomains;
* key(xi) = the set of subsubdomains containing xi;
* an object is a connected set (grid-edge adjacency) of Gamma nodes with the
  same key;
* its type: in 3D a key of 2 subsubdomains is a face, 3-4 an edge, 5 or more
  a vertex; in 2D 2 is an edge and 3 or more a vertex (for tensor-product
  fine partitions these are exactly 1, 2, 3 cut planes through the node);
* the selected (primal) objects are those whose type is in ``primal_mask``
  (1 = v, 2 = e, 4 = f; 7 = "vef", every object); they are numbered by their
  smallest global free-node index, which is the coarse numbering.
* bit 8 of ``primal_mask`` keeps only half of the codimension-one objects
  (faces in 3D, edges in 2D: the keys of two subsubdomains), the "half of
  the face constraints" of Section 5.1's vf-min selection (mask 1 | 4 | 8).
  The paper does not say which half; here it is a checkerboard over the
  fine partition: index each subsubdomain along each axis by the rank of its
  lowest element coordinate among all subsubdomains' lowest coordinates
  along that axis; a face between j1 < j2 is kept when the sum of j1's
  indices along the axes other than the face normal (the axis along which
  j1 and j2 differ most) is even.  On a tensor fine partition neighbouring
  faces of one interface plane then alternate.

Weights, eq. (W) and Remark 4: for a Gamma node xi and a subdomain i that
contains it, delta_i(xi) = sum of alpha_j over the subsubdomains j of key(xi)
that lie in Omega_i, divided by the sum of alpha_j over all of key(xi).  With
alpha_j = 1 this is eq. (W) (card ratio); with alpha_j = the coefficient on
Omega^_j it is Remark 4.  Where rho is not constant on a subsubdomain the
mean of rho over its elements is used.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from .q1 import Grid

TYPE_V, TYPE_E, TYPE_F = 1, 2, 4
HALF_CODIM1 = 8


@dataclasses.dataclass
class Classification:
    n_free: int
    n_sub: int
    node_subs: List[np.ndarray]        # per free node: sorted subdomain ids (only Gamma nodes kept > 1)
    is_gamma: np.ndarray               # bool [n_free]
    obj_nodes: List[np.ndarray]        # per object: sorted global free ids
    obj_key: List[tuple]               # per object: sorted subsubdomain ids
    obj_subs: List[np.ndarray]         # per object: sorted subdomain ids
    obj_type: np.ndarray               # TYPE_V / TYPE_E / TYPE_F
    node_obj: np.ndarray               # int [n_free], object id of Gamma nodes, -1 elsewhere
    coarse_objects: np.ndarray         # object ids of the selected objects, in coarse order
    sub_nodes: List[np.ndarray]        # per subdomain: sorted global free ids of its closure
    node_keys: Dict[int, tuple]        # Gamma node -> key
    subsub_parent: np.ndarray          # subsubdomain -> subdomain

    @property
    def n_coarse(self) -> int:
        return len(self.coarse_objects)

    def counts_by_type(self, selected_only: bool = True) -> Dict[str, int]:
        ids = self.coarse_objects if selected_only else np.arange(len(self.obj_nodes))
        t = self.obj_type[ids]
        return {"v": int(np.sum(t == TYPE_V)), "e": int(np.sum(t == TYPE_E)),
                "f": int(np.sum(t == TYPE_F))}


def object_type(dim: int, key_size: int) -> int:
    if dim == 3:
        if key_size == 2:
            return TYPE_F
        if key_size <= 4:
            return TYPE_E
        return TYPE_V
    return TYPE_E if key_size == 2 else TYPE_V


def _row_unique(a: np.ndarray) -> np.ndarray:
    """Sort each row and replace repeated values by -1, then sort again."""
    s = np.sort(a, axis=1)
    dup = np.zeros_like(s, dtype=bool)
    dup[:, 1:] = s[:, 1:] == s[:, :-1]
    s = np.where(dup, -1, s)
    return np.sort(s, axis=1)


def classify(n_el, elem_sub, elem_subsub, primal_mask: int = 7) -> Classification:
    g = Grid(n_el)
    elem_sub = np.asarray(elem_sub, dtype=np.int64)
    elem_subsub = np.asarray(elem_subsub, dtype=np.int64)
    n_sub = int(elem_sub.max()) + 1
    n_ss = int(elem_subsub.max()) + 1
    parent = np.full(n_ss, -1, dtype=np.int64)
    parent[elem_subsub] = elem_sub
    if np.any(parent[elem_subsub] != elem_sub):
        raise ValueError("a subsubdomain spans more than one subdomain")

    ne = g.node_elements()                           # [n_free, 2^d]
    subs = _row_unique(elem_sub[ne])
    keys = _row_unique(elem_subsub[ne])
    n_subs_per_node = np.sum(subs >= 0, axis=1)
    is_gamma = n_subs_per_node >= 2

    node_subs = [row[row >= 0] for row in subs]

    # group Gamma nodes by key, then split each group into connected pieces
    gamma_ids = np.nonzero(is_gamma)[0]
    _, key_id = np.unique(keys[gamma_ids], axis=0, return_inverse=True)
    key_id = key_id.reshape(-1)
    key_of_node = np.full(g.n_free, -1, dtype=np.int64)
    key_of_node[gamma_ids] = key_id
    fc = g.free_coords()
    rows, cols = [], []
    for d in range(g.dim):
        nb = fc.copy()
        nb[:, d] += 1
        nbi = g.free_index(nb)
        ok = is_gamma & (nbi >= 0)
        ok[ok] &= is_gamma[nbi[ok]]
        ok[ok] &= key_of_node[nbi[ok]] == key_of_node[ok]
        rows.append(np.nonzero(ok)[0])
        cols.append(nbi[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    adj = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(g.n_free, g.n_free))
    _, comp = connected_components(adj, directed=False)
    # components of Gamma nodes -> objects numbered by smallest node id
    gcomp = comp[gamma_ids]
    uniq, first = np.unique(gcomp, return_index=True)
    order = np.argsort(gamma_ids[first])
    comp_to_obj = np.full(comp.max() + 1, -1, dtype=np.int64)
    comp_to_obj[uniq[order]] = np.arange(len(uniq))
    node_obj = np.full(g.n_free, -1, dtype=np.int64)
    node_obj[gamma_ids] = comp_to_obj[gcomp]
    n_obj = len(uniq)

    sort_idx = np.argsort(node_obj[gamma_ids], kind="stable")
    sorted_nodes = gamma_ids[sort_idx]
    bounds = np.searchsorted(node_obj[sorted_nodes], np.arange(n_obj + 1))
    obj_nodes = [np.sort(sorted_nodes[bounds[o]:bounds[o + 1]]) for o in range(n_obj)]
    obj_key, obj_subs, obj_type = [], [], np.empty(n_obj, dtype=np.int64)
    for o, nodes in enumerate(obj_nodes):
        k = keys[nodes[0]]
        k = tuple(int(v) for v in k[k >= 0])
        obj_key.append(k)
        obj_subs.append(np.unique(parent[list(k)]))
        obj_type[o] = object_type(g.dim, len(k))
    keep = np.array([bool(obj_type[o] & primal_mask) for o in range(n_obj)], dtype=bool)
    if primal_mask & HALF_CODIM1:
        idx = subsub_grid_index(g, elem_subsub, n_ss)
        for o in range(n_obj):
            if keep[o] and len(obj_key[o]) == 2:
                keep[o] = checkerboard_even(idx, obj_key[o])
    selected = np.nonzero(keep)[0].astype(np.int64)
    # objects are already numbered by smallest node id, so selection keeps that order
    # closure of each subdomain: free nodes having subdomain i in their list
    flat_nodes = np.repeat(np.arange(g.n_free), subs.shape[1])
    flat_subs = subs.reshape(-1)
    keep = flat_subs >= 0
    flat_nodes, flat_subs = flat_nodes[keep], flat_subs[keep]
    o = np.lexsort((flat_nodes, flat_subs))
    flat_nodes, flat_subs = flat_nodes[o], flat_subs[o]
    sb = np.searchsorted(flat_subs, np.arange(n_sub + 1))
    sub_nodes = [flat_nodes[sb[i]:sb[i + 1]] for i in range(n_sub)]
    node_keys = {int(n): tuple(int(v) for v in keys[n][keys[n] >= 0]) for n in gamma_ids}
    return Classification(g.n_free, n_sub, node_subs, is_gamma, obj_nodes, obj_key,
                          obj_subs, obj_type, node_obj, selected, sub_nodes, node_keys,
                          parent)


def subsub_grid_index(g: Grid, elem_subsub: np.ndarray, n_ss: int) -> np.ndarray:
    """[n_ss, dim]: per axis, the rank of each subsubdomain's lowest element
    coordinate among the distinct lowest coordinates of all subsubdomains."""
    ec = g.element_coords()
    idx = np.empty((n_ss, g.dim), dtype=np.int64)
    for a in range(g.dim):
        lo = np.full(n_ss, np.iinfo(np.int64).max, dtype=np.int64)
        np.minimum.at(lo, elem_subsub, ec[:, a])
        _, idx[:, a] = np.unique(lo, return_inverse=True)
    return idx


def checkerboard_even(idx: np.ndarray, key: tuple) -> bool:
    """The half-selection rule for a codimension-one object between the two
    subsubdomains of key (see the module docstring)."""
    j1, j2 = key
    diff = np.abs(idx[j1] - idx[j2])
    normal = int(np.argmax(diff))
    s = int(np.sum(idx[j1])) - int(idx[j1][normal])
    return s % 2 == 0


def subsub_alpha(elem_subsub, rho, weighting: int) -> np.ndarray:
    """alpha_j per subsubdomain: 1 (eq. W) or the mean of rho over it (Remark 4)."""
    elem_subsub = np.asarray(elem_subsub, dtype=np.int64)
    n_ss = int(elem_subsub.max()) + 1
    if weighting == 0:
        return np.ones(n_ss)
    s = np.bincount(elem_subsub, weights=np.asarray(rho, dtype=float), minlength=n_ss)
    c = np.bincount(elem_subsub, minlength=n_ss)
    return s / c


def weight(cls: Classification, alpha: np.ndarray, node: int, sub: int) -> float:
    """delta_sub(node), eq. (W) / Remark 4; 1 for nodes inside one subdomain."""
    if not cls.is_gamma[node]:
        return 1.0
    key = cls.node_keys[int(node)]
    num = sum(alpha[j] for j in key if cls.subsub_parent[j] == sub)
    den = sum(alpha[j] for j in key)
    return float(num / den)
