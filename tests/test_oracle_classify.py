"""Pins of the oracle's subobject classification and weights (CPU)."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from conftest import golden_path
from oracle import classify, q1


def _read_golden(name):
    rows = []
    with open(golden_path(name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


def test_fig1_subobjects_and_weights():
    """Figure 1 right panel: 8 subedges and 5 vertices; eq. (W) example values."""
    p = W.fig1_problem()
    c = classify.classify(p.n_el, p.elem_sub, p.elem_subsub)
    g = q1.Grid(p.n_el)
    alpha = classify.subsub_alpha(p.elem_subsub, p.rho, 0)
    counts = c.counts_by_type(selected_only=False)
    verts = set()
    for o in range(len(c.obj_nodes)):
        if c.obj_type[o] == classify.TYPE_V:
            assert len(c.obj_nodes[o]) == 1
            verts.add(tuple(g.free_coords()[c.obj_nodes[o][0]]))
    for row in _read_golden("fig1.txt"):
        if row[0] == "subedges":
            assert counts["e"] == int(row[1])
        elif row[0] == "vertices":
            assert counts["v"] == int(row[1])
        elif row[0] == "vertex":
            assert (int(row[1]), int(row[2])) in verts
        elif row[0] == "delta":
            xi = g.free_index(np.array([int(row[1]), int(row[2])]))
            assert classify.weight(c, alpha, xi, int(row[4])) == pytest.approx(float(Fraction(row[5])))


def _remark4_problem(case):
    if case in ("two", "twomean"):
        n_el = (8, 4)
        ex = np.tile(np.arange(8), 4)
        ey = np.repeat(np.arange(4), 8)
        sub = (ex >= 4).astype(np.int32)
        rho = np.where(sub == 0, 1.0, 9.0)
        if case == "twomean":
            rho = np.where(sub == 0, 1.0, np.where(ey < 2, 6.0, 12.0))
        return n_el, sub, sub.copy(), rho
    p = W.fig1_problem()
    return p.n_el, p.elem_sub, p.elem_subsub, 2.0 ** p.elem_subsub


def test_remark4_weights_golden():
    """Remark 4's coefficient weights against values worked by hand, with
    asymmetric keys (Figure 1's split) and a coefficient that varies inside
    a subsubdomain (its mean is alpha_j); each subdomain's weights at a node
    sum to 1."""
    for row in _read_golden("remark4_weights.txt"):
        n_el, sub, ss, rho = _remark4_problem(row[1])
        c = classify.classify(n_el, sub, ss)
        alpha = classify.subsub_alpha(ss, rho, 1)
        xi = q1.Grid(n_el).free_index(np.array([int(row[2]), int(row[3])]))
        assert classify.weight(c, alpha, xi, int(row[5])) == pytest.approx(float(Fraction(row[6])), rel=1e-14), row
        assert sum(classify.weight(c, alpha, xi, int(i)) for i in c.node_subs[xi]) == pytest.approx(1.0)


def test_fig1_multiplicity_differs():
    # The paper contrasts delta_1(xi) = 2/3 with the multiplicity weight 1/2 at xi = (10, 5).
    p = W.fig1_problem()
    c = classify.classify(p.n_el, p.elem_sub, p.elem_subsub)
    xi = q1.Grid(p.n_el).free_index(np.array([10, 5]))
    assert len(c.node_subs[xi]) == 2          # multiplicity 2 -> weight 1/2
    assert len(c.node_keys[int(xi)]) == 3     # three subsubdomains


def closed_form_vef(N, k, L):
    """Every fine vertex, edge and face on Gamma for a 3D tensor partition:
    N subdomains per axis, n = N k / L subsubdomains per axis."""
    n = N * k // L
    faces = 3 * (N - 1) * n * n
    edges = 3 * n * ((n - 1) ** 2 - (n - N) ** 2)
    verts = (n - 1) ** 3 - (n - N) ** 3
    return faces + edges + verts, (verts, edges, faces)


@pytest.mark.parametrize("k", [4, 8])
def test_table1_coarse_size_brute_force(k):
    """Table 1, BDDC-SO(vef): brute-force classification equals the printed size."""
    golden = {(r[0], int(r[1])): int(r[2]) for r in _read_golden("table1.txt")}
    p = W.table1_problem(k)
    c = classify.classify(p.n_el, p.elem_sub, p.elem_subsub)
    total, (v, e, f) = closed_form_vef(10, k, 4)
    assert c.n_coarse == golden[("BDDC-SO(vef)", k)] == total
    assert c.counts_by_type() == {"v": v, "e": e, "f": f}


def test_table1_closed_form_matches_printed():
    golden = {(r[0], int(r[1])): int(r[2]) for r in _read_golden("table1.txt")}
    for k in (4, 8, 16, 24):
        assert closed_form_vef(10, k, 4)[0] == golden[("BDDC-SO(vef)", k)]
    # L = H: subobjects are the standard objects, the coarse size does not depend on k
    for k in (4, 8, 16):
        assert closed_form_vef(10, k, k)[0] == golden[("BDDC(vef)", k)]


def closed_form_vfmin(N, k, L):
    """Every fine vertex and half of the fine faces (no edges)."""
    _, (verts, _, faces) = closed_form_vef(N, k, L)
    return verts + faces // 2, (verts, 0, faces // 2)


def test_table1_vfmin_closed_form_matches_printed():
    """Table 1, BDDC-SO(vf-min): vertices plus half of the faces is the
    printed coarse size at k = 16 and 32 (Section 5.1)."""
    golden = {(r[0], int(r[1])): int(r[2]) for r in _read_golden("table1.txt")}
    for k in (16, 32):
        assert closed_form_vfmin(10, k, 4)[0] == golden[("BDDC-SO(vf-min)", k)]


@pytest.mark.parametrize("k", [4, 8])
def test_table1_vfmin_brute_force(k):
    """The half-face selection (mask 1|4|8) keeps exactly half of the faces
    of the Table 1 meshes and every vertex."""
    p = W.table1_problem(k)
    c = classify.classify(p.n_el, p.elem_sub, p.elem_subsub, primal_mask=13)
    total, (v, e, f) = closed_form_vfmin(10, k, 4)
    assert c.n_coarse == total
    assert c.counts_by_type() == {"v": v, "e": e, "f": f}


def _face_boxes(c, n_el):
    """Per face object: normal axis, plane coordinate, and its in-plane node
    ranges (grid coordinates)."""
    from oracle.q1 import Grid
    fc = Grid(n_el).free_coords()
    out = {}
    for o in range(len(c.obj_nodes)):
        if c.obj_type[o] != classify.TYPE_F:
            continue
        xyz = fc[c.obj_nodes[o]]
        lo, hi = xyz.min(axis=0), xyz.max(axis=0)
        (normal,) = np.nonzero(lo == hi)[0][:1]
        out[o] = (int(normal), int(lo[normal]), lo, hi)
    return out


@pytest.mark.parametrize("sizes", [(24, 8, 4), (24, 12, 4), (20, 10, 5)])
def test_half_faces_alternate_in_each_plane(sizes):
    """Two faces of one interface plane separated by a single fine edge line
    (in-plane neighbours) are never both kept or both dropped, and each
    interface plane keeps half of its faces (even counts) -- a checkerboard."""
    n, H, L = sizes
    p = W.config2_like(n=n, H=H, L=L, cfg=15, log_range=None)
    all_f = classify.classify(p.n_el, p.elem_sub, p.elem_subsub, primal_mask=4)
    half = classify.classify(p.n_el, p.elem_sub, p.elem_subsub, primal_mask=4 | 8)
    kept = set(int(o) for o in half.coarse_objects)
    boxes = _face_boxes(all_f, p.n_el)
    planes = {}
    for o, (a, t, lo, hi) in boxes.items():
        planes.setdefault((a, t), []).append(o)
    pairs = 0
    for (a, t), objs in planes.items():
        assert 2 * sum(o in kept for o in objs) == len(objs)
        ax = [b for b in range(3) if b != a]
        for i, o1 in enumerate(objs):
            for o2 in objs[i + 1:]:
                lo1, hi1, lo2, hi2 = boxes[o1][2], boxes[o1][3], boxes[o2][2], boxes[o2][3]
                for u, w in ((ax[0], ax[1]), (ax[1], ax[0])):
                    touch = hi1[u] + 2 == lo2[u] or hi2[u] + 2 == lo1[u]
                    same = lo1[w] == lo2[w] and hi1[w] == hi2[w]
                    if touch and same:
                        pairs += 1
                        assert (o1 in kept) != (o2 in kept), (o1, o2)
    assert pairs > 0


def test_standard_bddc_is_L_equals_H():
    p = W.table1_problem(4, L=4, subs_per_axis=3)
    q = W.tensor_problem(p.n_el, p.extra["sub_cuts"], p.extra["sub_cuts"])
    c = classify.classify(q.n_el, q.elem_sub, q.elem_subsub)
    # 3x3x3 subdomains: 54 faces, 36 edges, 8 vertices
    assert c.counts_by_type() == {"v": 8, "e": 36, "f": 54}


def test_config_sizes():
    """Coarse sizes of the 2D config and a reduced 3D config (H = 12h, L = 4h)."""
    c1 = classify.classify(*(lambda p: (p.n_el, p.elem_sub, p.elem_subsub))(W.config1()))
    assert c1.n_coarse == 177 and c1.counts_by_type() == {"v": 81, "e": 96, "f": 0}
    p = W.config2_like(n=24, H=12, L=4)
    c = classify.classify(p.n_el, p.elem_sub, p.elem_subsub)
    assert c.n_coarse == closed_form_vef(2, 12, 4)[0]


def test_weights_partition_of_unity():
    rng = np.random.default_rng(1)
    for p in (W.fig1_problem(), W.config2_like(n=12, H=6, L=3, cfg=9)):
        c = classify.classify(p.n_el, p.elem_sub, p.elem_subsub)
        for weighting in (0, 1):
            alpha = classify.subsub_alpha(p.elem_subsub, p.rho * (1 + rng.random(p.n_elements)), weighting)
            for node in np.nonzero(c.is_gamma)[0][::7]:
                s = sum(classify.weight(c, alpha, node, i) for i in c.node_subs[node])
                assert s == pytest.approx(1.0)


def test_symmetric_split_weights_are_multiplicity():
    # For a tensor fine partition every Gamma node's key is split evenly, so
    # the eq. (W) weight is 1 / multiplicity.
    p = W.config2_like(n=12, H=6, L=3, cfg=9)
    c = classify.classify(p.n_el, p.elem_sub, p.elem_subsub)
    alpha = classify.subsub_alpha(p.elem_subsub, p.rho, 0)
    for node in np.nonzero(c.is_gamma)[0]:
        for i in c.node_subs[node]:
            assert classify.weight(c, alpha, node, i) == pytest.approx(1.0 / len(c.node_subs[node]))


def test_objects_partition_gamma():
    p = W.config2_like(n=12, H=6, L=3, cfg=9)
    c = classify.classify(p.n_el, p.elem_sub, p.elem_subsub)
    allnodes = np.concatenate(c.obj_nodes)
    assert len(allnodes) == len(np.unique(allnodes)) == int(c.is_gamma.sum())
    # every node of an object has the same key and the same subdomain set
    for o, nodes in enumerate(c.obj_nodes):
        for v in nodes:
            assert c.node_keys[int(v)] == c.obj_key[o]
            assert list(c.node_subs[v]) == list(c.obj_subs[o])
