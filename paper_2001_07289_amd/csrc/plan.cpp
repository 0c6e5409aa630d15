// Host planner: validates the descriptors, classifies the interface into
// subobjects (Section 3, Remark 2 on classification), and lays out every
// per-subdomain table, block and coarse-tree front the device path uses.
#include "plan.h"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <numeric>
#include <unordered_map>

namespace bddcso {

int object_type(int dim, int key_size) {
  // Tensor fine partitions: a key of 2 subsubdomains is one cut plane (a face
  // in 3D, an edge in 2D), 4 is two cut planes, 8 is three.  Irregular
  // partitions fall in the nearest bracket.
  if (dim == 3) {
    if (key_size == 2) return 4;
    if (key_size <= 4) return 2;
    return 1;
  }
  return key_size == 2 ? 2 : 1;
}

namespace {

struct UnionFind {
  std::vector<int32_t> p;
  explicit UnionFind(size_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int32_t find(int32_t x) {
    while (p[x] != x) {
      p[x] = p[p[x]];
      x = p[x];
    }
    return x;
  }
  void unite(int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a == b) return;
    if (a < b) std::swap(a, b);
    p[a] = b;  // smaller index becomes the root
  }
};

bool fail(Error& err, int code, const std::string& msg) {
  err.code = code;
  err.msg = msg;
  return false;
}

}  // namespace

bool classify(int dim, const int64_t n_el[3], const double h[3], const int32_t* elem_sub,
              const int32_t* elem_subsub, Classification& c, Error& err) {
  if (dim != 2 && dim != 3) return fail(err, -1, "dim must be 2 or 3");
  if (!n_el || !h || !elem_sub || !elem_subsub) return fail(err, -1, "null descriptor pointer");
  c.dim = dim;
  for (int a = 0; a < 3; ++a) {
    if (a < dim) {
      if (n_el[a] < 2) return fail(err, -1, "need at least 2 elements per axis");
      if (!(h[a] > 0)) return fail(err, -1, "mesh spacing must be positive");
      if (n_el[a] > (1 << 20)) return fail(err, -1, "axis too long");
      c.ne[a] = n_el[a];
      c.h[a] = h[a];
      c.nf[a] = n_el[a] - 1;
    } else {
      c.ne[a] = 1;
      c.h[a] = 1.0;
      c.nf[a] = 1;
    }
  }
  c.n_elem = c.ne[0] * c.ne[1] * c.ne[2];
  c.n_free = c.nf[0] * c.nf[1] * c.nf[2];
  c.elem_sub.assign(elem_sub, elem_sub + c.n_elem);
  c.elem_subsub.assign(elem_subsub, elem_subsub + c.n_elem);
  int32_t max_s = -1, max_ss = -1;
  for (int64_t e = 0; e < c.n_elem; ++e) {
    if (c.elem_sub[e] < 0 || c.elem_subsub[e] < 0) return fail(err, -1, "negative subdomain id");
    max_s = std::max(max_s, c.elem_sub[e]);
    max_ss = std::max(max_ss, c.elem_subsub[e]);
  }
  c.n_sub = max_s + 1;
  c.n_ss = max_ss + 1;
  c.ss_parent.assign(c.n_ss, -1);
  for (int64_t e = 0; e < c.n_elem; ++e) {
    int32_t& par = c.ss_parent[c.elem_subsub[e]];
    if (par < 0) par = c.elem_sub[e];
    else if (par != c.elem_sub[e])
      return fail(err, -1, "subsubdomain " + std::to_string(c.elem_subsub[e]) +
                               " spans more than one subdomain");
  }
  for (int j = 0; j < c.n_ss; ++j)
    if (c.ss_parent[j] < 0) return fail(err, -1, "subsubdomain ids must be contiguous (empty id)");

  // subdomain boxes
  c.ebox.assign(c.n_sub, {INT32_MAX, INT32_MAX, INT32_MAX, -1, -1, -1});
  std::vector<int64_t> count(c.n_sub, 0);
  for (int64_t e = 0; e < c.n_elem; ++e) {
    int ec[3] = {(int)(e % c.ne[0]), (int)((e / c.ne[0]) % c.ne[1]), (int)(e / (c.ne[0] * c.ne[1]))};
    auto& b = c.ebox[c.elem_sub[e]];
    for (int a = 0; a < 3; ++a) {
      b[a] = std::min(b[a], ec[a]);
      b[3 + a] = std::max(b[3 + a], ec[a] + 1);
    }
    count[c.elem_sub[e]]++;
  }
  for (int s = 0; s < c.n_sub; ++s) {
    if (count[s] == 0) return fail(err, -1, "subdomain ids must be contiguous (empty id)");
    auto& b = c.ebox[s];
    int64_t vol = (int64_t)(b[3] - b[0]) * (b[4] - b[1]) * (b[5] - b[2]);
    if (vol != count[s])
      return fail(err, -1, "subdomain " + std::to_string(s) + " is not an axis-aligned box");
  }
  // elements of each subsubdomain (ascending element id)
  c.ss_eptr.assign(c.n_ss + 1, 0);
  for (int64_t e = 0; e < c.n_elem; ++e) c.ss_eptr[c.elem_subsub[e] + 1]++;
  for (int j = 0; j < c.n_ss; ++j) c.ss_eptr[j + 1] += c.ss_eptr[j];
  c.ss_elem.resize(c.n_elem);
  {
    std::vector<int32_t> pos(c.ss_eptr.begin(), c.ss_eptr.end() - 1);
    for (int64_t e = 0; e < c.n_elem; ++e) c.ss_elem[pos[c.elem_subsub[e]]++] = (int32_t)e;
  }

  // grid index of each subsubdomain along each axis
  c.ss_idx.assign(c.n_ss, {0, 0, 0});
  for (int a = 0; a < dim; ++a) {
    std::vector<int> lo(c.n_ss, INT32_MAX);
    for (int j = 0; j < c.n_ss; ++j)
      for (int t = c.ss_eptr[j]; t < c.ss_eptr[j + 1]; ++t) {
        const int64_t e = c.ss_elem[t];
        const int ec = a == 0 ? (int)(e % c.ne[0]) : a == 1 ? (int)((e / c.ne[0]) % c.ne[1])
                                                           : (int)(e / (c.ne[0] * c.ne[1]));
        lo[j] = std::min(lo[j], ec);
      }
    std::vector<int> d(lo);
    std::sort(d.begin(), d.end());
    d.erase(std::unique(d.begin(), d.end()), d.end());
    for (int j = 0; j < c.n_ss; ++j)
      c.ss_idx[j][a] = (int)(std::lower_bound(d.begin(), d.end(), lo[j]) - d.begin());
  }

  // Gamma nodes and their keys
  const int nadj = dim == 3 ? 8 : 4;
  c.node_gam.assign(c.n_free, -1);
  c.gam_node.clear();
  c.gam_kptr.assign(1, 0);
  c.gam_key.clear();
  for (int64_t f = 0; f < c.n_free; ++f) {
    int g[3];
    c.node_coords(f, g);
    int32_t subs[8], keys[8];
    int ns = 0, nk = 0;
    for (int l = 0; l < nadj; ++l) {
      int ex = g[0] - 1 + (l & 1), ey = g[1] - 1 + ((l >> 1) & 1);
      int ez = dim == 3 ? g[2] - 1 + ((l >> 2) & 1) : 0;
      int64_t e = ex + c.ne[0] * (ey + c.ne[1] * (int64_t)ez);
      int32_t s = c.elem_sub[e], k = c.elem_subsub[e];
      bool have = false;
      for (int q = 0; q < ns; ++q) have |= subs[q] == s;
      if (!have) subs[ns++] = s;
      have = false;
      for (int q = 0; q < nk; ++q) have |= keys[q] == k;
      if (!have) keys[nk++] = k;
    }
    if (ns < 2) continue;
    std::sort(keys, keys + nk);
    c.node_gam[f] = (int32_t)c.gam_node.size();
    c.gam_node.push_back(f);
    c.gam_key.insert(c.gam_key.end(), keys, keys + nk);
    c.gam_kptr.push_back((int32_t)c.gam_key.size());
  }
  const int64_t ng = (int64_t)c.gam_node.size();
  auto same_key = [&](int32_t a, int32_t b) {
    int la = c.gam_kptr[a + 1] - c.gam_kptr[a], lb = c.gam_kptr[b + 1] - c.gam_kptr[b];
    if (la != lb) return false;
    return std::equal(c.gam_key.begin() + c.gam_kptr[a], c.gam_key.begin() + c.gam_kptr[a + 1],
                      c.gam_key.begin() + c.gam_kptr[b]);
  };
  // objects: connected sets (grid-edge adjacency) of Gamma nodes with one key
  UnionFind uf(ng);
  for (int64_t q = 0; q < ng; ++q) {
    int g[3];
    c.node_coords(c.gam_node[q], g);
    for (int a = 0; a < dim; ++a) {
      if (g[a] + 1 > c.nf[a]) continue;
      int gn[3] = {g[0], g[1], g[2]};
      gn[a] += 1;
      int32_t r = c.node_gam[c.free_index(gn)];
      if (r >= 0 && same_key((int32_t)q, r)) uf.unite((int32_t)q, r);
    }
  }
  std::vector<int32_t> root_obj(ng, -1);
  c.gam_obj.assign(ng, -1);
  int32_t nobj = 0;
  for (int64_t q = 0; q < ng; ++q) {
    int32_t r = uf.find((int32_t)q);
    if (root_obj[r] < 0) root_obj[r] = nobj++;
    c.gam_obj[q] = root_obj[r];
  }
  c.obj_ptr.assign(nobj + 1, 0);
  for (int64_t q = 0; q < ng; ++q) c.obj_ptr[c.gam_obj[q] + 1]++;
  for (int o = 0; o < nobj; ++o) c.obj_ptr[o + 1] += c.obj_ptr[o];
  c.obj_gam.resize(ng);
  {
    std::vector<int32_t> pos(c.obj_ptr.begin(), c.obj_ptr.end() - 1);
    for (int64_t q = 0; q < ng; ++q) c.obj_gam[pos[c.gam_obj[q]]++] = (int32_t)q;
  }
  c.obj_type.resize(nobj);
  c.obj_sptr.assign(1, 0);
  c.obj_subs.clear();
  for (int o = 0; o < nobj; ++o) {
    int32_t q = c.obj_gam[c.obj_ptr[o]];
    int ks = c.gam_kptr[q + 1] - c.gam_kptr[q];
    c.obj_type[o] = (int8_t)object_type(dim, ks);
    std::vector<int32_t> ps;
    for (int k = c.gam_kptr[q]; k < c.gam_kptr[q + 1]; ++k) ps.push_back(c.ss_parent[c.gam_key[k]]);
    std::sort(ps.begin(), ps.end());
    ps.erase(std::unique(ps.begin(), ps.end()), ps.end());
    c.obj_subs.insert(c.obj_subs.end(), ps.begin(), ps.end());
    c.obj_sptr.push_back((int32_t)c.obj_subs.size());
  }
  return true;
}

namespace {

// Groups the non-empty planes of one set into diagonal blocks.
void make_blocks(const std::vector<int>& plane_count, int target, int start_rank,
                 std::vector<BlockDev>& out) {
  int np = (int)plane_count.size();
  int rank = start_rank;
  int z = 0;
  while (z < np) {
    if (plane_count[z] == 0) {
      ++z;
      continue;
    }
    BlockDev b{};
    b.start = rank;
    b.plane_lo = z;
    b.size = plane_count[z];
    b.first_n = plane_count[z];
    b.last_n = plane_count[z];
    int zz = z + 1;
    while (zz < np && plane_count[zz] > 0 && b.size + plane_count[zz] <= target) {
      b.size += plane_count[zz];
      b.last_n = plane_count[zz];
      ++zz;
    }
    b.plane_hi = zz;
    rank += b.size;
    out.push_back(b);
    z = zz;
  }
}

struct NDBuilder {
  const Classification& c;
  Plan& plan;
  std::vector<std::vector<int32_t>> dof_subs;   // per coarse dof
  std::vector<std::vector<int32_t>> sub_dofs;   // per sub (sorted)
  std::vector<double> cen[3];
  std::vector<int> mark;
  struct Node {
    std::vector<int32_t> P, B, kids, leaves;
    int parent = -1, level = 1;
  };
  std::vector<Node> nodes;

  NDBuilder(const Classification& cc, Plan& pp) : c(cc), plan(pp) {}

  int make(std::vector<int32_t>& S, std::vector<int32_t>& cand, int parent) {
    int t = (int)nodes.size();
    nodes.emplace_back();
    nodes[t].parent = parent;
    // split S along the axis of largest centroid extent, at the coordinate
    // boundary that best balances the two halves
    int best_axis = 0;
    double best_ext = -1;
    for (int a = 0; a < c.dim; ++a) {
      double lo = 1e300, hi = -1e300;
      for (int s : S) {
        lo = std::min(lo, cen[a][s]);
        hi = std::max(hi, cen[a][s]);
      }
      if (hi - lo > best_ext) {
        best_ext = hi - lo;
        best_axis = a;
      }
    }
    std::vector<int32_t> Ss = S;
    std::stable_sort(Ss.begin(), Ss.end(), [&](int32_t x, int32_t y) {
      return cen[best_axis][x] < cen[best_axis][y];
    });
    size_t cut = 0;
    size_t half = Ss.size() / 2;
    size_t best = SIZE_MAX;
    for (size_t k = 1; k < Ss.size(); ++k) {
      if (cen[best_axis][Ss[k]] == cen[best_axis][Ss[k - 1]]) continue;
      size_t d = k > half ? k - half : half - k;
      if (d < best) {
        best = d;
        cut = k;
      }
    }
    if (cut == 0) cut = half;  // all centroids equal along every axis
    std::vector<int32_t> S1(Ss.begin(), Ss.begin() + cut), S2(Ss.begin() + cut, Ss.end());
    for (int s : S1) mark[s] = 1;
    for (int s : S2) mark[s] = 2;
    std::vector<int32_t> c1, c2;
    for (int32_t d : cand) {
      bool in1 = false, in2 = false;
      for (int s : dof_subs[d]) {
        in1 |= mark[s] == 1;
        in2 |= mark[s] == 2;
      }
      if (in1 && !in2) c1.push_back(d);
      else if (in2 && !in1) c2.push_back(d);
      else nodes[t].P.push_back(d);
    }
    for (int s : S) mark[s] = 0;
    std::sort(nodes[t].P.begin(), nodes[t].P.end());
    // boundary: dofs touching S that do not lie inside S
    {
      std::vector<int32_t> all;
      for (int s : S) all.insert(all.end(), sub_dofs[s].begin(), sub_dofs[s].end());
      std::sort(all.begin(), all.end());
      all.erase(std::unique(all.begin(), all.end()), all.end());
      for (int s : S) mark[s] = 3;
      for (int32_t d : all) {
        bool inside = true;
        for (int s : dof_subs[d]) inside &= mark[s] == 3;
        if (!inside) nodes[t].B.push_back(d);
      }
      for (int s : S) mark[s] = 0;
    }
    for (auto* side : {&S1, &S2}) {
      auto& cs = side == &S1 ? c1 : c2;
      if (side->size() == 1) {
        nodes[t].leaves.push_back((*side)[0]);
      } else {
        int k = make(*side, cs, t);
        nodes[t].kids.push_back(k);
      }
    }
    int lev = 1;
    for (int k : nodes[t].kids) lev = std::max(lev, nodes[k].level + 1);
    nodes[t].level = lev;
    return t;
  }
};

}  // namespace

bool half_keep(const Classification& c, int obj) {
  const int32_t q = c.obj_gam[c.obj_ptr[obj]];
  if (c.gam_kptr[q + 1] - c.gam_kptr[q] != 2) return true;
  const auto& i1 = c.ss_idx[c.gam_key[c.gam_kptr[q]]];
  const auto& i2 = c.ss_idx[c.gam_key[c.gam_kptr[q] + 1]];
  int normal = 0, best = -1, sum = 0;
  for (int a = 0; a < c.dim; ++a) {
    const int d = std::abs(i1[a] - i2[a]);
    if (d > best) {
      best = d;
      normal = a;
    }
    sum += i1[a];
  }
  return (sum - i1[normal]) % 2 == 0;
}

bool build_plan(const Classification& c, int primal_mask, int block_target, int coarse_solver,
                Plan& plan, Error& err) {
  plan = Plan();
  plan.primal_mask = primal_mask;
  plan.block_target = block_target > 0 ? block_target : 192;
  plan.coarse_solver = coarse_solver;
  const int dim = c.dim;
  const int pa = dim - 1;  // plane axis
  // coarse numbering: selected objects in object order (smallest free index)
  plan.obj_coarse.assign(c.n_obj(), -1);
  for (int o = 0; o < c.n_obj(); ++o)
    if ((c.obj_type[o] & primal_mask) && (!(primal_mask & kHalfCodim1) || half_keep(c, o))) {
      plan.obj_coarse[o] = (int32_t)plan.coarse_obj.size();
      plan.coarse_obj.push_back(o);
    }
  plan.n_coarse = (int64_t)plan.coarse_obj.size();

  plan.subs.resize(c.n_sub);
  int64_t loc_off = 0, I_off = 0, r_off = 0, g_off = 0, v_off = 0, a_off = 0, c_off = 0, sel_off = 0;
  int64_t G_off = 0, Z_off = 0, XG_off = 0, Sc_off = 0, T_off = 0, PhiG_off = 0, YG_off = 0, Kc_off = 0;
  std::vector<std::vector<int32_t>> sub_dofs(c.n_sub);
  for (int s = 0; s < c.n_sub; ++s) {
    SubDev& S = plan.subs[s];
    std::memset(&S, 0, sizeof(S));
    const auto& b = c.ebox[s];
    for (int a = 0; a < 3; ++a) {
      S.elo[a] = b[a];
      S.ehi[a] = b[3 + a];
      if (a < dim) {
        int lo = std::max(b[a], 1), hi = std::min(b[3 + a], (int)c.ne[a] - 1);
        S.lo[a] = lo;
        S.m[a] = hi - lo + 1;
      } else {
        S.lo[a] = 1;
        S.m[a] = 1;
      }
      if (S.m[a] < 1) return fail(err, -1, "subdomain without free nodes");
    }
    S.n_loc = S.m[0] * S.m[1] * S.m[2];
    S.loc_off = loc_off;
    S.I_off = I_off;
    S.r_off = r_off;
    S.g_off = g_off;
    S.v_off = v_off;
    S.a_off = a_off;
    S.am_off = a_off - s;
    S.c_off = c_off;
    // A subdomain away from the Dirichlet boundary has the constants in the
    // kernel of its local matrix.  Primal point constraints (eliminated)
    // remove them; without any, one interior node is left out of the r-set
    // (the pin) and the constant is carried as one extra unknown of the
    // constrained Neumann problem.
    bool floating = true;
    for (int a = 0; a < dim; ++a)
      if (b[a] == 0 || b[3 + a] == (int)c.ne[a]) floating = false;
    int pin_l = -1;
    if (floating) {
      int npt = 0, first_interior = -1;
      for (int l = 0; l < S.n_loc; ++l) {
        int x = l % S.m[0], y = (l / S.m[0]) % S.m[1], z = l / (S.m[0] * S.m[1]);
        int gcoord[3] = {S.lo[0] + x, S.lo[1] + y, S.lo[2] + z};
        int32_t q = c.node_gam[c.free_index(gcoord)];
        if (q < 0) {
          if (first_interior < 0) first_interior = l;
          continue;
        }
        int32_t o = c.gam_obj[q];
        if (plan.obj_coarse[o] >= 0 && c.obj_ptr[o + 1] - c.obj_ptr[o] == 1) ++npt;
      }
      if (npt == 0) {
        if (first_interior < 0)
          return fail(err, -1, "floating subdomain " + std::to_string(s) +
                                   " has neither a primal point constraint nor an interior node");
        pin_l = first_interior;
      }
    }
    S.pin = pin_l;
    // classify local nodes
    std::vector<int32_t> lI(S.n_loc, -1), lr(S.n_loc, -1), lg(S.n_loc, -1);
    std::vector<int> cntI(S.m[pa], 0), cntR(S.m[pa], 0);
    std::vector<int32_t> local_coarse;
    int nI = 0, nr = 0, ngl = 0, nv = 0;
    for (int l = 0; l < S.n_loc; ++l) {
      int x = l % S.m[0], y = (l / S.m[0]) % S.m[1], z = l / (S.m[0] * S.m[1]);
      int gcoord[3] = {S.lo[0] + x, S.lo[1] + y, S.lo[2] + z};
      int64_t f = c.free_index(gcoord);
      int32_t q = c.node_gam[f];
      int plane = pa == 2 ? z : y;
      bool vert = false;
      if (q < 0) {
        lI[l] = nI++;
        cntI[plane]++;
      } else {
        lg[l] = ngl++;
        int32_t o = c.gam_obj[q];
        int32_t cid = plan.obj_coarse[o];
        if (cid >= 0) {
          local_coarse.push_back(cid);
          vert = (c.obj_ptr[o + 1] - c.obj_ptr[o]) == 1;
        }
      }
      if (vert) {
        plan.v_loc.push_back(l);
        nv++;
      } else if (l != pin_l) {
        lr[l] = nr++;
        cntR[plane]++;
      }
    }
    if (pin_l >= 0 && nv != 0) return fail(err, -1, "internal: pinned subdomain with primal points");
    std::sort(local_coarse.begin(), local_coarse.end());
    local_coarse.erase(std::unique(local_coarse.begin(), local_coarse.end()), local_coarse.end());
    S.n_I = nI;
    S.n_r = nr;
    S.n_g = ngl;
    S.n_v = nv;
    S.n_c = (int)local_coarse.size();
    sub_dofs[s] = local_coarse;
    plan.loc_I.insert(plan.loc_I.end(), lI.begin(), lI.end());
    plan.loc_r.insert(plan.loc_r.end(), lr.begin(), lr.end());
    plan.loc_g.insert(plan.loc_g.end(), lg.begin(), lg.end());
    for (int l = 0; l < S.n_loc; ++l) {
      if (lI[l] >= 0) plan.I_loc.push_back(l);
      if (lr[l] >= 0) plan.r_loc.push_back(l);
    }
    // the Gamma neighbours of each interior node (the nonzeros of K_{I Gamma}),
    // by neighbour code t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1), in I order
    if (plan.kig_ptr.empty()) plan.kig_ptr.push_back(0);
    for (int l = 0; l < S.n_loc; ++l) {
      if (lI[l] < 0) continue;
      const int cl[3] = {l % S.m[0], (l / S.m[0]) % S.m[1], l / (S.m[0] * S.m[1])};
      for (int t = 0; t < 27; ++t) {
        const int cn[3] = {cl[0] + t % 3 - 1, cl[1] + (t / 3) % 3 - 1, cl[2] + t / 9 - 1};
        bool in = true;
        for (int a = 0; a < 3; ++a) in = in && cn[a] >= 0 && cn[a] < S.m[a];
        if (!in) continue;
        const int ln = cn[0] + S.m[0] * (cn[1] + S.m[1] * cn[2]);
        if (lg[ln] >= 0) {
          plan.kig_t.push_back((int8_t)t);
          plan.kig_own.push_back((int32_t)plan.kig_ptr.size() - 1);
          plan.kig_sub.push_back(s);
        }
      }
      plan.kig_ptr.push_back((int32_t)plan.kig_t.size());
    }
    // Gamma entries
    for (int l = 0; l < S.n_loc; ++l) {
      if (lg[l] < 0) continue;
      int x = l % S.m[0], y = (l / S.m[0]) % S.m[1], z = l / (S.m[0] * S.m[1]);
      int gcoord[3] = {S.lo[0] + x, S.lo[1] + y, S.lo[2] + z};
      plan.g_loc.push_back(l);
      plan.g_gam.push_back(c.node_gam[c.free_index(gcoord)]);
      plan.g_r.push_back(lr[l]);
      plan.g_sub.push_back(s);
      plan.g_v.push_back(-1);
    }
    // the interior neighbours of each Gamma entry (the nonzeros of K_{Gamma I})
    if (plan.kgi_ptr.empty()) plan.kgi_ptr.push_back(0);
    for (int l = 0; l < S.n_loc; ++l) {
      if (lg[l] < 0) continue;
      const int cl[3] = {l % S.m[0], (l / S.m[0]) % S.m[1], l / (S.m[0] * S.m[1])};
      for (int t = 0; t < 27; ++t) {
        const int cn[3] = {cl[0] + t % 3 - 1, cl[1] + (t / 3) % 3 - 1, cl[2] + t / 9 - 1};
        bool in = true;
        for (int a = 0; a < 3; ++a) in = in && cn[a] >= 0 && cn[a] < S.m[a];
        if (!in) continue;
        const int ln = cn[0] + S.m[0] * (cn[1] + S.m[1] * cn[2]);
        if (lI[ln] >= 0) {
          plan.kgi_t.push_back((int8_t)t);
          plan.kgi_own.push_back((int32_t)plan.kgi_ptr.size() - 1);
        }
      }
      plan.kgi_ptr.push_back((int32_t)plan.kgi_t.size());
    }
    // vertex index of each Gamma entry
    {
      int vi = 0;
      for (int64_t k = v_off; k < v_off + nv; ++k, ++vi) {
        int l = plan.v_loc[k];
        plan.g_v[g_off + lg[l]] = vi;
      }
    }
    // selected rows: the Gamma entries, then the r-set nodes of the primal
    // vertices' stencils that are not on Gamma (the rows of Phi that the
    // local coarse matrix and the per-iteration products read)
    {
      S.sel_off = sel_off;
      std::vector<int32_t> ls(lg);
      for (int e = 0; e < ngl; ++e) plan.sel_r.push_back(plan.g_r[g_off + e]);
      int ns = ngl;
      for (int64_t k = v_off; k < v_off + nv; ++k) {
        const int l = plan.v_loc[k];
        const int cv[3] = {l % S.m[0], (l / S.m[0]) % S.m[1], l / (S.m[0] * S.m[1])};
        for (int t = 0; t < 27; ++t) {
          const int dz = dim == 3 ? t / 9 - 1 : 0, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
          if (dim == 2 && t >= 9) continue;
          const int cn[3] = {cv[0] + dx, cv[1] + dy, cv[2] + dz};
          bool in = true;
          for (int a = 0; a < 3; ++a) in = in && cn[a] >= 0 && cn[a] < S.m[a];
          if (!in) continue;
          const int ln = cn[0] + S.m[0] * (cn[1] + S.m[1] * cn[2]);
          if (lr[ln] < 0 || ls[ln] >= 0) continue;
          ls[ln] = ns++;
          plan.sel_r.push_back(lr[ln]);
        }
      }
      S.n_s = ns;
      sel_off += ns;
      plan.loc_sel.insert(plan.loc_sel.end(), ls.begin(), ls.end());
    }
    // local coarse: vertices and averages, in coarse order.  The averages
    // are numbered by the first plane of their object, so that at each
    // block of the forward basis solve the columns already reached form a
    // prefix (the vertices are numbered by local node, so by plane, already).
    auto node_plane = [&](int32_t q) {
      int gcoord[3];
      c.node_coords(c.gam_node[q], gcoord);
      return pa == 2 ? gcoord[2] - S.lo[2] : gcoord[1] - S.lo[1];
    };
    std::vector<int> avg_key, avg_k;
    for (int k = 0; k < S.n_c; ++k) {
      int32_t o = plan.coarse_obj[local_coarse[k]];
      if (c.obj_ptr[o + 1] - c.obj_ptr[o] == 1) continue;
      int key = INT32_MAX;
      for (int t = c.obj_ptr[o]; t < c.obj_ptr[o + 1]; ++t) key = std::min(key, node_plane(c.obj_gam[t]));
      avg_key.push_back(key);
      avg_k.push_back(k);
    }
    std::vector<int> avg_order(avg_k.size());
    std::iota(avg_order.begin(), avg_order.end(), 0);
    std::stable_sort(avg_order.begin(), avg_order.end(), [&](int x, int y) { return avg_key[x] < avg_key[y]; });
    std::vector<int> avg_of_k(S.n_c, -1);
    for (size_t j = 0; j < avg_order.size(); ++j) avg_of_k[avg_k[avg_order[j]]] = (int)j;
    std::vector<int32_t> v_c(nv, -1);
    const int na = (int)avg_k.size();
    for (int k = 0; k < S.n_c; ++k) {
      int32_t cid = local_coarse[k];
      int32_t o = plan.coarse_obj[cid];
      plan.c_glob.push_back(cid);
      int sz = c.obj_ptr[o + 1] - c.obj_ptr[o];
      if (sz == 1) {
        int32_t q = c.obj_gam[c.obj_ptr[o]];
        int gcoord[3];
        c.node_coords(c.gam_node[q], gcoord);
        int l = (gcoord[0] - S.lo[0]) + S.m[0] * ((gcoord[1] - S.lo[1]) + S.m[1] * (gcoord[2] - S.lo[2]));
        int vi = plan.g_v[g_off + lg[l]];
        if (vi < 0) return fail(err, -6, "internal: vertex not found");
        plan.c_kind.push_back(vi);
        v_c[vi] = k;
      } else {
        plan.c_kind.push_back(-(avg_of_k[k] + 1));
      }
    }
    plan.a_ptr.push_back((int32_t)plan.a_r.size());
    for (int j = 0; j < na; ++j) {
      const int k = avg_k[avg_order[j]];
      const int32_t o = plan.coarse_obj[local_coarse[k]];
      for (int t = c.obj_ptr[o]; t < c.obj_ptr[o + 1]; ++t) {
        int32_t q = c.obj_gam[t];
        int gcoord[3];
        c.node_coords(c.gam_node[q], gcoord);
        int l = (gcoord[0] - S.lo[0]) + S.m[0] * ((gcoord[1] - S.lo[1]) + S.m[1] * (gcoord[2] - S.lo[2]));
        plan.a_r.push_back(lr[l]);
        plan.a_g.push_back(lg[l]);
      }
      plan.a_c.push_back(k);
      plan.a_ptr.push_back((int32_t)plan.a_r.size());
    }
    for (int vi = 0; vi < nv; ++vi) {
      if (v_c[vi] < 0) return fail(err, -6, "internal: vertex without coarse dof");
      plan.v_c.push_back(v_c[vi]);
    }
    S.n_a = na;
    // blocks
    S.bI_off = (int64_t)plan.blocks.size();
    make_blocks(cntI, plan.block_target, 0, plan.blocks);
    S.nbI = (int)(plan.blocks.size() - S.bI_off);
    S.bR_off = (int64_t)plan.blocks.size();
    make_blocks(cntR, plan.block_target, 0, plan.blocks);
    S.nbR = (int)(plan.blocks.size() - S.bR_off);
    // The columns of [X | Y'] in the order the forward solve reaches them: an
    // average from its first plane on, a vertex from the plane below its own
    // (its stiffness column touches the planes next to it).  Column j of the
    // right-hand side (an average for j < na, else vertex j - na) is stored
    // at z_col[j]; at each r block the reached columns are a prefix.
    {
      std::vector<int> key(na + nv), ord(na + nv);
      for (int a = 0; a < na; ++a) key[a] = avg_key[avg_order[a]];
      for (int v = 0; v < nv; ++v) {
        const int l = plan.v_loc[v_off + v];
        const int vp = pa == 2 ? l / (S.m[0] * S.m[1]) : (l / S.m[0]) % S.m[1];
        key[na + v] = std::max(vp - 1, 0);
      }
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return key[x] < key[y]; });
      std::vector<int32_t> zc(na + nv);
      for (int q = 0; q < na + nv; ++q) zc[ord[q]] = q;
      plan.z_col.insert(plan.z_col.end(), zc.begin(), zc.end());
      for (int64_t b = S.bR_off; b < S.bR_off + S.nbR; ++b) {
        BlockDev& B = plan.blocks[b];
        const int last = B.plane_hi - 1;
        B.za = 0;
        while (B.za < na + nv && key[ord[B.za]] <= last) ++B.za;
      }
      if (S.nbR > 0) plan.blocks[S.bR_off + S.nbR - 1].za = na + nv;  // every column by the last block
    }
    // coupling rows between consecutive blocks of each set
    for (int setR = 0; setR < 2; ++setR) {
      const int64_t b0 = setR ? S.bR_off : S.bI_off;
      const int nbs = setR ? S.nbR : S.nbI;
      const std::vector<int32_t>& ls = setR ? lr : lI;
      std::vector<int32_t> sl;
      for (int l = 0; l < S.n_loc; ++l)
        if (ls[l] >= 0) sl.push_back(l);
      const int nt = dim == 3 ? 9 : 3;
      auto add_rows = [&](const BlockDev& B, bool first, int dir) {
        const int cnt = first ? B.first_n : B.last_n;
        const int base = first ? B.start : B.start + B.size - B.last_n;
        for (int i = 0; i < cnt; ++i) {
          const int l = sl[base + i];
          int c[3] = {l % S.m[0], (l / S.m[0]) % S.m[1], l / (S.m[0] * S.m[1])};
          plan.cpl_sub.push_back(s);
          plan.cpl_loc.push_back(l);
          plan.cpl_dir.push_back(dir);
          for (int t = 0; t < 5; ++t) {
            int32_t jl = -1;
            if (first && (dim == 3 || t < 2)) {
              int cn[3] = {c[0] + kInPlaneLower[t][0], c[1] + (dim == 3 ? kInPlaneLower[t][1] : 0), c[2]};
              bool ok = true;
              for (int a = 0; a < 3; ++a) ok = ok && cn[a] >= 0 && cn[a] < S.m[a];
              if (ok) {
                const int32_t rk = ls[cn[0] + S.m[0] * (cn[1] + S.m[1] * cn[2])];
                if (rk >= 0) jl = rk - B.start;
              }
            }
            plan.ipl_rank.push_back(jl);
          }
          for (int t = 0; t < 9; ++t) {
            int cn[3] = {c[0], c[1], c[2]};
            bool ok = t < nt;
            if (dim == 3) {
              cn[2] += dir;
              cn[0] += t % 3 - 1;
              cn[1] += t / 3 - 1;
            } else {
              cn[1] += dir;
              cn[0] += t - 1;
            }
            for (int a = 0; a < 3; ++a) ok = ok && cn[a] >= 0 && cn[a] < S.m[a];
            int32_t rk = -1;
            if (ok) rk = ls[cn[0] + S.m[0] * (cn[1] + S.m[1] * cn[2])];
            plan.cpl_rank.push_back(rk);
          }
        }
      };
      for (int k = 0; k < nbs; ++k) {
        BlockDev& B = plan.blocks[b0 + k];
        B.cf_off = -1;
        B.cb_off = -1;
        if (k > 0 && plan.blocks[b0 + k - 1].plane_hi == B.plane_lo) {
          B.cf_off = (int64_t)plan.cpl_sub.size();
          add_rows(B, true, -1);
        }
        if (k + 1 < nbs && B.plane_hi == plan.blocks[b0 + k + 1].plane_lo) {
          B.cb_off = (int64_t)plan.cpl_sub.size();
          add_rows(B, false, 1);
        }
      }
    }
    for (int64_t k = S.bI_off; k < (int64_t)plan.blocks.size(); ++k) {
      BlockDev& B = plan.blocks[k];
      // columns start on 16-element (128-byte in FP64) boundaries, so the
      // 16-row tiles of the solves and sweeps are whole cache lines
      B.ld = (B.size + 15) / 16 * 16;
      G_off = (G_off + 15) / 16 * 16;
      B.G_off = G_off;
      G_off += (int64_t)B.ld * B.size;
      plan.max_block = std::max(plan.max_block, B.size);
    }
    plan.max_nbI = std::max(plan.max_nbI, S.nbI);
    plan.max_nbR = std::max(plan.max_nbR, S.nbR);
    // pools
    S.Z_off = Z_off;
    Z_off += (int64_t)S.n_r * (S.n_a + S.n_v);
    S.XG_off = XG_off;
    XG_off += (int64_t)S.n_s * S.n_a;
    S.Sc_off = Sc_off;
    Sc_off += (int64_t)S.n_a * S.n_a;
    S.T_off = T_off;
    T_off += (int64_t)S.n_a * S.n_c;
    S.PhiG_off = PhiG_off;
    PhiG_off += (int64_t)S.n_s * S.n_v;
    S.YG_off = YG_off;
    YG_off += (int64_t)S.n_g * S.n_v;
    S.Kc_off = Kc_off;
    Kc_off += (int64_t)S.n_c * S.n_c;
    loc_off += S.n_loc;
    I_off += S.n_I;
    r_off += S.n_r;
    g_off += S.n_g;
    v_off += S.n_v;
    a_off += S.n_a + 1;
    c_off += S.n_c;
    plan.max_na = std::max(plan.max_na, S.n_a);
    plan.max_nc = std::max(plan.max_nc, S.n_c);
    plan.max_nr = std::max(plan.max_nr, S.n_r);
    plan.max_nloc = std::max(plan.max_nloc, S.n_loc);
    plan.max_ng = std::max(plan.max_ng, S.n_g);
    plan.max_ns = std::max(plan.max_ns, S.n_s);
    plan.max_zcols = std::max(plan.max_zcols, S.n_a + S.n_v);
  }
  plan.tot_loc = loc_off;
  plan.tot_I = I_off;
  plan.tot_r = r_off;
  plan.tot_g = g_off;
  plan.tot_v = v_off;
  plan.tot_a = (int64_t)plan.a_c.size();
  plan.tot_c = c_off;
  plan.pool_G = G_off;
  plan.pool_Z = Z_off;
  plan.pool_XG = XG_off;
  plan.pool_Sc = Sc_off;
  plan.pool_T = T_off;
  plan.pool_PhiG = PhiG_off;
  plan.pool_YG = YG_off;
  plan.pool_Kc = Kc_off;

  // Gamma index -> entries; coarse id -> local coarse entries
  const int64_t ng = (int64_t)c.gam_node.size();
  plan.gam_eptr.assign(ng + 1, 0);
  for (int32_t q : plan.g_gam) plan.gam_eptr[q + 1]++;
  for (int64_t q = 0; q < ng; ++q) plan.gam_eptr[q + 1] += plan.gam_eptr[q];
  plan.gam_ent.resize(plan.g_gam.size());
  {
    std::vector<int32_t> pos(plan.gam_eptr.begin(), plan.gam_eptr.end() - 1);
    for (size_t e = 0; e < plan.g_gam.size(); ++e) plan.gam_ent[pos[plan.g_gam[e]]++] = (int32_t)e;
  }
  plan.crs_eptr.assign(plan.n_coarse + 1, 0);
  for (int32_t cid : plan.c_glob) plan.crs_eptr[cid + 1]++;
  for (int64_t k = 0; k < plan.n_coarse; ++k) plan.crs_eptr[k + 1] += plan.crs_eptr[k];
  plan.crs_ent.resize(plan.c_glob.size());
  {
    std::vector<int32_t> pos(plan.crs_eptr.begin(), plan.crs_eptr.end() - 1);
    for (size_t e = 0; e < plan.c_glob.size(); ++e) plan.crs_ent[pos[plan.c_glob[e]]++] = (int32_t)e;
  }
  // greedy colouring: subdomains sharing a coarse dof get different colours
  {
    std::vector<int> color(c.n_sub, -1);
    std::vector<int> stamp;
    int ncol = 0;
    for (int s = 0; s < c.n_sub; ++s) {
      std::vector<char> used(ncol + 1, 0);
      for (int32_t cid : sub_dofs[s]) {
        int32_t o = plan.coarse_obj[cid];
        for (int t = c.obj_sptr[o]; t < c.obj_sptr[o + 1]; ++t) {
          int s2 = c.obj_subs[t];
          if (s2 != s && color[s2] >= 0) used[color[s2]] = 1;
        }
      }
      int col = 0;
      while (col < ncol && used[col]) ++col;
      if (col == ncol) ++ncol;
      color[s] = col;
      plan.subs[s].color = col;
    }
    plan.color_subs.assign(ncol, {});
    for (int s = 0; s < c.n_sub; ++s) plan.color_subs[color[s]].push_back(s);
  }

  // coarse tree
  NDBuilder nd(c, plan);
  nd.sub_dofs = sub_dofs;
  nd.dof_subs.resize(plan.n_coarse);
  for (int64_t k = 0; k < plan.n_coarse; ++k) {
    int32_t o = plan.coarse_obj[k];
    nd.dof_subs[k].assign(c.obj_subs.begin() + c.obj_sptr[o], c.obj_subs.begin() + c.obj_sptr[o + 1]);
  }
  for (int a = 0; a < 3; ++a) {
    nd.cen[a].resize(c.n_sub);
    for (int s = 0; s < c.n_sub; ++s) nd.cen[a][s] = 0.5 * (c.ebox[s][a] + c.ebox[s][3 + a]);
  }
  nd.mark.assign(c.n_sub, 0);
  std::vector<int32_t> all_subs(c.n_sub), all_dofs(plan.n_coarse);
  std::iota(all_subs.begin(), all_subs.end(), 0);
  std::iota(all_dofs.begin(), all_dofs.end(), 0);
  if (c.n_sub == 1) {
    if (plan.n_coarse != 0) return fail(err, -6, "internal: coarse dofs without interface");
    nd.nodes.emplace_back();
    nd.nodes[0].leaves.push_back(0);
  } else if (coarse_solver == 1) {
    nd.nodes.emplace_back();
    nd.nodes[0].P = all_dofs;
    nd.nodes[0].leaves = all_subs;
  } else {
    nd.make(all_subs, all_dofs, -1);
  }
  const int nfr = (int)nd.nodes.size();
  plan.fronts.resize(nfr);
  int64_t off = 0, voff = 0, ioff = 0, poff = 0;
  std::vector<std::unordered_map<int32_t, int32_t>> pos_of(nfr);
  int max_level = 0;
  for (int t = 0; t < nfr; ++t) {
    auto& N = nd.nodes[t];
    FrontDev& F = plan.fronts[t];
    F.p = (int)N.P.size();
    F.n = (int)(N.P.size() + N.B.size());
    F.parent = N.parent;
    F.level = N.level;
    F.off = off;
    F.voff = voff;
    F.idx_off = ioff;
    off += (int64_t)F.n * F.n;
    voff += F.n;
    ioff += F.n;
    if (N.parent >= 0) {
      // the border in the parent's order (parents precede their children
      // here): the extend-add then takes the child's update block lower
      // triangle to the parent's lower triangle, rows in increasing order
      const auto& pp = pos_of[N.parent];
      auto key = [&](int32_t d) {
        auto it = pp.find(d);
        return it == pp.end() ? INT32_MAX : it->second;  // not nested: reported below
      };
      std::stable_sort(N.B.begin(), N.B.end(), [&](int32_t x, int32_t y) { return key(x) < key(y); });
    }
    for (int32_t d : N.P) plan.front_idx.push_back(d);
    for (int32_t d : N.B) plan.front_idx.push_back(d);
    for (int k = 0; k < F.n; ++k) pos_of[t][plan.front_idx[F.idx_off + k]] = k;
    for (int s : N.leaves) plan.subs[s].front = t;
    max_level = std::max(max_level, F.level);
  }
  for (int t = 0; t < nfr; ++t) {
    FrontDev& F = plan.fronts[t];
    F.pmap_off = poff;
    if (F.parent >= 0) {
      for (int k = F.p; k < F.n; ++k) {
        auto it = pos_of[F.parent].find(plan.front_idx[F.idx_off + k]);
        if (it == pos_of[F.parent].end()) return fail(err, -6, "internal: front not nested");
        plan.front_pmap.push_back(it->second);
      }
      poff += F.n - F.p;
    } else if (F.n != F.p) {
      return fail(err, -6, "internal: root front with boundary");
    }
  }
  plan.sub_fmap.resize(plan.c_glob.size());
  for (int s = 0; s < c.n_sub; ++s) {
    SubDev& S = plan.subs[s];
    for (int k = 0; k < S.n_c; ++k) {
      auto it = pos_of[S.front].find(plan.c_glob[S.c_off + k]);
      if (it == pos_of[S.front].end()) return fail(err, -6, "internal: subdomain dof outside its front");
      plan.sub_fmap[S.c_off + k] = it->second;
    }
  }
  // gather assembly: a front's sources are its children and the subdomains
  // it splits off, each with a map from the front's positions to the
  // source's (child border position, or local coarse index; -1: none)
  plan.front_gather = true;
  for (int t = 0; t < nfr; ++t) {
    FrontDev& F = plan.fronts[t];
    const auto& N = nd.nodes[t];
    std::vector<int> src(N.kids.begin(), N.kids.end());
    for (int s : N.leaves) src.push_back(-(s + 1));
    F.nsrc = (int)src.size();
    F.src[0] = F.src[1] = 0;
    F.src_map[0] = F.src_map[1] = 0;
    if (src.size() > 2) {
      plan.front_gather = false;
      continue;
    }
    for (size_t q = 0; q < src.size(); ++q) {
      F.src[q] = src[q];
      F.src_map[q] = (int64_t)plan.front_imap.size();
      if (src[q] >= 0) {
        const FrontDev& C = plan.fronts[src[q]];
        for (int i = 0; i < F.n; ++i) {
          auto it = pos_of[src[q]].find(plan.front_idx[F.idx_off + i]);
          plan.front_imap.push_back(it != pos_of[src[q]].end() && it->second >= C.p ? it->second - C.p : -1);
        }
      } else {
        const SubDev& S = plan.subs[-src[q] - 1];
        std::unordered_map<int32_t, int32_t> loc;
        for (int k = 0; k < S.n_c; ++k) loc[plan.c_glob[S.c_off + k]] = k;
        for (int i = 0; i < F.n; ++i) {
          auto it = loc.find(plan.front_idx[F.idx_off + i]);
          plan.front_imap.push_back(it != loc.end() ? it->second : -1);
        }
      }
    }
  }
  if (!plan.front_gather)
    for (auto& F : plan.fronts) F.nsrc = -1;
  // The front kernels address one front's FP64 entries with 32-bit byte
  // offsets (the front's base pointer is 64-bit): every front must stay
  // below 4 GiB, i.e. fewer than 23,170 rows.
  for (int t = 0; t < nfr; ++t) {
    const FrontDev& F = plan.fronts[t];
    if ((int64_t)F.n * F.n * (int64_t)sizeof(double) >= ((int64_t)1 << 32))
      return fail(err, -1, "coarse front " + std::to_string(t) + " has " + std::to_string(F.n) +
                               " rows: its " + std::to_string((int64_t)F.n * F.n * 8) +
                               " bytes exceed the 4 GiB a front may hold (choose the nested-dissection "
                               "coarse solver, or fewer coarse dofs)");
  }
  plan.front_pool = off;
  plan.front_vec = voff;
  plan.front_idx_total = ioff;
  plan.level_fronts.assign(max_level + 1, {});
  plan.level_slot_children.assign(max_level + 1, {});
  for (int t = 0; t < nfr; ++t) plan.level_fronts[plan.fronts[t].level].push_back(t);
  for (int L = 0; L <= max_level; ++L) {
    for (int t : plan.level_fronts[L]) {
      auto& kids = nd.nodes[t].kids;
      for (size_t j = 0; j < kids.size(); ++j) {
        if (plan.level_slot_children[L].size() <= j) plan.level_slot_children[L].resize(j + 1);
        plan.level_slot_children[L][j].push_back(kids[j]);
      }
    }
  }
  return true;
}

}  // namespace bddcso
