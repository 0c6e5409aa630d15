// Host-side descriptors, interface classification and the solve plan.
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "types.h"

namespace bddcso {

struct Error {
  int code;
  std::string msg;
};

// Mesh, partitions and the classification of Gamma into subobjects
// (Section 3 and Remark 2 on classification).  Independent of the primal
// selection.
struct Classification {
  int dim = 3;
  int64_t ne[3] = {1, 1, 1};   // elements per axis (ne[2] = 1 in 2D)
  double h[3] = {1, 1, 1};
  int64_t nf[3] = {1, 1, 1};   // free nodes per axis (nf[2] = 1 in 2D)
  int64_t n_free = 0, n_elem = 0;
  int n_sub = 0, n_ss = 0;
  std::vector<int32_t> elem_sub, elem_subsub, ss_parent;
  std::vector<std::array<int, 6>> ebox;   // per subdomain: elo[3], ehi[3]
  std::vector<int32_t> ss_eptr, ss_elem;  // elements of each subsubdomain
  // per subsubdomain and axis: rank of its lowest element coordinate among
  // the distinct lowest coordinates of all subsubdomains (the fine
  // partition's grid index for tensor partitions)
  std::vector<std::array<int, 3>> ss_idx;
  // Gamma nodes (free nodes shared by >= 2 subdomains), ascending free index
  std::vector<int64_t> gam_node;
  std::vector<int32_t> node_gam;          // free index -> Gamma index or -1
  std::vector<int32_t> gam_kptr, gam_key; // key: sorted subsubdomain ids
  std::vector<int32_t> gam_obj;           // Gamma index -> object
  // objects, numbered by their smallest free index
  std::vector<int32_t> obj_ptr, obj_gam;  // Gamma indices of each object
  std::vector<int8_t> obj_type;           // 1 vertex, 2 edge, 4 face
  std::vector<int32_t> obj_sptr, obj_subs;// subdomains of each object

  int n_obj() const { return (int)obj_type.size(); }
  void node_coords(int64_t free_idx, int g[3]) const {
    g[0] = (int)(free_idx % nf[0]) + 1;
    int64_t t = free_idx / nf[0];
    g[1] = (int)(t % nf[1]) + 1;
    g[2] = dim == 3 ? (int)(t / nf[1]) + 1 : 1;
  }
  int64_t free_index(const int g[3]) const {
    return (int64_t)(g[0] - 1) + nf[0] * ((int64_t)(g[1] - 1) + nf[1] * (int64_t)(g[2] - 1));
  }
};

// Everything that depends on the primal selection and the options but not on
// the coefficient: per-subdomain index tables, blocks, coarse numbering, the
// nested-dissection tree of the coarse problem, pool sizes.
struct Plan {
  int primal_mask = 7;
  int block_target = 192;
  int coarse_solver = 0;
  int64_t n_coarse = 0;
  std::vector<int32_t> coarse_obj;   // coarse id -> object
  std::vector<int32_t> obj_coarse;   // object -> coarse id or -1

  std::vector<SubDev> subs;
  std::vector<int32_t> loc_I, loc_r, loc_g;   // per local node: rank in I / r / Gamma entries, -1
  std::vector<int32_t> I_loc, r_loc;          // set order -> local node
  std::vector<int32_t> z_col;                 // per local coarse entry j (average j < n_a, else
                                              // vertex j - n_a): its column of [X | Y']
  std::vector<int32_t> kig_ptr;               // per interior node (all subdomains): its Gamma neighbours
  std::vector<int8_t> kig_t;                  //   as 27-point neighbour codes
  std::vector<int32_t> kig_own, kig_sub;      //   per entry: its interior node (global I order), subdomain
  std::vector<int32_t> kgi_ptr;               // per Gamma entry (all subdomains): its interior neighbours
  std::vector<int8_t> kgi_t;                  //   as 27-point neighbour codes
  std::vector<int32_t> kgi_own;               //   per entry: its Gamma entry (global order)
  std::vector<int32_t> g_loc, g_gam, g_r, g_v, g_sub; // per Gamma entry
  std::vector<int32_t> loc_sel;   // per local node: selected-row index or -1
  std::vector<int32_t> sel_r;     // per selected row: r rank (-1 at primal vertices)
  std::vector<int32_t> v_loc, v_c;            // per vertex: local node, local coarse index
  std::vector<int32_t> a_ptr, a_r, a_c;       // averages: CSR of r ranks; local coarse index
  std::vector<int32_t> a_g;                   // per a_r entry: its Gamma-local index (= selected row)
  std::vector<int32_t> c_glob, c_kind;        // per local coarse: global id; vertex idx or -(a+1)
  std::vector<BlockDev> blocks;
  // plane couplings between consecutive blocks: per row (a node of a block's
  // first or last plane) the set ranks of its 9 (3 in 2D) neighbours in the
  // adjacent plane, -1 where absent
  std::vector<int32_t> cpl_rank, cpl_sub, cpl_loc, cpl_dir;
  // per coupling row of a first plane (dir -1), the block-local ranks of its
  // in-plane stencil neighbours of rank at most its own (itself, then x-1;
  // in 3D also (x-1, y-1), (x, y-1), (x+1, y-1)), -1 where absent or on a
  // last-plane row: the entries of A_kk that the Schur coupling adds itself
  std::vector<int32_t> ipl_rank;

  std::vector<int32_t> gam_eptr, gam_ent;     // Gamma index -> Gamma entries
  std::vector<int32_t> crs_eptr, crs_ent;     // coarse id -> local coarse entries
  std::vector<std::vector<int32_t>> color_subs;

  // coarse tree
  std::vector<FrontDev> fronts;
  std::vector<int32_t> front_idx;             // coarse ids of front positions
  std::vector<int32_t> front_pmap;            // positions p..n-1 -> parent positions
  std::vector<int32_t> front_imap;            // gather maps (FrontDev::src_map)
  bool front_gather = true;                   // every front has at most 2 sources
  std::vector<int32_t> sub_fmap;              // local coarse entry -> position in its front
  std::vector<std::vector<int32_t>> level_fronts;       // fronts per level (bottom-up)
  std::vector<std::vector<std::vector<int32_t>>> level_slot_children; // [level][slot] children
  int64_t front_pool = 0, front_vec = 0, front_idx_total = 0;

  // totals
  int64_t tot_loc = 0, tot_I = 0, tot_r = 0, tot_g = 0, tot_v = 0, tot_a = 0, tot_c = 0;
  int64_t pool_G = 0, pool_Z = 0, pool_XG = 0, pool_Sc = 0, pool_T = 0, pool_PhiG = 0, pool_YG = 0, pool_Kc = 0;
  int max_block = 0, max_na = 0, max_nc = 0, max_nr = 0, max_nloc = 0, max_ng = 0, max_ns = 0;
  int max_nbI = 0, max_nbR = 0;
  int max_zcols = 0;
};

// Builds the classification; returns false and fills err on invalid input.
bool classify(int dim, const int64_t n_el[3], const double h[3], const int32_t* elem_sub,
              const int32_t* elem_subsub, Classification& c, Error& err);

bool build_plan(const Classification& c, int primal_mask, int block_target, int coarse_solver,
                Plan& plan, Error& err);

// Primal selection bit 8: keep half of the codimension-one objects (faces in
// 3D, edges in 2D), by the checkerboard rule of half_keep.
constexpr int kHalfCodim1 = 8;

// True when the object (key of two subsubdomains j1 < j2) is kept by the
// half selection: the sum of j1's grid indices over the axes other than the
// normal (the axis along which j1 and j2 differ most, the first on ties) is
// even.
bool half_keep(const Classification& c, int obj);

int object_type(int dim, int key_size);

}  // namespace bddcso
