// Device kernels of the BDDC-SO path and their host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "types.h"

namespace bddcso {

// Pivots per panel of the batched sweeps (scratch per matrix: 2 slots of
// n x kSweepNB + kSweepNB^2 entries).
constexpr int kSweepNB = 32;
// Pivots per slab when sweeping matrices above 272 rows; their scratch needs
// n x kSlab entries per matrix.
constexpr int kSlab = 192;
// Largest matrix swept by the register-resident kernel (one workgroup per
// matrix); larger ones take the slab path.
constexpr int kRegSweepMaxRows = 304;

// Geometry passed by value to kernels.
struct Geo {
  int dim;
  int ne[3];        // elements per axis (ne[2] = 1 in 2D)
  int nf[3];        // free nodes per axis (nf[2] = 1 in 2D)
  int64_t n_free, n_elem;
};

// Records HIP events around the launches of one kernel class, with the
// algorithmic flops and bytes of each launch.  Classes: 1 sweep update,
// 2 block solve, 3 batched GEMM, 4 sweep panel.
struct Profiler {
  virtual ~Profiler() {}
  virtual void begin(int cls, hipStream_t s) = 0;
  virtual void end(int cls, double flops, double bytes, hipStream_t s) = 0;
};

// A second stream and two events for the slab sweep's look-ahead: the next
// slab's pivot block is swept on s2 while the current trailing update runs.
struct SweepAux {
  hipStream_t s2;
  hipEvent_t a, b, c;
};

// Device views of the plan tables.
struct PlanDev {
  const SubDev* subs;
  const BlockDev* blocks;
  const int32_t *loc_I, *loc_r, *loc_g;
  const int32_t *I_loc, *r_loc;
  const int32_t* z_col;     // per local coarse entry (c_off order: averages, then vertices): its column of [X | Y']
  const int32_t* kig_ptr;   // per interior node (global I order) into the K_{I Gamma} entries
  const int8_t* kig_t;      // neighbour code of each entry
  const int32_t *kig_own, *kig_sub;  // interior node (global I order) and subdomain of each entry
  int64_t n_kig;
  int32_t* kig_col;         // free index of the neighbour (filled by the setup)
  double* kig_val;          // K_{I Gamma} entry (filled by the setup from rho)
  const int32_t* kgi_ptr;   // per Gamma entry (global order) into the K_{Gamma I} entries
  const int8_t* kgi_t;      // neighbour code of each entry
  const int32_t* kgi_own;   // Gamma entry (global order) of each entry
  int64_t n_kgi;
  int32_t* kgi_col;         // interior index of the neighbour in its subdomain (filled by the setup)
  double* kgi_val;          // K_{Gamma I} entry (filled by the setup from rho)
  const int32_t *g_loc, *g_gam, *g_r, *g_v, *g_sub;
  const int32_t *loc_sel, *sel_r;
  const int32_t *v_loc, *v_c;
  const int32_t *a_ptr, *a_r, *a_g, *a_c;  // a_g: selected row (Gamma entry) of each a_r node
  const int32_t *c_glob, *c_kind;
  const int32_t *gam_eptr, *gam_ent;
  const int64_t* gam_node;
  const int32_t *gam_kptr, *gam_key, *ss_parent, *ss_eptr, *ss_elem;
  const int32_t *crs_eptr, *crs_ent;
  const FrontDev* fronts;
  const int32_t *front_idx, *front_pmap, *sub_fmap, *front_imap;
  // per front vector entry and scatter slot: the vector index of the child
  // border value the entry receives, -1 for none ([entry][n_slot])
  const int32_t* front_pull;
  int n_slot;
  const double* khat;  // 8x8 unit-coefficient element matrix (2D replicated over the z bit)
  const int32_t *cpl_rank, *cpl_sub, *cpl_loc, *cpl_dir;
  const double* cpl_coef;  // 9 coefficients per coupling row (filled at setup)
  const int32_t* ipl_rank;  // 5 in-plane lower stencil ranks per coupling row (block-local, -1: none)
  const double* ipl_coef;   // their A_kk entries (filled at setup)
  int64_t n_cpl;
  int n_sub;
  int64_t tot_I, tot_r, tot_g, tot_c, tot_a, n_gam, n_coarse;
  int max_block, max_na, max_nc, max_ng, max_ns, max_nloc, max_nr, max_nI, max_zcols, max_plane, max_nv;
  int max_nar;    // r-set nodes of one subdomain's averages
  int n_pinned;  // subdomains with a pin (SubDev::pin >= 0)
  int mr_min;    // right-hand sides from which the many-RHS kernels run
};

// ---- launchers (defined in kernels.hip) ---------------------------------
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s, int max_blocks = 65536);
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
// the primal vertices' stencil coefficients and codes (k_kc_identity's input)
void launch_vertex_stencil(const PlanDev& P, const Geo& g, const double* rho, double* vcoef, int32_t* vcode,
                           int max_nv, hipStream_t s);
// the K_{I Gamma} entries of every interior node (free index of the Gamma
// neighbour and the stiffness entry from rho) and the K_{Gamma I} entries of
// every Gamma entry (interior index of the neighbour and the entry)
void launch_kig_fill(const PlanDev& P, const Geo& g, const double* rho, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

void launch_q1_apply(const Geo& g, const double* khat, const double* rho, const double* x,
                     double* y, int nrhs, hipStream_t s);
void launch_alpha(const PlanDev& P, int n_ss, const double* rho, int weighting, double* alpha,
                  hipStream_t s);
void launch_delta(const PlanDev& P, const double* alpha, double* delta, hipStream_t s);
void launch_coupling_coefs(const PlanDev& P, const Geo& g, const double* rho, double* coef, double* icoef,
                           hipStream_t s);

template <typename T>
struct Kern {
  // setup
  static void block_assemble(const PlanDev& P, const Geo& g, const double* rho, int setR, T* G, int max_nb,
                             hipStream_t s);
  static void schur_couple(const PlanDev& P, int setR, int k, T* G, hipStream_t s);
  // reg_max: largest matrix of the register-resident sweep; lookahead: slab
  // look-ahead mode (0 by the update's size, 1 none, 2 always beside);
  // utile: tile rows of the slab trailing update (64 or 128); slab_w: slab
  // width (0 by the batch, 96 or 192)
  static void sweep(SweepDesc* d_desc, const SweepDesc* h_desc, int nprob, int maxn, int maxp, T* pool,
                    T* scratch, int64_t scr_stride, int* status, int status_code, hipStream_t s,
                    Profiler* prof, const SweepAux* aux = nullptr, int reg_max = kRegSweepMaxRows,
                    int lookahead = 0, int utile = 64, int slab_w = 0);
  static void gemm(const GemmDesc* d_desc, const GemmDesc* h_desc, int nprob, int maxm, int maxn,
                   const T* A, int transA, const T* B, int transB, T* C, T alpha, T beta, hipStream_t s,
                   Profiler* prof);
  static void rhs_fill(const PlanDev& P, const Geo& g, const double* rho, T* Z, hipStream_t s);
  static void couple_multi(const PlanDev& P, const Geo& g, const double* rho, int k, int fwd,
                           int ncols_max, T* Z, T* tmp, int64_t tmp_stride, hipStream_t s, int sub0, int nsub);
  static void object_means(const PlanDev& P, const T* Z, T* XG, T* Sc, T* Tv, T* PhiG, T* YG, hipStream_t s);
  // rows of [X | Phi initialised to Y'] at the selected rows
  static void lam_assemble(const PlanDev& P, const T* Sc, const T* LV, T* Lam, hipStream_t s);
  // also writes Y' at the Gamma entries (YG)
  static void kc_identity(const PlanDev& P, const Geo& g, const double* rho, const T* PS,
                          const T* Lam, T* Kc, double* vcoef, int32_t* vcode, int max_nv, hipStream_t s);
  static void kc_to_front(const PlanDev& P, const int32_t* subs_of_color, int ns, const T* Kc,
                          double* fpool, hipStream_t s);
  // every front of a level assembled from its sources (gather plans only)
  static void front_gather(const PlanDev& P, const int32_t* fr, int nfr, int maxn, const T* Kc, double* fpool,
                           hipStream_t s);
  // per-iteration
  static void gather_I(const PlanDev& P, const Geo& g, const double* r, T* vI, int nrhs, hipStream_t s);
  static void block_solve(const PlanDev& P, const Geo& g, const double* rho, int setR, const T* G,
                          T* v, int nrhs, hipStream_t s, Profiler* prof, double g_entries,
                          double vec_entries, int set_max_block);
  static void gamma_kgi(const PlanDev& P, const Geo& g, const double* rho, const T* vI, T* q,
                        int nrhs, hipStream_t s);
  static void gamma_t(const PlanDev& P, const Geo& g, const double* r, const T* q, const double* delta,
                      T* gv, int nrhs, hipStream_t s);
  static void neumann_rhs(const PlanDev& P, const T* gv, T* vR, int nrhs, hipStream_t s);
  static void mu(const PlanDev& P, const T* vR, const T* Sc, T* mu_out, int nrhs, hipStream_t s);
  static void coarse_rhs_local(const PlanDev& P, const T* XG, const T* PhiG, const T* Lam, const double* eps,
                               const T* gv, T* wv, T* bci, int nrhs,
                               hipStream_t s);
  // v2 on Gamma = u - X_Gamma (mu + Lambda u_c) + Y'_Gamma u_c (equal to
  // u - X_Gamma mu + Phi_Gamma u_c, as Phi = Y' - X Lambda)
  static void v2(const PlanDev& P, const T* vR, const T* XG, const T* mu_in, const T* lu, const T* YG,
                 const double* uc, T* v2_out, int nrhs, hipStream_t s);
  // lu = Lambda u_c per subdomain (the local coarse values of u_c)
  static void lam_uc(const PlanDev& P, const T* Lam, const double* uc, T* lu, int nrhs, hipStream_t s);
  // pinned subdomains (SubDev::pin): the constant of the local kernel
  static void float_setup(const PlanDev& P, const T* Sc, T* Lam, double* eps, double* fdelta, hipStream_t s);
  static void float_mu(const PlanDev& P, const T* gv, T* mu_io, const double* eps, const double* fdelta,
                       double* fc, int nrhs, hipStream_t s);
  static void float_v2(const PlanDev& P, const double* uc, const double* eps, const double* fc, T* v2, int nrhs,
                       hipStream_t s);
  // Y' at the Gamma entries, from [X | Y']
  static void interior_rhs(const PlanDev& P, const Geo& g, const double* rho, const double* r,
                           const double* w, T* vI, int nrhs, hipStream_t s);
  static void scatter_I(const PlanDev& P, const Geo& g, const T* vI, double* z, int nrhs, hipStream_t s);
};

void launch_gamma_w(const PlanDev& P, const Geo& g, const double* v2_d, const float* v2_f,
                    const double* delta, double* z, int nrhs, hipStream_t s);
void launch_front_zero_lower(const PlanDev& P, const int32_t* fronts, int nfr, int maxn, double* fpool,
                             hipStream_t s);
void launch_front_child_scatter(const PlanDev& P, const int32_t* children, int nchild, int maxn,
                                double* fpool, hipStream_t s);
void launch_front_vec_init(const PlanDev& P, const int32_t* fr, int nfr, int maxn, const double* bci_d,
                           const float* bci_f, double* fvec, int64_t fvec_stride, int nrhs, hipStream_t s);
void launch_front_vec_scatter(const PlanDev& P, const int32_t* children, int nchild, int maxn,
                              double* fvec, int64_t fvec_stride, int nrhs, hipStream_t s);
// pull: with part (the chunked single-RHS form), the entries take their
// children's border values themselves (P.front_pull, in slot order) instead
// of a preceding launch_front_vec_scatter
void launch_front_fwd(const PlanDev& P, const int32_t* fr, int nfr, int maxn, int maxp,
                      const double* fpool, double* fvec, double* xh, int64_t fvec_stride,
                      int nrhs, hipStream_t s,
                      double* part = nullptr, bool pull = false);
void launch_front_bwd(const PlanDev& P, const int32_t* fr, int nfr, int maxp, int maxb,
                      const double* fpool, const double* xh, int64_t fvec_stride, double* uc,
                      int nrhs, hipStream_t s);
void launch_kc_to_f64(const float* src, double* dst, int64_t n, hipStream_t s);

// PCG helpers.  Scalars live on the device: dots[slot*nrhs + j].
void launch_dot(const double* a, const double* b, int64_t n, int nrhs, double* partial,
                int nblocks, double* out, hipStream_t s);
void launch_pcg_xr(double* x, double* r, const double* p, const double* q, const double* rz,
                   const double* pq, const int32_t* active, int64_t n, int nrhs, hipStream_t s);
void launch_pcg_p(double* p, const double* z, const double* rz_new, const double* rz_old,
                  const int32_t* active, int64_t n, int nrhs, hipStream_t s);
void launch_pcg_p_flex(double* p, const double* z, const double* zdr, const double* rz_old,
                       const int32_t* active, int64_t n, int nrhs, hipStream_t s);
void launch_sub(const double* a, const double* b, double* out, int64_t n, hipStream_t s);
void launch_copy16(const void* a, void* b, int64_t n16, hipStream_t s);
int kc_cols(const PlanDev& P);
int64_t max_lds_bytes(const PlanDev& P, int elt, int max_nrhs);
// Chunks of pivot columns of the split forward front step (partial-sum rows).
int front_fwd_chunks(int maxp);

void launch_element_grad(const Geo& g, const double* khat, const double* rho, const double* u,
                         const double* lam, double* out, int nrhs, hipStream_t s);
// mode 0: box mean F; 1: its transpose; 2: exp of the box mean
void launch_box_filter(const Geo& g, const double* in, double* out, int mode, hipStream_t s);

}  // namespace bddcso

namespace bddcso {
// PCG bookkeeping; kd: the iteration index in device memory (advanced by
// book2), or nullptr to use k.
void launch_pcg_book1(int nrhs, int k, const int32_t* kd, const double* rz, const double* pq, const double* rr,
                      const double* tol2, int32_t* active, int32_t* iters, int32_t* flags, double* hist_alpha,
                      int32_t* nactive, hipStream_t s);
void launch_pcg_book2(int nrhs, int k, int32_t* kd, double* rz, const double* num, const double* rz_new,
                      const int32_t* active, double* hist_beta, hipStream_t s);
void launch_copy_f64(const double* a, double* b, int64_t n, hipStream_t s);
}  // namespace bddcso
