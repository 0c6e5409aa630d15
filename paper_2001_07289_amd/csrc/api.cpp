// C ABI of the BDDC-SO solver: planning, device memory, setup, the
// preconditioner application and the PCG driver.  Every numeric step runs in
// the kernels of kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bddcso.h"
#include "kernels.h"
#include "plan.h"

using namespace bddcso;

namespace {

thread_local std::string g_last_error;

bddcso_status set_err(bddcso_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

struct HipFail {
  hipError_t e;
  std::string where;
};

#define HIPCHK(x)                                                        \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) throw HipFail{e_, std::string(#x)};            \
  } while (0)

// The unit-coefficient Q1 element matrix, indexed [a*8+b] with local node
// a = bit x + 2 bit y + 4 bit z.  It is the tensor sum of 1D stiffness
// (1/h)[1 -1; -1 1] and mass h/6 [2 1; 1 2] factors.  In 2D the z bit is
// ignored (the table is replicated over it).
void element_table(int dim, const double h[3], double out[64]) {
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) {
      double k[3], m[3];
      for (int d = 0; d < 3; ++d) {
        bool same = ((a >> d) & 1) == ((b >> d) & 1);
        k[d] = (same ? 1.0 : -1.0) / h[d];
        m[d] = h[d] * (same ? 2.0 : 1.0) / 6.0;
      }
      out[a * 8 + b] = dim == 3 ? k[0] * m[1] * m[2] + m[0] * k[1] * m[2] + m[0] * m[1] * k[2]
                                : k[0] * m[1] + m[0] * k[1];
    }
}

// Extreme eigenvalues of a symmetric tridiagonal matrix by Sturm-sequence
// bisection (Wilkinson, The Algebraic Eigenvalue Problem, ch. 5).
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    double off = i ? e[i - 1] * e[i - 1] : 0.0;
    q = d[i] - x - (i ? off / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}

void tridiag_extremes(const std::vector<double>& d, const std::vector<double>& e, double& lo, double& hi) {
  const int n = (int)d.size();
  if (n == 0) {
    lo = hi = 1.0;
    return;
  }
  double a = 1e300, b = -1e300;
  for (int i = 0; i < n; ++i) {
    double r = (i ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
    a = std::min(a, d[i] - r);
    b = std::max(b, d[i] + r);
  }
  auto kth = [&](int k) {  // k-th smallest eigenvalue, 0-based
    double l = a, u = b;
    for (int it = 0; it < 200; ++it) {
      double mid = 0.5 * (l + u);
      if (sturm_count(d, e, mid) > k) u = mid;
      else l = mid;
      if (u - l <= 1e-15 * std::max(std::fabs(l), std::fabs(u))) break;
    }
    return 0.5 * (l + u);
  };
  lo = kth(0);
  hi = kth(n - 1);
}

// Device memory of one preconditioner.  Three modes share one allocation
// sequence: MALLOC (the library allocates each buffer), COUNT (host only:
// sums the aligned sizes, returns placeholder addresses that are never
// dereferenced, copies nothing) and CARVE (buffers are cut, in the same
// order, from a caller-owned workspace).
struct WorkspaceShort {
  size_t need, have;
};

struct DevMem {
  enum Mode { MALLOC, COUNT, CARVE } mode = MALLOC;
  static constexpr size_t kAlign = 256;
  char* base = nullptr;  // CARVE: the workspace
  size_t cap = 0;        // CARVE: its size
  size_t used = 0;       // COUNT / CARVE: bytes laid out so far
  std::vector<void*> ptrs;
  int64_t bytes = 0;
  template <typename T>
  T* alloc(int64_t n) {
    if (n <= 0) n = 1;
    const size_t b = (size_t)n * sizeof(T);
    if (mode == MALLOC) {
      void* p = nullptr;
      HIPCHK(hipMalloc(&p, b));
      ptrs.push_back(p);
      bytes += (int64_t)b;
      return (T*)p;
    }
    const size_t off = (used + kAlign - 1) / kAlign * kAlign;
    used = off + b;
    bytes = (int64_t)used;
    if (mode == COUNT) return (T*)(uintptr_t)(kAlign + off);
    if (used > cap) throw WorkspaceShort{used, cap};
    return (T*)(base + off);
  }
  template <typename T>
  T* upload(const std::vector<T>& v, hipStream_t s) {
    T* p = alloc<T>((int64_t)v.size());
    if (mode != COUNT && !v.empty())
      HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

struct GraphPair {
  hipGraphExec_t g1 = nullptr, g2 = nullptr;
};

struct Batch {
  void* desc = nullptr;  // device descriptor array
  int n = 0, maxm = 0, maxn = 0, maxp = 0;
  std::vector<GemmDesc> hg;   // host copies (work accounting)
  std::vector<SweepDesc> hs;
};

// Kernel classes timed by the profiler (bit c of the mask records class c):
// 1 sweep_update, 2 block_solve, 3 gemm, 4 sweep_panel, 5 sweep_small,
// 6 schur_couple, 7 couple_multi, 8 q1_apply.
constexpr int kNumClasses = 8;

struct EventProfiler : Profiler {
  int mask = 0;  // bit c: record class c
  struct Rec {
    std::vector<hipEvent_t> ev;  // begin/end pairs
    size_t used = 0;
    double flops = 0, bytes = 0;          // as executed by the kernels
    double ref_flops = 0, ref_bytes = 0;  // the reference count of the same work
    int64_t launches = 0;
  } rec[kNumClasses + 1];
  bool on(int c) const { return c >= 1 && c <= kNumClasses && (mask & (1 << c)); }
  hipEvent_t next(Rec& r) {
    if (r.used == r.ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      r.ev.push_back(e);
    }
    return r.ev[r.used++];
  }
  void begin(int c, hipStream_t s) override {
    if (!on(c)) return;
    hipEvent_t e = next(rec[c]);
    if (e) (void)hipEventRecord(e, s);
  }
  void end(int c, double f, double b, hipStream_t s) override {
    if (!on(c)) return;
    hipEvent_t e = next(rec[c]);
    if (e) (void)hipEventRecord(e, s);
    rec[c].flops += f;
    rec[c].bytes += b;
    ++rec[c].launches;
  }
  // work of launches booked under class c by the reference count (banded
  // Cholesky factors and triangular solves), added beside the executed count
  void ref(int c, double f, double b) {
    if (!on(c)) return;
    rec[c].ref_flops += f;
    rec[c].ref_bytes += b;
  }
  void reset(int m) {
    mask = m;
    for (auto& r : rec) {
      r.used = 0;
      r.flops = r.bytes = r.ref_flops = r.ref_bytes = 0;
      r.launches = 0;
    }
  }
  ~EventProfiler() override {
    for (auto& r : rec)
      for (hipEvent_t e : r.ev) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct bddcso_problem {
  Classification c;
  std::map<std::tuple<int, int, int>, std::shared_ptr<Plan>> plans;
  double khat[64];
};

namespace {

template <typename T>
struct Numeric {
  T *G = nullptr, *Z = nullptr, *XG = nullptr, *Sc = nullptr, *Tm = nullptr, *Lam = nullptr,
    *PhiG = nullptr, *YG = nullptr, *Kc = nullptr;
  T *tmp = nullptr, *sw = nullptr, *sw2 = nullptr;
  int64_t tmp_stride = 0, sw_stride = 0;
  // per-iteration
  T *vI = nullptr, *vR = nullptr, *q = nullptr, *gv = nullptr, *v2 = nullptr, *mu = nullptr, *bci = nullptr;
  T* lu = nullptr;  // Lambda u_c per subdomain (averages), from the coarse solve
};

}  // namespace

struct bddcso_precond {
  bddcso_problem* prob = nullptr;
  std::shared_ptr<Plan> plan;
  bddcso_options opt{};
  Geo geo{};
  PlanDev P{};
  DevMem mem;
  int precision = 0;
  Numeric<double> nd;
  Numeric<float> nf;
  double *rho = nullptr, *alpha = nullptr, *delta = nullptr, *khat = nullptr, *cpl_coef = nullptr;
  double* ipl_coef = nullptr;  // in-plane A_kk entries of the first-plane coupling rows
  double* vcoef = nullptr;    // stencil rows of the primal vertices (27 per vertex)
  int32_t* vcode = nullptr;
  int max_nv = 0;
  double *fpool = nullptr, *fsw = nullptr, *uc = nullptr, *fvec = nullptr, *xh = nullptr;
  double* fpart = nullptr;  // partial products of the split forward front step (few right-hand sides)
  int64_t fsw_stride = 0;
  int32_t* status = nullptr;
  // batches
  std::vector<std::vector<Batch>> swI, swR;  // per block index k: size buckets
  std::vector<Batch> gfwd[2], gbwd[2];  // block GEMMs of the basis solves, per half of the subdomains
  int zsplit = 0;                       // first subdomain of the second half
  std::vector<Batch> swSc;                          // size buckets
  Batch gLam, gSel;
  std::vector<std::vector<Batch>> swFront;          // per level: size buckets
  std::vector<int32_t*> color_dev;                  // per colour
  std::vector<int> color_n;
  std::vector<std::vector<int32_t*>> slot_dev;      // [level][slot]
  std::vector<std::vector<int>> slot_n, slot_maxn;
  std::vector<int32_t*> level_dev;
  std::vector<int> level_n, level_maxn, level_maxp, level_maxb;
  int32_t* all_fronts = nullptr;  // every front, all levels (one launch initialises their vectors)
  int all_n = 0, all_maxn = 0;
  // PCG
  double *r = nullptr, *p = nullptr, *qv = nullptr, *z = nullptr, *rold = nullptr, *dtmp = nullptr;
  double* partial = nullptr;
  int dot_blocks = 512;
  double* sc = nullptr;  // scalar slots, 8 x max_nrhs
  double *hist_a = nullptr, *hist_b = nullptr;
  int32_t *active = nullptr, *iters = nullptr, *flags = nullptr, *nactive = nullptr;
  int32_t* h_nactive = nullptr;  // pinned
  int max_nrhs = 1;
  int64_t generation = 0;  // numeric setups done (bddcso_refactor calls)
  // graph mode (options.graph): capture stream, the numeric setup's graph,
  // and per right-hand-side count the two halves of a PCG iteration
  hipStream_t sg = nullptr;
  // coarse factorization stream: in ordinary (non-graph) mode the setup
  // leaves it running and the next preconditioner application's coarse
  // solve waits for it, so that application's local solves overlap the
  // latency-bound upper levels of the factorization
  hipStream_t s4 = nullptr;
  hipEvent_t ev_kc = nullptr, ev_coarse = nullptr;
  bool coarse_pending = false;
  hipGraphExec_t g_setup = nullptr;
  std::map<int, GraphPair> iter_graphs;
  double* xk = nullptr;      // x of graph-mode solves [max_nrhs][n_free]
  // pinned subdomains: e / delta per average, delta per subdomain, and the
  // constant c of the last Neumann solves per (rhs, subdomain)
  double *feps = nullptr, *fdelta = nullptr, *fc = nullptr;
  int32_t* kdev = nullptr;   // iteration index of graph-mode solves
  EventProfiler prof;
  hipStream_t s2 = nullptr;                 // second stream of the setup
  hipStream_t s3 = nullptr;                 // third stream: the interior factors
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_fork_i = nullptr, ev_join_i = nullptr;
  hipEvent_t ev_cfork = nullptr, ev_cjoin = nullptr;  // coarse solve beside the Neumann solves
  hipEvent_t ev_cpl = nullptr;                         // plane-coupling coefficients ready
  hipEvent_t ev_la = nullptr, ev_lb = nullptr, ev_lc = nullptr;  // slab look-ahead of the coarse fronts
  hipEvent_t ev_zf = nullptr, ev_zj = nullptr;  // fork and join of the two halves of the basis solves
  double gI_entries = 0, gR_entries = 0;  // G entries streamed by one block solve
  // Reference counts (lexicographic band factors of each subdomain, bandwidth
  // b = m_x m_y + m_x + 1 in 3D, m_x + 1 in 2D): band entries of L_I and L_r,
  // banded Cholesky flops n b^2 per diagonal block of the two chains, and
  // the banded forward and backward solves of [X | Y'] (4 nnz(L_r) flops
  // per column).  Executed counts of the coupling kernels per launch.
  double refI_nnz = 0, refR_nnz = 0, ref_basis_flops = 0;
  std::vector<double> refI_potrf, refR_potrf;           // per block index k
  std::vector<double> sc_flops[2], sc_bytes[2];         // schur_couple, per set and k
  std::vector<double> cm_flops[2][2], cm_bytes[2][2];   // couple_multi, [half][fwd], per k
  int max_block_I = 0, max_block_R = 0;   // largest diagonal block of each set
  Profiler* P_() { return prof.mask ? &prof : nullptr; }
};

namespace {

template <typename T>
Numeric<T>& num(bddcso_precond* pc);
template <>
Numeric<double>& num<double>(bddcso_precond* pc) {
  return pc->nd;
}
template <>
Numeric<float>& num<float>(bddcso_precond* pc) {
  return pc->nf;
}

// Host-side guard run once per setup: every descriptor a batched kernel will
// index must lie inside the pool it addresses, so a planning mistake is an
// error status rather than an out-of-bounds device access.
struct PlanFail {
  std::string what;
};

int64_t extent(int64_t off, int rows, int cols, int ld) {
  return rows <= 0 || cols <= 0 ? off : off + (int64_t)(cols - 1) * ld + rows;
}

void check_sweeps(const std::vector<SweepDesc>& v, int64_t pool, int64_t scratch_slots, const char* name) {
  if ((int64_t)v.size() > scratch_slots)
    throw PlanFail{std::string(name) + ": more problems than sweep scratch slots"};
  for (const SweepDesc& d : v) {
    if (d.off < 0 || d.p < 0 || d.p > d.n || d.ld < d.n || extent(d.off, d.n, d.n, d.ld) > pool)
      throw PlanFail{std::string(name) + ": sweep descriptor outside its pool"};
    // the sweep kernels address a matrix's entries by 32-bit byte offsets
    if ((int64_t)d.n * d.ld * (int64_t)sizeof(double) >= ((int64_t)1 << 32))
      throw PlanFail{std::string(name) + ": a matrix of " + std::to_string(d.n) + " rows exceeds 4 GiB"};
  }
}

// Non-transposed operands: A is m x k, B is k x n, C is m x n (column-major).
void check_gemms(const std::vector<GemmDesc>& v, int64_t pa, int64_t pb, int64_t pcx, const char* name) {
  for (const GemmDesc& d : v)
    if (d.a < 0 || d.b < 0 || d.c < 0 || d.lda < d.m || d.ldb < d.k || d.ldc < d.m ||
        extent(d.a, d.m, d.k, d.lda) > pa || extent(d.b, d.k, d.n, d.ldb) > pb || extent(d.c, d.m, d.n, d.ldc) > pcx)
      throw PlanFail{std::string(name) + ": GEMM descriptor outside its pools"};
}

Batch make_gemm_batch(DevMem& mem, const std::vector<GemmDesc>& v, hipStream_t s) {
  Batch b;
  b.n = (int)v.size();
  for (auto& d : v) {
    b.maxm = std::max(b.maxm, d.m);
    b.maxn = std::max(b.maxn, d.n);
  }
  b.desc = mem.upload(v, s);
  b.hg = v;
  return b;
}

Batch make_sweep_batch(DevMem& mem, const std::vector<SweepDesc>& v, hipStream_t s) {
  Batch b;
  b.n = (int)v.size();
  for (auto& d : v) {
    b.maxn = std::max(b.maxn, d.n);
    b.maxp = std::max(b.maxp, d.p);
  }
  b.desc = mem.upload(v, s);
  b.hs = v;
  return b;
}

// Splits a batch of sweeps into buckets by the register-sweep instance
// their sizes need (the instance of a launch follows its largest matrix),
// so that small matrices of an uneven batch run at their own instance's
// occupancy; matrices above the register sweep form the last bucket.
std::vector<Batch> make_sweep_buckets(DevMem& mem, const std::vector<SweepDesc>& v, hipStream_t s, int reg_max) {
  const int lim[] = {64, 128, 176, 192, 272, kRegSweepMaxRows, INT32_MAX};
  std::vector<std::vector<SweepDesc>> g(7);
  for (const SweepDesc& d : v) {
    int c = 0;
    if (d.n > reg_max) c = 6;
    else
      while (d.n > lim[c]) ++c;
    g[c].push_back(d);
  }
  std::vector<Batch> out;
  for (auto& b : g)
    if (!b.empty()) out.push_back(make_sweep_batch(mem, b, s));
  return out;
}

template <typename T>
void alloc_numeric(bddcso_precond* pc, hipStream_t s) {
  const Plan& pl = *pc->plan;
  Numeric<T>& N = num<T>(pc);
  DevMem& m = pc->mem;
  const int nr = pc->max_nrhs;
  N.G = m.alloc<T>(pl.pool_G);
  N.Z = m.alloc<T>(pl.pool_Z);
  N.XG = m.alloc<T>(pl.pool_XG);
  N.Sc = m.alloc<T>(pl.pool_Sc);
  N.Tm = m.alloc<T>(pl.pool_T);
  N.Lam = m.alloc<T>(pl.pool_T);
  N.PhiG = m.alloc<T>(pl.pool_PhiG);
  N.YG = m.alloc<T>(pl.pool_YG);
  N.Kc = m.alloc<T>(pl.pool_Kc);
  N.tmp_stride = (int64_t)pl.max_block * std::max(pl.max_zcols, 1);
  N.tmp = m.alloc<T>(N.tmp_stride * pl.subs.size());
  int maxsw = std::max(pl.max_block, pl.max_na);
  N.sw_stride = std::max<int64_t>(2 * ((int64_t)maxsw * kSweepNB + kSweepNB * kSweepNB), (int64_t)maxsw * kSlab);
  N.sw = m.alloc<T>(N.sw_stride * pl.subs.size());
  N.sw2 = m.alloc<T>(N.sw_stride * pl.subs.size());
  N.vI = m.alloc<T>(pl.tot_I * nr);
  N.vR = m.alloc<T>(pl.tot_r * nr);
  N.q = m.alloc<T>(pl.tot_g * nr);
  N.gv = m.alloc<T>(pl.tot_g * nr);
  N.v2 = m.alloc<T>(pl.tot_g * nr);
  N.mu = m.alloc<T>(pl.tot_a * nr);
  N.lu = m.alloc<T>(pl.tot_a * nr);
  N.bci = m.alloc<T>(pl.tot_c * nr);
  (void)s;
}

// Builds every descriptor batch of the plan (static for the precond's life).
void build_batches(bddcso_precond* pc, hipStream_t s) {
  const Plan& pl = *pc->plan;
  DevMem& m = pc->mem;
  const int ns = (int)pl.subs.size();
  const int64_t tmp_stride = (int64_t)pl.max_block * std::max(pl.max_zcols, 1);
  for (int setR = 0; setR < 2; ++setR) {
    int nbmax = setR ? pl.max_nbR : pl.max_nbI;
    auto& vec = setR ? pc->swR : pc->swI;
    for (int k = 0; k < nbmax; ++k) {
      std::vector<SweepDesc> d;
      for (int sidx = 0; sidx < ns; ++sidx) {
        const SubDev& S = pl.subs[sidx];
        int nb = setR ? S.nbR : S.nbI;
        if (k >= nb) continue;
        const BlockDev& B = pl.blocks[(setR ? S.bR_off : S.bI_off) + k];
        d.push_back({B.G_off, B.size, B.size, B.ld});
      }
      check_sweeps(d, pl.pool_G, ns, setR ? "K_rr blocks" : "K_II blocks");
      vec.push_back(make_sweep_buckets(m, d, s, pc->opt.sweep_reg_rows));
    }
  }
  pc->zsplit = ns / 2;
  for (int k = 0; k < pl.max_nbR; ++k) for (int h = 0; h < 2; ++h) {
    std::vector<GemmDesc> f, b;
    for (int sidx = h ? pc->zsplit : 0; sidx < (h ? ns : pc->zsplit); ++sidx) {
      const SubDev& S = pl.subs[sidx];
      int ncols = S.n_a + S.n_v;
      if (k >= S.nbR || ncols == 0) continue;
      const BlockDev& B = pl.blocks[S.bR_off + k];
      // forward: only the columns the right-hand sides have reached (the
      // others are still zero), a prefix in the stored column order
      if (B.za > 0)
        f.push_back({B.G_off, sidx * tmp_stride, S.Z_off + B.start, B.size, B.za, B.size, B.ld, B.size, S.n_r});
      if (k + 1 < S.nbR) {
        const BlockDev& N = pl.blocks[S.bR_off + k + 1];
        if (B.plane_hi == N.plane_lo)
          b.push_back({B.G_off + (int64_t)B.ld * (B.size - B.last_n), sidx * tmp_stride, S.Z_off + B.start,
                       B.size, ncols, B.last_n, B.ld, B.last_n, S.n_r});
      }
    }
    check_gemms(f, pl.pool_G, tmp_stride * ns, pl.pool_Z, "forward block GEMM");
    check_gemms(b, pl.pool_G, tmp_stride * ns, pl.pool_Z, "backward block GEMM");
    pc->gfwd[h].push_back(make_gemm_batch(m, f, s));
    pc->gbwd[h].push_back(make_gemm_batch(m, b, s));
  }
  {
    std::vector<SweepDesc> d;
    std::vector<GemmDesc> lam, phir;
    for (int sidx = 0; sidx < ns; ++sidx) {
      const SubDev& S = pl.subs[sidx];
      if (S.n_a > 0) {
        d.push_back({S.Sc_off, S.n_a, S.n_a, S.n_a});
        // only Lambda's vertex columns need the product (T_v packed in the
        // Lambda buffer, Lambda_v packed in the right-hand side buffer)
        if (S.n_v > 0) lam.push_back({S.Sc_off, S.T_off, S.T_off, S.n_a, S.n_v, S.n_a, S.n_a, S.n_a, S.n_a});
      }
      // every subdomain with vertices: the product writes Phi's vertex
      // columns at all selected rows (-X Lambda_v, 0 when there are no
      // averages); Lambda_v is packed in the right-hand side buffer
      if (S.n_v > 0)
        phir.push_back({S.XG_off, S.T_off, S.PhiG_off, S.n_s, S.n_v, S.n_a, S.n_s, std::max(S.n_a, 1), S.n_s});
    }
    check_sweeps(d, pl.pool_Sc, ns, "S_c");
    check_gemms(lam, pl.pool_Sc, pl.pool_T, pl.pool_T, "Lambda GEMM");
    check_gemms(phir, pl.pool_XG, pl.pool_T, pl.pool_PhiG, "Phi GEMM");
    pc->swSc = make_sweep_buckets(m, d, s, pc->opt.sweep_reg_rows);
    pc->gLam = make_gemm_batch(m, lam, s);
    pc->gSel = make_gemm_batch(m, phir, s);
  }
  // G entries streamed by one block solve of each set
  for (const SubDev& S : pl.subs)
    for (int setR = 0; setR < 2; ++setR) {
      const int nb = setR ? S.nbR : S.nbI;
      for (int k = 0; k < nb; ++k) {
        const BlockDev& B = pl.blocks[(setR ? S.bR_off : S.bI_off) + k];
        int& mbs = setR ? pc->max_block_R : pc->max_block_I;
        mbs = std::max(mbs, B.size);
        // lower triangle (forward) and the band of rows >= size - last_n (backward)
        const double lb = B.last_n, base = B.size - B.last_n;
        double e = (double)B.size * (B.size + 1) / 2 + (B.cb_off >= 0 ? lb * base + lb * (lb + 1) / 2 : 0.0);
        (setR ? pc->gR_entries : pc->gI_entries) += e;
      }
    }
  // colours
  for (auto& cs : pl.color_subs) {
    pc->color_dev.push_back(m.upload(cs, s));
    pc->color_n.push_back((int)cs.size());
  }
  // fronts per level
  const int nlev = (int)pl.level_fronts.size();
  pc->slot_dev.assign(nlev, {});
  pc->slot_n.assign(nlev, {});
  pc->slot_maxn.assign(nlev, {});
  int maxfn = 0;
  for (int L = 0; L < nlev; ++L) {
    std::vector<SweepDesc> d;
    int mn = 0, mp = 0, mb = 0;
    for (int t : pl.level_fronts[L]) {
      const FrontDev& F = pl.fronts[t];
      d.push_back({F.off, F.n, F.p, F.n});
      mn = std::max(mn, F.n);
      mp = std::max(mp, F.p);
      mb = std::max(mb, F.n - F.p);
      maxfn = std::max(maxfn, F.n);
    }
    check_sweeps(d, pl.front_pool, (int64_t)d.size(), "coarse fronts");
    pc->swFront.push_back(make_sweep_buckets(m, d, s, pc->opt.sweep_reg_rows));
    pc->level_dev.push_back(m.upload(pl.level_fronts[L], s));
    pc->level_n.push_back((int)pl.level_fronts[L].size());
    pc->level_maxn.push_back(mn);
    pc->level_maxp.push_back(mp);
    pc->level_maxb.push_back(mb);
    for (auto& ch : pl.level_slot_children[L]) {
      int cm = 0;
      for (int c : ch) cm = std::max(cm, pl.fronts[c].n - pl.fronts[c].p);
      pc->slot_dev[L].push_back(m.upload(ch, s));
      pc->slot_n[L].push_back((int)ch.size());
      pc->slot_maxn[L].push_back(cm);
    }
  }
  {
    std::vector<int32_t> all;
    for (int L = 0; L < nlev; ++L) all.insert(all.end(), pl.level_fronts[L].begin(), pl.level_fronts[L].end());
    pc->all_n = (int)all.size();
    pc->all_maxn = maxfn;
    if (!all.empty()) pc->all_fronts = m.upload(all, s);
  }
  int maxlev = 1;
  for (int L = 0; L < nlev; ++L) maxlev = std::max(maxlev, pc->level_n[L]);
  pc->fsw_stride = std::max<int64_t>(2 * ((int64_t)std::max(maxfn, 1) * kSweepNB + kSweepNB * kSweepNB),
                                     (int64_t)std::max(maxfn, 1) * kSlab);
  pc->fsw = m.alloc<double>(pc->fsw_stride * maxlev);
}

// Reference and executed work of the profiled kernel classes (host only,
// from the plan): see the bddcso_precond fields.
double band_width(int dim, int mx, int my) { return dim == 3 ? (double)mx * my + mx + 1 : (double)mx + 1; }
double band_nnz(double n, double b) { return n > b ? n * (b + 1) - b * (b + 1) / 2 : n * (n + 1) / 2; }

void precompute_refs(bddcso_precond* pc) {
  const Plan& pl = *pc->plan;
  const Classification& c = pc->prob->c;
  const double es = pc->precision == 1 ? 4.0 : 8.0;
  const int ns = (int)pl.subs.size();
  pc->refI_potrf.assign(pl.max_nbI, 0.0);
  pc->refR_potrf.assign(pl.max_nbR, 0.0);
  for (int st = 0; st < 2; ++st) {
    const int nb = st ? pl.max_nbR : pl.max_nbI;
    pc->sc_flops[st].assign(nb, 0.0);
    pc->sc_bytes[st].assign(nb, 0.0);
  }
  for (int h = 0; h < 2; ++h)
    for (int f = 0; f < 2; ++f) {
      pc->cm_flops[h][f].assign(pl.max_nbR, 0.0);
      pc->cm_bytes[h][f].assign(pl.max_nbR, 0.0);
    }
  for (int sidx = 0; sidx < ns; ++sidx) {
    const SubDev& S = pl.subs[sidx];
    int mI[2];
    for (int a = 0; a < 2; ++a) mI[a] = S.m[a] - (S.elo[a] > 0 ? 1 : 0) - (S.ehi[a] < (int)c.ne[a] ? 1 : 0);
    const double bI = band_width(c.dim, mI[0], mI[1]), bR = band_width(c.dim, S.m[0], S.m[1]);
    pc->refI_nnz += band_nnz(S.n_I, bI);
    pc->refR_nnz += band_nnz(S.n_r, bR);
    const int ncols = S.n_a + S.n_v;
    pc->ref_basis_flops += 4.0 * band_nnz(S.n_r, bR) * ncols;
    for (int st = 0; st < 2; ++st) {
      const int nb = st ? S.nbR : S.nbI;
      const BlockDev* blk = pl.blocks.data() + (st ? S.bR_off : S.bI_off);
      const double bw = st ? bR : bI;
      for (int k = 0; k < nb; ++k) {
        const BlockDev& B = blk[k];
        (st ? pc->refR_potrf : pc->refI_potrf)[k] += (double)B.size * bw * bw;
        if (k > 0 && B.cf_off >= 0) {
          const double lp = blk[k - 1].last_n, fn = B.first_n;
          // G_{k-1}'s last-plane block read, S_k's lower triangle written; the
          // coupling and in-plane stencil tables (9 and 5 ranks and coefficients per row)
          pc->sc_bytes[st][k] += es * (lp * lp + fn * (fn + 1) / 2) + 12.0 * 14.0 * fn;
          pc->sc_flops[st][k] += 18.0 * (lp * fn + fn * (fn + 1) / 2);
        }
        if (!st || ncols == 0) continue;
        const int h = sidx < pc->zsplit ? 0 : 1;
        if (B.za > 0) {  // forward coupling product over the reached columns
          const bool cpl = k > 0 && B.cf_off >= 0;
          pc->cm_bytes[h][1][k] += es * 2.0 * B.size * B.za +
                                   (cpl ? es * blk[k - 1].last_n * B.za + 12.0 * 9.0 * B.first_n : 0.0);
          pc->cm_flops[h][1][k] += cpl ? 18.0 * B.first_n * B.za : 0.0;
        }
        if (k + 1 < nb && B.cb_off >= 0) {  // backward coupling product
          pc->cm_bytes[h][0][k] += es * ((double)blk[k + 1].first_n * ncols + (double)B.last_n * ncols) +
                                   12.0 * 9.0 * B.last_n;
          pc->cm_flops[h][0][k] += 18.0 * B.last_n * ncols;
        }
      }
    }
  }
}

// Reference (Cholesky-equivalent) flops of the sweeps of one batch, booked
// under the class its launches time: the register path (class 5) or the
// slab path (pivot blocks and panels class 4, trailing updates class 1).
// A matrix of n rows with p pivots: p^3/3 to factor the pivots,
// (n - p) p^2 for the border, (n - p)^2 p for the Schur update.
void ref_sweep_batch(bddcso_precond* pc, const Batch& b) {
  if (!pc->P_()) return;
  double fac = 0, upd = 0;
  for (const SweepDesc& d : b.hs) {
    const double n = d.n, p = d.p, m = n - p;
    fac += p * p * p / 3.0 + m * p * p;
    upd += m * m * p;
  }
  if (b.maxn <= pc->opt.sweep_reg_rows) pc->prof.ref(5, fac + upd, 0.0);
  else {
    pc->prof.ref(4, fac, 0.0);
    pc->prof.ref(1, upd, 0.0);
  }
}

// executed = reference flops of a batch of GEMM products (2 m n k each)
void ref_gemm_batch(bddcso_precond* pc, const Batch& b) {
  if (!pc->P_()) return;
  double f = 0;
  for (const GemmDesc& d : b.hg) f += 2.0 * d.m * d.n * d.k;
  pc->prof.ref(3, f, 0.0);
}

template <typename T>
void numeric_setup(bddcso_precond* pc, hipStream_t s, bool leave_coarse) {
  // a previous setup's coarse factorization may still read the local coarse
  // matrices this one rewrites
  if (pc->coarse_pending) HIPCHK(hipStreamWaitEvent(s, pc->ev_coarse, 0));
  const Plan& pl = *pc->plan;
  Numeric<T>& N = num<T>(pc);
  const PlanDev& P = pc->P;
  const Geo& g = pc->geo;
  const double* rho = pc->rho;
  launch_fill_i32(pc->status, 1, 0, s);
  // on a second stream: the plane-coupling coefficients (first needed by the
  // second plane's Schur update).  Nothing else runs beside the K_rr chain:
  // its sweeps are latency-bound but fill every compute unit and its Schur
  // updates are bandwidth-bound, so streaming work beside it (or beside the
  // coarse factorization later) slows it about as much as it takes alone.
  HIPCHK(hipEventRecord(pc->ev_fork, s));
  HIPCHK(hipStreamWaitEvent(pc->s2, pc->ev_fork, 0));
  launch_coupling_coefs(P, g, rho, pc->cpl_coef, pc->ipl_coef, pc->s2);
  // the vertex stencils depend on rho only; the second stream has slack here
  launch_vertex_stencil(P, g, rho, pc->vcoef, pc->vcode, pc->max_nv, pc->s2);
  HIPCHK(hipEventRecord(pc->ev_cpl, pc->s2));
  launch_alpha(P, pc->prob->c.n_ss, rho, pc->opt.weighting, pc->alpha, s);
  launch_kig_fill(P, g, rho, s);
  launch_delta(P, pc->alpha, pc->delta, s);
  // local block-tridiagonal factors of K_II and K_rr (lower triangles written whole)
  Kern<T>::block_assemble(P, g, rho, 0, N.G, pl.max_nbI, s);
  Kern<T>::block_assemble(P, g, rho, 1, N.G, pl.max_nbR, s);
  auto factor_chain = [&](int setR, hipStream_t ss) {
    T* sws = setR ? N.sw : N.sw2;
    auto& sw = setR ? pc->swR : pc->swI;
    for (int k = 0; k < (int)sw.size(); ++k) {
      if (k == 1 && setR) HIPCHK(hipStreamWaitEvent(ss, pc->ev_cpl, 0));  // the coupling coefficients
      if (k > 0) {
        if (pc->P_()) pc->prof.begin(6, ss);
        Kern<T>::schur_couple(P, setR, k, N.G, ss);
        if (pc->P_()) {
          pc->prof.end(6, pc->sc_flops[setR][k], pc->sc_bytes[setR][k], ss);
          pc->prof.ref(6, pc->sc_flops[setR][k], pc->sc_bytes[setR][k]);
        }
      }
      int maxn = 0;
      for (const Batch& b : sw[k]) {
        Kern<T>::sweep((SweepDesc*)b.desc, b.hs.data(), b.n, b.maxn, b.maxp, N.G, sws, N.sw_stride, pc->status,
                       setR ? 2 : 1, ss, pc->P_(), nullptr, pc->opt.sweep_reg_rows, pc->opt.slab_lookahead,
                       pc->opt.update_tile, pc->opt.slab_width);
        maxn = std::max(maxn, b.maxn);
      }
      if (pc->P_()) {  // banded Cholesky of block k of every subdomain
        const double f = (setR ? pc->refR_potrf : pc->refI_potrf)[k];
        if (maxn <= pc->opt.sweep_reg_rows) pc->prof.ref(5, f, 0.0);
        else pc->prof.ref(4, f, 0.0);
      }
    }
  };
  factor_chain(1, s);
  HIPCHK(hipStreamWaitEvent(s, pc->ev_cpl, 0));  // also when K_rr has a single block
  // [X | Y'] = K_rr^{-1} [C_r^T | -K_rv]
  if (sizeof(T) == 8) launch_fill_f64((double*)N.Z, pl.pool_Z, 0.0, s);
  else launch_fill_f32((float*)N.Z, pl.pool_Z, 0.0f, s);
  Kern<T>::rhs_fill(P, g, rho, N.Z, s);
  // Two halves of the subdomains, each a chain of coupling products (HBM)
  // and block GEMMs (MFMA) on its own stream.  The second half starts one
  // coupling product later, so one half's GEMMs run beside the other's
  // coupling products.
  const int nk = (int)pc->gfwd[0].size();
  auto zchain = [&](int h, hipStream_t ss) {
    const int sub0 = h ? pc->zsplit : 0, nsub = h ? (int)pl.subs.size() - pc->zsplit : pc->zsplit;
    auto couple = [&](int k, int fwd) {
      if (pc->P_()) pc->prof.begin(7, ss);
      Kern<T>::couple_multi(P, g, rho, k, fwd, pl.max_zcols, N.Z, N.tmp, N.tmp_stride, ss, sub0, nsub);
      if (pc->P_()) {
        pc->prof.end(7, pc->cm_flops[h][fwd][k], pc->cm_bytes[h][fwd][k], ss);
        pc->prof.ref(7, pc->cm_flops[h][fwd][k], pc->cm_bytes[h][fwd][k]);
      }
    };
    for (int k = 0; k < nk; ++k) {
      couple(k, 1);
      if (k == 0 && h == 0) {
        HIPCHK(hipEventRecord(pc->ev_zf, ss));
        HIPCHK(hipStreamWaitEvent(pc->s2, pc->ev_zf, 0));
      }
      const Batch& b = pc->gfwd[h][k];
      Kern<T>::gemm((GemmDesc*)b.desc, b.hg.data(), b.n, b.maxm, b.maxn, N.G, 0, N.tmp, 0, N.Z, (T)-1, (T)0, ss,
                    pc->P_());
    }
    for (int k = nk - 2; k >= 0; --k) {
      couple(k, 0);
      const Batch& b = pc->gbwd[h][k];
      Kern<T>::gemm((GemmDesc*)b.desc, b.hg.data(), b.n, b.maxm, b.maxn, N.G, 0, N.tmp, 0, N.Z, (T)1, (T)1, ss,
                    pc->P_());
    }
  };
  zchain(0, s);
  if (nk == 0) {
    HIPCHK(hipEventRecord(pc->ev_zf, s));
    HIPCHK(hipStreamWaitEvent(pc->s2, pc->ev_zf, 0));
  }
  zchain(1, pc->s2);
  HIPCHK(hipEventRecord(pc->ev_zj, pc->s2));
  HIPCHK(hipStreamWaitEvent(s, pc->ev_zj, 0));
  // the banded forward and backward solves the block GEMMs stand for
  if (pc->P_()) pc->prof.ref(3, pc->ref_basis_flops, 0.0);
  // constraint Schur complement and the coarse basis
  // X at the selected rows, S_c, the vertex columns of Lambda's right-hand
  // sides (packed in Lambda's buffer until the product), and Y' in Phi's
  // vertex columns and at the Gamma entries
  Kern<T>::object_means(P, N.Z, N.XG, N.Sc, N.Lam, N.PhiG, N.YG, s);
  for (const Batch& b : pc->swSc) {
    Kern<T>::sweep((SweepDesc*)b.desc, b.hs.data(), b.n, b.maxn, b.maxp, N.Sc, N.sw, N.sw_stride, pc->status, 3, s,
                   pc->P_(), nullptr, pc->opt.sweep_reg_rows, pc->opt.slab_lookahead, pc->opt.update_tile, pc->opt.slab_width);
    ref_sweep_batch(pc, b);
  }
  Kern<T>::gemm((GemmDesc*)pc->gLam.desc, pc->gLam.hg.data(), pc->gLam.n, pc->gLam.maxm, pc->gLam.maxn, N.Sc, 0,
                N.Lam, 0, N.Tm, (T)-1, (T)0, s, pc->P_());
  ref_gemm_batch(pc, pc->gLam);
  Kern<T>::lam_assemble(P, N.Sc, N.Tm, N.Lam, s);
  Kern<T>::float_setup(P, N.Sc, N.Lam, pc->feps, pc->fdelta, s);
  // Phi = Y' - X Lambda, only at the selected rows (Gamma and the vertices'
  // stencils) and only in the vertex columns
  Kern<T>::gemm((GemmDesc*)pc->gSel.desc, pc->gSel.hg.data(), pc->gSel.n, pc->gSel.maxm, pc->gSel.maxn, N.XG, 0,
                N.Tm, 0, N.PhiG, (T)-1, (T)1, s, pc->P_());  // added to Y' (and the unit rows) already there
  ref_gemm_batch(pc, pc->gSel);
  Kern<T>::kc_identity(P, g, rho, N.PhiG, N.Lam, N.Kc, pc->vcoef, pc->vcode, pc->max_nv, s);
  // The interior (Dirichlet) factors are needed only when the preconditioner
  // is applied, so they are built on a third stream while the coarse
  // factorization runs (its upper levels occupy few compute units); the
  // caller's stream waits for them at the end.
  // Scatter plans: the fronts' lower triangles are zeroed first (they are
  // summed into); alone on the GPU this streaming pass is short, while
  // beside the factor chains it slows their latency-bound sweeps.
  if (!pl.front_gather) launch_front_zero_lower(P, pc->all_fronts, pc->all_n, pc->all_maxn, pc->fpool, s);
  HIPCHK(hipEventRecord(pc->ev_fork_i, s));
  HIPCHK(hipStreamWaitEvent(pc->s3, pc->ev_fork_i, 0));
  factor_chain(0, pc->s3);
  HIPCHK(hipEventRecord(pc->ev_join_i, pc->s3));
  // coarse: assemble into the fronts and factor level by level (FP64), on
  // the fourth stream.  Fronts with at most two sources gather them (each
  // entry written once); otherwise the local coarse matrices are added by
  // colour classes and the children's update blocks in slot order.
  // (on the caller's stream itself when the setup must end with it, as in a
  // captured graph)
  hipStream_t sc = leave_coarse ? pc->s4 : s;
  if (leave_coarse) {
    HIPCHK(hipEventRecord(pc->ev_kc, s));
    HIPCHK(hipStreamWaitEvent(sc, pc->ev_kc, 0));
  }
  if (!pl.front_gather)
    for (size_t c = 0; c < pc->color_dev.size(); ++c)
      Kern<T>::kc_to_front(P, pc->color_dev[c], pc->color_n[c], N.Kc, pc->fpool, sc);
  for (size_t L = 0; L < pc->swFront.size(); ++L) {
    if (pl.front_gather)
      Kern<T>::front_gather(P, pc->level_dev[L], pc->level_n[L], pc->level_maxn[L], N.Kc, pc->fpool, sc);
    else
      for (size_t j = 0; j < pc->slot_dev[L].size(); ++j)
        launch_front_child_scatter(P, pc->slot_dev[L][j], pc->slot_n[L][j], pc->slot_maxn[L][j], pc->fpool, sc);
    const SweepAux aux{pc->s2, pc->ev_la, pc->ev_lb, pc->ev_lc};
    for (const Batch& b : pc->swFront[L]) {
      Kern<double>::sweep((SweepDesc*)b.desc, b.hs.data(), b.n, b.maxn, b.maxp, pc->fpool, pc->fsw,
                          pc->fsw_stride, pc->status, 4, sc, pc->P_(), &aux, pc->opt.sweep_reg_rows,
                          pc->opt.slab_lookahead, pc->opt.update_tile, pc->opt.slab_width);
      ref_sweep_batch(pc, b);
    }
  }
  if (leave_coarse) HIPCHK(hipEventRecord(pc->ev_coarse, sc));
  HIPCHK(hipStreamWaitEvent(s, pc->ev_join_i, 0));  // the interior factors
  pc->coarse_pending = leave_coarse;
}

// The coarse solve of the local right-hand sides bci (FP64 or FP32: one is
// null), assembled into the fronts' vectors as the forward solve starts.
void coarse_solve(bddcso_precond* pc, const double* bci_d, const float* bci_f, int nrhs, hipStream_t s) {
  const PlanDev& P = pc->P;
  const Plan& pl = *pc->plan;
  const int nlev = (int)pc->level_dev.size();
  const int64_t stride = pl.front_vec;
  launch_front_vec_init(P, pc->all_fronts, pc->all_n, pc->all_maxn, bci_d, bci_f, pc->fvec, stride, nrhs, s);
  double* part = nrhs < pc->P.mr_min ? pc->fpart : nullptr;
  const bool pull = part && P.front_pull;  // the chunked forward step gathers the children's values itself
  for (int L = 0; L < nlev; ++L) {
    if (!pull)
      for (size_t j = 0; j < pc->slot_dev[L].size(); ++j)
        launch_front_vec_scatter(P, pc->slot_dev[L][j], pc->slot_n[L][j], pc->slot_maxn[L][j], pc->fvec, stride,
                                 nrhs, s);
    launch_front_fwd(P, pc->level_dev[L], pc->level_n[L], pc->level_maxn[L], pc->level_maxp[L], pc->fpool,
                     pc->fvec, pc->xh, stride, nrhs, s, part, pull);
  }
  for (int L = nlev - 1; L >= 0; --L)
    launch_front_bwd(P, pc->level_dev[L], pc->level_n[L], pc->level_maxp[L], pc->level_maxb[L], pc->fpool, pc->xh,
                     stride, pc->uc, nrhs, s);
}

template <typename T>
void apply_B(bddcso_precond* pc, const double* r, double* z, int nrhs, hipStream_t s) {
  const Plan& pl = *pc->plan;
  Numeric<T>& N = num<T>(pc);
  const PlanDev& P = pc->P;
  const Geo& g = pc->geo;
  const double* rho = pc->rho;
  // 1-2: Dirichlet solves and (I - P)^T on Gamma
  Kern<T>::gather_I(P, g, r, N.vI, nrhs, s);
  Kern<T>::block_solve(P, g, rho, 0, N.G, N.vI, nrhs, s, pc->P_(), pc->gI_entries, (double)pl.tot_I,
                       pc->max_block_I);
  if (pc->P_()) pc->prof.ref(2, 4.0 * pc->refI_nnz * nrhs, sizeof(T) * (2.0 * pc->refI_nnz + 2.0 * pl.tot_I * nrhs));
  Kern<T>::gamma_kgi(P, g, rho, N.vI, N.q, nrhs, s);
  // 3: E^T
  Kern<T>::gamma_t(P, g, r, N.q, pc->delta, N.gv, nrhs, s);
  // 4: constrained Neumann solves, and 5-6: the coarse problem, which needs
  // only E^T's output and runs on a second stream beside them (the Neumann
  // solves are bandwidth-bound, the coarse solve a chain of small
  // latency-bound kernels).  The Neumann solves are enqueued first so the
  // GPU starts them while the host is still launching the coarse chain.
  HIPCHK(hipEventRecord(pc->ev_cfork, s));
  if (sizeof(T) == 8) launch_fill_f64((double*)N.vR, pl.tot_r * nrhs, 0.0, s);
  else launch_fill_f32((float*)N.vR, pl.tot_r * nrhs, 0.0f, s);
  Kern<T>::neumann_rhs(P, N.gv, N.vR, nrhs, s);
  Kern<T>::block_solve(P, g, rho, 1, N.G, N.vR, nrhs, s, pc->P_(), pc->gR_entries, (double)pl.tot_r,
                       pc->max_block_R);
  if (pc->P_()) pc->prof.ref(2, 4.0 * pc->refR_nnz * nrhs, sizeof(T) * (2.0 * pc->refR_nnz + 2.0 * pl.tot_r * nrhs));
  Kern<T>::mu(P, N.vR, N.Sc, N.mu, nrhs, s);
  Kern<T>::float_mu(P, N.gv, N.mu, pc->feps, pc->fdelta, pc->fc, nrhs, s);
  HIPCHK(hipStreamWaitEvent(pc->s2, pc->ev_cfork, 0));
  // X_Gamma^T g per average goes through lu, which lam_uc below refills
  // and only v2 (after the join) reads
  Kern<T>::coarse_rhs_local(P, N.XG, N.PhiG, N.Lam, pc->feps, N.gv, N.lu, N.bci, nrhs, pc->s2);
  if (pc->coarse_pending) HIPCHK(hipStreamWaitEvent(pc->s2, pc->ev_coarse, 0));
  if (sizeof(T) == 8) coarse_solve(pc, (const double*)N.bci, nullptr, nrhs, pc->s2);
  else coarse_solve(pc, nullptr, (const float*)N.bci, nrhs, pc->s2);
  Kern<T>::lam_uc(P, N.Lam, pc->uc, N.lu, nrhs, pc->s2);
  HIPCHK(hipEventRecord(pc->ev_cjoin, pc->s2));
  HIPCHK(hipStreamWaitEvent(s, pc->ev_cjoin, 0));
  // 7-8: v2 on Gamma and E
  Kern<T>::v2(P, N.vR, N.XG, N.mu, N.lu, N.YG, pc->uc, N.v2, nrhs, s);
  Kern<T>::float_v2(P, pc->uc, pc->feps, pc->fc, N.v2, nrhs, s);
  if (sizeof(T) == 8) launch_gamma_w(P, g, (const double*)N.v2, nullptr, pc->delta, z, nrhs, s);
  else launch_gamma_w(P, g, nullptr, (const float*)N.v2, pc->delta, z, nrhs, s);
  // 9-10: harmonic extension into the interiors
  Kern<T>::interior_rhs(P, g, rho, r, z, N.vI, nrhs, s);
  Kern<T>::block_solve(P, g, rho, 0, N.G, N.vI, nrhs, s, pc->P_(), pc->gI_entries, (double)pl.tot_I,
                       pc->max_block_I);
  if (pc->P_()) pc->prof.ref(2, 4.0 * pc->refI_nnz * nrhs, sizeof(T) * (2.0 * pc->refI_nnz + 2.0 * pl.tot_I * nrhs));
  Kern<T>::scatter_I(P, g, N.vI, z, nrhs, s);
}

// Captures the work body enqueues on the preconditioner's capture stream
// (and on the streams it forks to) into an instantiated graph.
template <typename F>
hipGraphExec_t capture_graph(bddcso_precond* pc, F&& body) {
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  HIPCHK(hipStreamBeginCapture(pc->sg, hipStreamCaptureModeThreadLocal));
  try {
    body(pc->sg);
  } catch (...) {
    if (hipStreamEndCapture(pc->sg, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    throw;
  }
  HIPCHK(hipStreamEndCapture(pc->sg, &g));
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) throw HipFail{e, "hipGraphInstantiate"};
  return ex;
}

void apply_B_any(bddcso_precond* pc, const double* r, double* z, int nrhs, hipStream_t s) {
  if (pc->precision == 1) apply_B<float>(pc, r, z, nrhs, s);
  else apply_B<double>(pc, r, z, nrhs, s);
}

std::shared_ptr<Plan> get_plan(bddcso_problem* p, const bddcso_options& o, Error& err) {
  int bt = o.block_target > 0 ? o.block_target : 192;
  auto key = std::make_tuple(o.primal_mask, bt, o.coarse_solver);
  auto it = p->plans.find(key);
  if (it != p->plans.end()) return it->second;
  auto pl = std::make_shared<Plan>();
  if (!build_plan(p->c, o.primal_mask, bt, o.coarse_solver, *pl, err)) return nullptr;
  p->plans[key] = pl;
  return pl;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

}  // namespace

extern "C" void bddcso_precond_destroy(bddcso_precond* pc);

namespace {

// Lays out (allocates, carves or counts, by pc->mem.mode) every device
// buffer of the preconditioner and uploads the plan's tables.
void layout(bddcso_precond* pc, hipStream_t s) {
  const bddcso_problem* p = pc->prob;
  const bddcso_options& o = pc->opt;
  const Classification& c = p->c;
  const Plan& pl = *pc->plan;
  DevMem& m = pc->mem;
  PlanDev& P = pc->P;
  P.subs = m.upload(pl.subs, s);
  P.blocks = m.upload(pl.blocks, s);
  P.loc_I = m.upload(pl.loc_I, s);
  P.loc_r = m.upload(pl.loc_r, s);
  P.loc_g = m.upload(pl.loc_g, s);
  P.I_loc = m.upload(pl.I_loc, s);
  P.z_col = m.upload(pl.z_col, s);
  P.kig_ptr = m.upload(pl.kig_ptr, s);
  P.kig_t = m.upload(pl.kig_t, s);
  P.kig_own = m.upload(pl.kig_own, s);
  P.kig_sub = m.upload(pl.kig_sub, s);
  P.n_kig = (int64_t)pl.kig_t.size();
  P.kig_col = m.alloc<int32_t>((int64_t)pl.kig_t.size());
  P.kig_val = m.alloc<double>((int64_t)pl.kig_t.size());
  P.kgi_ptr = m.upload(pl.kgi_ptr, s);
  P.kgi_t = m.upload(pl.kgi_t, s);
  P.kgi_own = m.upload(pl.kgi_own, s);
  P.n_kgi = (int64_t)pl.kgi_t.size();
  P.kgi_col = m.alloc<int32_t>((int64_t)pl.kgi_t.size());
  P.kgi_val = m.alloc<double>((int64_t)pl.kgi_t.size());
  P.r_loc = m.upload(pl.r_loc, s);
  P.g_loc = m.upload(pl.g_loc, s);
  P.g_gam = m.upload(pl.g_gam, s);
  P.g_r = m.upload(pl.g_r, s);
  P.loc_sel = m.upload(pl.loc_sel, s);
  P.sel_r = m.upload(pl.sel_r, s);
  P.g_v = m.upload(pl.g_v, s);
  P.g_sub = m.upload(pl.g_sub, s);
  P.v_loc = m.upload(pl.v_loc, s);
  P.v_c = m.upload(pl.v_c, s);
  P.a_ptr = m.upload(pl.a_ptr, s);
  P.a_r = m.upload(pl.a_r, s);
  P.a_g = m.upload(pl.a_g, s);
  P.a_c = m.upload(pl.a_c, s);
  P.c_glob = m.upload(pl.c_glob, s);
  P.c_kind = m.upload(pl.c_kind, s);
  P.gam_eptr = m.upload(pl.gam_eptr, s);
  P.gam_ent = m.upload(pl.gam_ent, s);
  P.gam_node = m.upload(c.gam_node, s);
  P.gam_kptr = m.upload(c.gam_kptr, s);
  P.gam_key = m.upload(c.gam_key, s);
  P.ss_parent = m.upload(c.ss_parent, s);
  P.ss_eptr = m.upload(c.ss_eptr, s);
  P.ss_elem = m.upload(c.ss_elem, s);
  P.crs_eptr = m.upload(pl.crs_eptr, s);
  P.crs_ent = m.upload(pl.crs_ent, s);
  P.fronts = m.upload(pl.fronts, s);
  P.front_idx = m.upload(pl.front_idx, s);
  P.front_pmap = m.upload(pl.front_pmap, s);
  {
    // per front vector entry and scatter slot, the child border value the
    // entry receives (the single-RHS coarse forward step pulls them in slot
    // order instead of running the scatter launches), -1 for none
    int ns = 0;
    for (const auto& lv : pl.level_slot_children) ns = std::max(ns, (int)lv.size());
    std::vector<int32_t> pull;
    if (ns > 0 && pl.front_vec > 0) {
      if (pl.front_vec > INT32_MAX) throw PlanFail{"coarse front vectors above 2^31 entries"};
      pull.assign((size_t)pl.front_vec * ns, -1);
      for (const auto& lv : pl.level_slot_children)
        for (size_t j = 0; j < lv.size(); ++j)
          for (int c : lv[j]) {
            const FrontDev& C = pl.fronts[c];
            const FrontDev& F = pl.fronts[C.parent];
            for (int k = 0; k < C.n - C.p; ++k)
              pull[(size_t)(F.voff + pl.front_pmap[C.pmap_off + k]) * ns + j] = (int32_t)(C.voff + C.p + k);
          }
    }
    P.n_slot = pull.empty() ? 0 : ns;
    P.front_pull = pull.empty() ? nullptr : m.upload(pull, s);
  }
  P.front_imap = pl.front_imap.empty() ? nullptr : m.upload(pl.front_imap, s);
  P.sub_fmap = m.upload(pl.sub_fmap, s);
  P.cpl_rank = m.upload(pl.cpl_rank, s);
  P.cpl_sub = m.upload(pl.cpl_sub, s);
  P.cpl_loc = m.upload(pl.cpl_loc, s);
  P.cpl_dir = m.upload(pl.cpl_dir, s);
  P.n_cpl = (int64_t)pl.cpl_sub.size();
  pc->cpl_coef = m.alloc<double>(P.n_cpl * 9);
  P.cpl_coef = pc->cpl_coef;
  P.ipl_rank = m.upload(pl.ipl_rank, s);
  pc->ipl_coef = m.alloc<double>(P.n_cpl * 5);
  P.ipl_coef = pc->ipl_coef;
  std::vector<double> kh(p->khat, p->khat + 64);
  pc->khat = m.upload(kh, s);
  P.khat = pc->khat;
  if (m.mode != DevMem::COUNT) HIPCHK(hipStreamSynchronize(s));
  P.n_sub = c.n_sub;
  P.tot_I = pl.tot_I;
  P.tot_r = pl.tot_r;
  P.tot_g = pl.tot_g;
  P.tot_c = pl.tot_c;
  P.tot_a = pl.tot_a;
  P.n_gam = (int64_t)c.gam_node.size();
  P.n_coarse = pl.n_coarse;
  P.max_block = pl.max_block;
  P.max_na = pl.max_na;
  P.max_nc = pl.max_nc;
  P.max_ng = pl.max_ng;
  P.max_ns = pl.max_ns;
  P.max_nloc = pl.max_nloc;
  P.max_nr = pl.max_nr;
  int max_nI = 0, max_plane = 0;
  for (auto& S : pl.subs) max_nI = std::max(max_nI, S.n_I);
  for (auto& B : pl.blocks) max_plane = std::max(max_plane, std::max(B.first_n, B.last_n));
  P.max_nI = max_nI;
  P.max_zcols = pl.max_zcols;
  P.max_plane = max_plane;
  P.max_nv = 0;
  P.max_nar = 0;
  P.n_pinned = 0;
  for (auto& S : pl.subs) {
    P.max_nv = std::max(P.max_nv, S.n_v);
    P.max_nar = std::max(P.max_nar, pl.a_ptr[S.a_off + S.n_a] - pl.a_ptr[S.a_off]);
    if (S.pin >= 0) ++P.n_pinned;
  }
  P.mr_min = o.mr_min_rhs;
  if (max_lds_bytes(P, o.precision == 1 ? 4 : 8, o.max_nrhs) > 160 * 1024)
    throw PlanFail{"a subdomain plane or block is too large for the LDS staging of the local kernels"};

  pc->rho = m.alloc<double>(c.n_elem);
  for (auto& S : pl.subs) pc->max_nv = std::max(pc->max_nv, S.n_v);
  pc->vcoef = m.alloc<double>(pl.tot_v * 27);
  pc->vcode = m.alloc<int32_t>(pl.tot_v * 27);
  pc->alpha = m.alloc<double>(c.n_ss);
  pc->delta = m.alloc<double>(pl.tot_g);
  pc->status = m.alloc<int32_t>(1);
  pc->fpool = m.alloc<double>(pl.front_pool);
  const int nr = pc->max_nrhs;
  pc->uc = m.alloc<double>(pl.n_coarse * nr);
  pc->fvec = m.alloc<double>(pl.front_vec * nr);
  pc->xh = m.alloc<double>(pl.front_vec * nr);
  {
    int maxp = 1;
    for (auto& F : pl.fronts) maxp = std::max(maxp, F.p);
    pc->fpart = m.alloc<double>((int64_t)front_fwd_chunks(maxp) * std::max(1, std::min(nr, o.mr_min_rhs - 1)) *
                                pl.front_vec);
  }
  if (o.precision == 1) alloc_numeric<float>(pc, s);
  else alloc_numeric<double>(pc, s);
  build_batches(pc, s);
  precompute_refs(pc);
  const int64_t n = c.n_free;
  pc->r = m.alloc<double>(n * nr);
  pc->p = m.alloc<double>(n * nr);
  pc->qv = m.alloc<double>(n * nr);
  pc->z = m.alloc<double>(n * nr);
  pc->rold = m.alloc<double>(n * nr);
  pc->dtmp = m.alloc<double>(n * nr);
  pc->partial = m.alloc<double>((int64_t)pc->dot_blocks * nr);
  pc->sc = m.alloc<double>(8 * BDDCSO_MAX_RHS);
  int maxit = std::max(o.maxit, o.fixed_iters) + 1;
  pc->hist_a = m.alloc<double>((int64_t)maxit * nr);
  pc->hist_b = m.alloc<double>((int64_t)maxit * nr);
  pc->active = m.alloc<int32_t>(nr);
  pc->iters = m.alloc<int32_t>(nr);
  pc->flags = m.alloc<int32_t>(nr);
  pc->nactive = m.alloc<int32_t>(1);
  pc->xk = m.alloc<double>(n * nr);
  pc->kdev = m.alloc<int32_t>(1);
  pc->feps = m.alloc<double>(pl.tot_a);
  pc->fdelta = m.alloc<double>(c.n_sub);
  pc->fc = m.alloc<double>((int64_t)c.n_sub * nr);
}

// Streams, events and the pinned flag of the convergence test (no device
// memory of the preconditioner's own).
void make_streams(bddcso_precond* pc) {
  HIPCHK(hipHostMalloc((void**)&pc->h_nactive, sizeof(int32_t) * 4, hipHostMallocDefault));
  HIPCHK(hipStreamCreateWithFlags(&pc->s2, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&pc->s3, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&pc->sg, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&pc->s4, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_kc, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_coarse, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_fork_i, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_cpl, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_cfork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_cjoin, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_join_i, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_join, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_la, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_lb, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_lc, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_zf, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&pc->ev_zj, hipEventDisableTiming));
}

// Validates the options, plans, and builds a preconditioner object whose
// device memory is laid out in the given mode.  COUNT: host only, *need gets
// the workspace size and nothing is kept.
bddcso_status create_precond(bddcso_problem* p, const bddcso_options* opts, DevMem::Mode mode, void* ws,
                             size_t ws_bytes, hipStream_t s, bddcso_precond** out, size_t* need) {
  *out = nullptr;
  bddcso_options o;
  if (opts) o = *opts;
  else bddcso_default_options(&o);
  if (o.max_nrhs < 1 || o.max_nrhs > BDDCSO_MAX_RHS) return set_err(BDDCSO_EINVAL, "max_nrhs out of range");
  if (o.precision != 0 && o.precision != 1) return set_err(BDDCSO_EINVAL, "precision must be 0 or 1");
  if ((o.primal_mask & 7) == 0 || o.primal_mask > 15)
    return set_err(BDDCSO_EINVAL, "primal_mask must select v, e or f (bits 1, 2, 4; bit 8 halves the faces)");
  if (o.coarse_solver != 0 && o.coarse_solver != 1) return set_err(BDDCSO_EINVAL, "coarse_solver must be 0 or 1");
  if (o.maxit < 0 || o.fixed_iters < 0) return set_err(BDDCSO_EINVAL, "maxit and fixed_iters must be >= 0");
  if (o.graph != 0 && o.graph != 1) return set_err(BDDCSO_EINVAL, "graph must be 0 or 1");
  if (o.sweep_reg_rows == 0) o.sweep_reg_rows = kRegSweepMaxRows;
  if (o.sweep_reg_rows < 16 || o.sweep_reg_rows > kRegSweepMaxRows)
    return set_err(BDDCSO_EINVAL, "sweep_reg_rows must be 0 or in 16..304");
  if (o.slab_lookahead < 0 || o.slab_lookahead > 2) return set_err(BDDCSO_EINVAL, "slab_lookahead must be 0, 1 or 2");
  if (o.mr_min_rhs == 0) o.mr_min_rhs = 4;
  if (o.mr_min_rhs < 1) return set_err(BDDCSO_EINVAL, "mr_min_rhs must be >= 0");
  if (o.update_tile == 0) o.update_tile = 64;
  if (o.update_tile != 64 && o.update_tile != 128) return set_err(BDDCSO_EINVAL, "update_tile must be 0, 64 or 128");
  if (o.slab_width != 0 && o.slab_width != 96 && o.slab_width != 192)
    return set_err(BDDCSO_EINVAL, "slab_width must be 0, 96 or 192");
  Error err;
  std::shared_ptr<Plan> plan;
  try {
    plan = get_plan(p, o, err);
  } catch (const std::bad_alloc&) {
    return set_err(BDDCSO_ENOMEM, "host allocation failed while planning");
  }
  if (!plan) return set_err(BDDCSO_EINVAL, err.msg);
  auto* pc = new (std::nothrow) bddcso_precond();
  if (!pc) return set_err(BDDCSO_ENOMEM, "host allocation failed");
  pc->prob = p;
  pc->plan = plan;
  pc->opt = o;
  pc->precision = o.precision;
  pc->max_nrhs = o.max_nrhs;
  pc->mem.mode = mode;
  pc->mem.base = (char*)ws;
  pc->mem.cap = ws_bytes;
  const Classification& c = p->c;
  Geo& g = pc->geo;
  g.dim = c.dim;
  for (int a = 0; a < 3; ++a) {
    g.ne[a] = (int)c.ne[a];
    g.nf[a] = (int)c.nf[a];
  }
  g.n_free = c.n_free;
  g.n_elem = c.n_elem;
  try {
    layout(pc, s);
    if (mode == DevMem::COUNT) {
      if (need) *need = pc->mem.used;
      bddcso_precond_destroy(pc);
      return BDDCSO_OK;
    }
    make_streams(pc);
  } catch (const PlanFail& f) {
    bddcso_precond_destroy(pc);
    return set_err(BDDCSO_EINVAL, "inconsistent plan: " + f.what);
  } catch (const WorkspaceShort& w) {
    bddcso_precond_destroy(pc);
    return set_err(BDDCSO_EINVAL, "workspace too small: " + std::to_string(w.have) + " bytes given, at least " +
                                      std::to_string(w.need) + " needed (bddcso_setup_workspace_size)");
  } catch (const HipFail& f) {
    bddcso_precond_destroy(pc);
    if (f.e == hipErrorOutOfMemory)
      return set_err(BDDCSO_ENOMEM, "device allocation failed: " + f.where);
    return set_err(BDDCSO_EHIP, f.where + ": " + hipGetErrorString(f.e));
  } catch (const std::bad_alloc&) {
    bddcso_precond_destroy(pc);
    return set_err(BDDCSO_ENOMEM, "host allocation failed");
  }
  *out = pc;
  return BDDCSO_OK;
}

}  // namespace

extern "C" {

void bddcso_default_options(bddcso_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->primal_mask = 7;
  o->weighting = 1;
  o->precision = 0;
  o->coarse_solver = 0;
  o->max_nrhs = 1;
  o->maxit = 1000;
  o->rtol = 1e-8;
  o->fixed_iters = 0;
  o->flexible = 0;
  o->block_target = 0;
  o->graph = 0;
  o->sweep_reg_rows = 0;
  o->slab_lookahead = 0;
  o->mr_min_rhs = 0;
  o->update_tile = 0;
  o->slab_width = 0;
}

const char* bddcso_last_error(void) { return g_last_error.c_str(); }

bddcso_status bddcso_problem_create(int dim, const int64_t n_el[3], const double h[3], const int32_t* elem_sub,
                                    const int32_t* elem_subsub, bddcso_problem** out) {
  if (!out) return set_err(BDDCSO_EINVAL, "null output pointer");
  *out = nullptr;
  auto* p = new (std::nothrow) bddcso_problem();
  if (!p) return set_err(BDDCSO_ENOMEM, "host allocation failed");
  Error err;
  try {
    if (!classify(dim, n_el, h, elem_sub, elem_subsub, p->c, err)) {
      delete p;
      return set_err(BDDCSO_EINVAL, err.msg);
    }
  } catch (const std::bad_alloc&) {
    delete p;
    return set_err(BDDCSO_ENOMEM, "host allocation failed during classification");
  }
  element_table(dim, p->c.h, p->khat);
  *out = p;
  return BDDCSO_OK;
}

bddcso_status bddcso_problem_info(const bddcso_problem* p, int primal_mask, int64_t* n_free, int64_t* n_gamma,
                                  int64_t* n_coarse, int* n_sub, int64_t counts[3]) {
  if (!p) return set_err(BDDCSO_EINVAL, "null problem");
  if (n_free) *n_free = p->c.n_free;
  if (n_gamma) *n_gamma = (int64_t)p->c.gam_node.size();
  if (n_sub) *n_sub = p->c.n_sub;
  int64_t cnt[3] = {0, 0, 0};
  for (int o = 0; o < p->c.n_obj(); ++o)
    if ((p->c.obj_type[o] & primal_mask) && (!(primal_mask & kHalfCodim1) || half_keep(p->c, o))) {
      int t = p->c.obj_type[o];
      cnt[t == 1 ? 0 : (t == 2 ? 1 : 2)]++;
    }
  if (n_coarse) *n_coarse = cnt[0] + cnt[1] + cnt[2];
  if (counts) {
    counts[0] = cnt[0];
    counts[1] = cnt[1];
    counts[2] = cnt[2];
  }
  return BDDCSO_OK;
}

void bddcso_precond_destroy(bddcso_precond* pc) {
  if (!pc) return;
  if (pc->s2) (void)hipStreamSynchronize(pc->s2);
  if (pc->s3) (void)hipStreamSynchronize(pc->s3);
  if (pc->sg) (void)hipStreamSynchronize(pc->sg);
  if (pc->s4) (void)hipStreamSynchronize(pc->s4);
  if (pc->g_setup) (void)hipGraphExecDestroy(pc->g_setup);
  for (auto& kv : pc->iter_graphs) {
    if (kv.second.g1) (void)hipGraphExecDestroy(kv.second.g1);
    if (kv.second.g2) (void)hipGraphExecDestroy(kv.second.g2);
  }
  pc->mem.release();
  if (pc->ev_fork) (void)hipEventDestroy(pc->ev_fork);
  if (pc->ev_join) (void)hipEventDestroy(pc->ev_join);
  if (pc->ev_la) (void)hipEventDestroy(pc->ev_la);
  if (pc->ev_lb) (void)hipEventDestroy(pc->ev_lb);
  if (pc->ev_lc) (void)hipEventDestroy(pc->ev_lc);
  if (pc->ev_zf) (void)hipEventDestroy(pc->ev_zf);
  if (pc->ev_zj) (void)hipEventDestroy(pc->ev_zj);
  if (pc->ev_cpl) (void)hipEventDestroy(pc->ev_cpl);
  if (pc->ev_cfork) (void)hipEventDestroy(pc->ev_cfork);
  if (pc->ev_cjoin) (void)hipEventDestroy(pc->ev_cjoin);
  if (pc->ev_fork_i) (void)hipEventDestroy(pc->ev_fork_i);
  if (pc->ev_join_i) (void)hipEventDestroy(pc->ev_join_i);
  if (pc->s2) (void)hipStreamDestroy(pc->s2);
  if (pc->s3) (void)hipStreamDestroy(pc->s3);
  if (pc->sg) (void)hipStreamDestroy(pc->sg);
  if (pc->s4) (void)hipStreamDestroy(pc->s4);
  if (pc->ev_kc) (void)hipEventDestroy(pc->ev_kc);
  if (pc->ev_coarse) (void)hipEventDestroy(pc->ev_coarse);
  if (pc->h_nactive) (void)hipHostFree(pc->h_nactive);
  delete pc;
}

void bddcso_problem_destroy(bddcso_problem* p) { delete p; }

bddcso_status bddcso_refactor(bddcso_precond* pc, const double* rho_dev, void* stream) {
  if (!pc || !rho_dev) return set_err(BDDCSO_EINVAL, "null argument");
  hipStream_t s = as_stream(stream);
  try {
    HIPCHK(hipMemcpyAsync(pc->rho, rho_dev, pc->geo.n_elem * sizeof(double), hipMemcpyDeviceToDevice, s));
    ++pc->generation;
    if (pc->opt.graph && !pc->P_()) {
      if (!pc->g_setup)
        pc->g_setup = capture_graph(pc, [&](hipStream_t ss) {
          if (pc->precision == 1) numeric_setup<float>(pc, ss, false);
          else numeric_setup<double>(pc, ss, false);
        });
      HIPCHK(hipGraphLaunch(pc->g_setup, s));
      pc->coarse_pending = false;
    } else if (pc->precision == 1) {
      numeric_setup<float>(pc, s, !pc->opt.graph);
    } else {
      numeric_setup<double>(pc, s, !pc->opt.graph);
    }
    HIPCHK(hipGetLastError());
  } catch (const HipFail& f) {
    return set_err(BDDCSO_EHIP, f.where + ": " + hipGetErrorString(f.e));
  }
  return BDDCSO_OK;
}

bddcso_status bddcso_check_pivots(bddcso_precond* pc, void* stream) {
  if (!pc) return set_err(BDDCSO_EINVAL, "null precond");
  int st = 0;
  hipStream_t s = as_stream(stream);
  if (pc->coarse_pending && hipStreamWaitEvent(s, pc->ev_coarse, 0) != hipSuccess)
    return set_err(BDDCSO_EHIP, "wait for the coarse factorization failed");
  if (hipMemcpyAsync(&st, pc->status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_err(BDDCSO_EHIP, "status copy failed");
  static const char* what[] = {"", "an interior (Dirichlet) block", "a constrained Neumann block",
                               "the constraint Schur complement", "the coarse matrix"};
  if (st > 0)
    return set_err(BDDCSO_ESINGULAR, std::string("non-positive pivot in ") + what[std::min(st, 4)] +
                                         " (not enough primal constraints, or rho <= 0)");
  return BDDCSO_OK;
}

bddcso_status bddcso_setup_workspace_size(bddcso_problem* p, const bddcso_options* opts, size_t* bytes) {
  if (!p || !bytes) return set_err(BDDCSO_EINVAL, "null argument");
  bddcso_precond* pc = nullptr;
  size_t need = 0;
  bddcso_status st = create_precond(p, opts, DevMem::COUNT, nullptr, 0, nullptr, &pc, &need);
  if (st != BDDCSO_OK) return st;
  *bytes = need;
  return BDDCSO_OK;
}

bddcso_status bddcso_setup(bddcso_problem* p, const double* rho_dev, const bddcso_options* opts,
                           void* workspace_dev, size_t ws_bytes, void* stream, bddcso_precond** out) {
  if (!p || !rho_dev || !out) return set_err(BDDCSO_EINVAL, "null argument");
  *out = nullptr;
  if (workspace_dev && ((uintptr_t)workspace_dev % DevMem::kAlign))
    return set_err(BDDCSO_EINVAL, "workspace must be 256-byte aligned");
  bddcso_precond* pc = nullptr;
  bddcso_status st = create_precond(p, opts, workspace_dev ? DevMem::CARVE : DevMem::MALLOC, workspace_dev,
                                    ws_bytes, as_stream(stream), &pc, nullptr);
  if (st != BDDCSO_OK) return st;
  st = bddcso_refactor(pc, rho_dev, stream);
  if (st == BDDCSO_OK) st = bddcso_check_pivots(pc, stream);
  if (st != BDDCSO_OK) {
    std::string msg = g_last_error;
    bddcso_precond_destroy(pc);
    return set_err(st, msg);
  }
  *out = pc;
  return BDDCSO_OK;
}

bddcso_status bddcso_operator_apply(const bddcso_precond* pc, const double* x, double* y, int nrhs, void* stream) {
  if (!pc || !x || !y) return set_err(BDDCSO_EINVAL, "null argument");
  if (nrhs < 1) return set_err(BDDCSO_EINVAL, "nrhs must be >= 1");
  if (x == y) return set_err(BDDCSO_EINVAL, "x and y must be distinct");
  launch_q1_apply(pc->geo, pc->khat, pc->rho, x, y, nrhs, as_stream(stream));
  if (hipGetLastError() != hipSuccess) return set_err(BDDCSO_EHIP, "q1 apply launch failed");
  return BDDCSO_OK;
}

bddcso_status bddcso_apply(bddcso_precond* pc, const double* r, double* z, int nrhs, void* stream) {
  if (!pc || !r || !z) return set_err(BDDCSO_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > pc->max_nrhs) return set_err(BDDCSO_EINVAL, "nrhs must be in 1..max_nrhs");
  if (r == z) return set_err(BDDCSO_EINVAL, "r and z must be distinct");
  try {
    apply_B_any(pc, r, z, nrhs, as_stream(stream));
  } catch (const HipFail& f) {
    return set_err(BDDCSO_EHIP, "HIP error in apply: " + f.where);
  }
  if (hipGetLastError() != hipSuccess) return set_err(BDDCSO_EHIP, "kernel launch failed in apply");
  return BDDCSO_OK;
}

}  // extern "C"

namespace {

// Device state of one PCG solve: the vectors ([nrhs][n_free] each), the dot
// partials, the scalar slots (8 x BDDCSO_MAX_RHS), the per-iteration
// (alpha, beta) history and the per-column flags.
struct Krylov {
  double *r, *p, *qv, *z, *rold, *dtmp, *partial, *sc, *hist_a, *hist_b;
  int32_t *active, *iters, *flags, *nactive;
};

Krylov precond_krylov(bddcso_precond* pc) {
  return {pc->r, pc->p, pc->qv, pc->z, pc->rold, pc->dtmp, pc->partial, pc->sc, pc->hist_a, pc->hist_b,
          pc->active, pc->iters, pc->flags, pc->nactive};
}

// Cuts a Krylov state for nrhs columns, in a fixed order with 256-byte
// aligned pieces, from base (nullptr: only counts).  Returns the bytes used.
size_t carve_krylov(char* base, int64_t n, int nr, int dot_blocks, int maxit, Krylov* k) {
  size_t used = 0;
  auto take = [&](size_t bytes) {
    const size_t off = (used + 255) / 256 * 256;
    used = off + std::max<size_t>(bytes, 1);
    return base ? (void*)(base + off) : nullptr;
  };
  const size_t vec = (size_t)n * nr * sizeof(double);
  Krylov t;
  t.r = (double*)take(vec);
  t.p = (double*)take(vec);
  t.qv = (double*)take(vec);
  t.z = (double*)take(vec);
  t.rold = (double*)take(vec);
  t.dtmp = (double*)take(vec);
  t.partial = (double*)take((size_t)dot_blocks * nr * sizeof(double));
  t.sc = (double*)take(8 * BDDCSO_MAX_RHS * sizeof(double));
  t.hist_a = (double*)take((size_t)(maxit + 1) * nr * sizeof(double));
  t.hist_b = (double*)take((size_t)(maxit + 1) * nr * sizeof(double));
  t.active = (int32_t*)take(nr * sizeof(int32_t));
  t.iters = (int32_t*)take(nr * sizeof(int32_t));
  t.flags = (int32_t*)take(nr * sizeof(int32_t));
  t.nactive = (int32_t*)take(sizeof(int32_t));
  if (k) *k = t;
  return used;
}

bddcso_status solve_impl(bddcso_precond* pc, const Krylov& K, const double* b, double* x, int nrhs,
                         bddcso_stats* stats, void* stream) {
  hipStream_t s = as_stream(stream);
  auto t0 = std::chrono::steady_clock::now();
  const int64_t n = pc->geo.n_free;
  const int nr = nrhs;
  const bddcso_options& o = pc->opt;
  const bool flex = o.flexible || pc->precision == 1;
  const int limit = o.fixed_iters > 0 ? o.fixed_iters : o.maxit;
  double* SC = K.sc;
  double *s_bb = SC, *s_rz = SC + 64, *s_pq = SC + 128, *s_rr = SC + 192, *s_rzn = SC + 256, *s_num = SC + 320,
         *s_tol = SC + 384;
  std::vector<double> hbb(nr), htol(nr);
  std::vector<int32_t> hact(nr);
  int k_done = 0;
  try {
    // With the coarse factorization still running (ordinary mode), its
    // pivots are checked after the solve instead, so the first application's
    // local solves overlap it; a non-positive pivot then still returns
    // ESINGULAR.
    const bool defer_pivots = pc->coarse_pending;
    if (!defer_pivots) {
      bddcso_status pst = bddcso_check_pivots(pc, stream);
      if (pst != BDDCSO_OK) return pst;
    }
    launch_fill_f64(x, n * nr, 0.0, s);
    HIPCHK(hipMemcpyAsync(K.r, b, n * nr * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_dot(b, b, n, nr, K.partial, pc->dot_blocks, s_bb, s);
    HIPCHK(hipMemcpyAsync(hbb.data(), s_bb, nr * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int j = 0; j < nr; ++j) {
      if (!std::isfinite(hbb[j])) return set_err(BDDCSO_EINVAL, "right-hand side is not finite");
      htol[j] = o.fixed_iters > 0 ? -1.0 : o.rtol * o.rtol * hbb[j];
      hact[j] = hbb[j] > 0.0 ? 1 : 0;
    }
    HIPCHK(hipMemcpyAsync(s_tol, htol.data(), nr * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(K.active, hact.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice, s));
    launch_fill_i32(K.iters, nr, 0, s);
    launch_fill_i32(K.flags, nr, 0, s);
    apply_B_any(pc, K.r, K.z, nr, s);
    HIPCHK(hipMemcpyAsync(K.p, K.z, n * nr * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_dot(K.r, K.z, n, nr, K.partial, pc->dot_blocks, s_rz, s);
    int any = 0;
    for (int j = 0; j < nr; ++j) any |= hact[j];
    // One iteration in two halves: the operator and the x, r update up to
    // the convergence test, then the preconditioner and the p update.
    // kd: device iteration counter of replayed graphs (nullptr: k).
    auto half1 = [&](hipStream_t ss, int k, const int32_t* kd, double* xw) {
      if (pc->P_()) pc->prof.begin(8, ss);
      launch_q1_apply(pc->geo, pc->khat, pc->rho, K.p, K.qv, nr, ss);
      if (pc->P_()) {  // x read and y written per column, rho once
        const double f = 2.0 * (pc->geo.dim == 3 ? 27 : 9) * (double)n * nr;
        const double b = 8.0 * (2.0 * (double)n * nr + (double)pc->geo.n_elem);
        pc->prof.end(8, f, b, ss);
        pc->prof.ref(8, f, b);
      }
      launch_dot(K.p, K.qv, n, nr, K.partial, pc->dot_blocks, s_pq, ss);
      if (flex) launch_copy_f64(K.r, K.rold, n * nr, ss);
      launch_pcg_xr(xw, K.r, K.p, K.qv, s_rz, s_pq, K.active, n, nr, ss);
      launch_dot(K.r, K.r, n, nr, K.partial, pc->dot_blocks, s_rr, ss);
      launch_pcg_book1(nr, k, kd, s_rz, s_pq, s_rr, s_tol, K.active, K.iters, K.flags, K.hist_a, K.nactive, ss);
    };
    auto half2 = [&](hipStream_t ss, int k, int32_t* kd) {
      apply_B_any(pc, K.r, K.z, nr, ss);
      launch_dot(K.r, K.z, n, nr, K.partial, pc->dot_blocks, s_rzn, ss);
      if (flex) {
        launch_sub(K.r, K.rold, K.dtmp, n * nr, ss);
        launch_dot(K.z, K.dtmp, n, nr, K.partial, pc->dot_blocks, s_num, ss);
        launch_pcg_p(K.p, K.z, s_num, s_rz, K.active, n, nr, ss);
        launch_pcg_book2(nr, k, kd, s_rz, s_num, s_rzn, K.active, K.hist_b, ss);
      } else {
        launch_pcg_p(K.p, K.z, s_rzn, s_rz, K.active, n, nr, ss);
        launch_pcg_book2(nr, k, kd, s_rz, s_rzn, s_rzn, K.active, K.hist_b, ss);
      }
    };
    // Graph mode: the two halves are captured once per right-hand-side
    // count and replayed; x accumulates in the preconditioner's own buffer.
    const bool graph = o.graph && !pc->P_() && K.r == pc->r;
    GraphPair* gp = nullptr;
    if (graph) {
      gp = &pc->iter_graphs[nr];
      if (!gp->g1) gp->g1 = capture_graph(pc, [&](hipStream_t ss) { half1(ss, 0, pc->kdev, pc->xk); });
      if (!gp->g2) gp->g2 = capture_graph(pc, [&](hipStream_t ss) { half2(ss, 0, pc->kdev); });
      launch_fill_f64(pc->xk, n * nr, 0.0, s);
      launch_fill_i32(pc->kdev, 1, 0, s);
    }
    for (int k = 0; any && k < limit; ++k) {
      if (graph) HIPCHK(hipGraphLaunch(gp->g1, s));
      else half1(s, k, nullptr, x);
      k_done = k + 1;
      if (o.fixed_iters <= 0) {
        HIPCHK(hipMemcpyAsync(pc->h_nactive, K.nactive, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (*pc->h_nactive == 0) break;
      }
      if (k + 1 == limit) break;
      if (graph) HIPCHK(hipGraphLaunch(gp->g2, s));
      else half2(s, k, nullptr);
    }
    if (graph) launch_copy_f64(pc->xk, x, n * nr, s);
    HIPCHK(hipGetLastError());
    // results
    std::vector<int32_t> it(nr), fl(nr);
    std::vector<double> rr(nr), ha((size_t)std::max(k_done, 1) * nr), hb((size_t)std::max(k_done, 1) * nr);
    HIPCHK(hipMemcpyAsync(it.data(), K.iters, nr * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(fl.data(), K.flags, nr * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rr.data(), s_rr, nr * sizeof(double), hipMemcpyDeviceToHost, s));
    if (k_done > 0) {
      HIPCHK(hipMemcpyAsync(ha.data(), K.hist_a, (size_t)k_done * nr * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(hb.data(), K.hist_b, (size_t)k_done * nr * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (defer_pivots) {
      bddcso_status pst = bddcso_check_pivots(pc, stream);
      if (pst != BDDCSO_OK) return pst;
    }
    auto t1 = std::chrono::steady_clock::now();
    bool breakdown = false, noconv = false;
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->nrhs = nr;
      stats->n_coarse = pc->plan->n_coarse;
      stats->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    for (int j = 0; j < nr; ++j) {
      if (fl[j] & 2) breakdown = true;
      bool conv = (fl[j] & 1) || hbb[j] == 0.0;
      if (o.fixed_iters > 0) conv = rr[j] <= o.rtol * o.rtol * hbb[j];
      if (!conv && o.fixed_iters <= 0) noconv = true;
      if (stats) {
        stats->iters[j] = it[j];
        stats->converged[j] = conv ? 1 : 0;
        stats->relres[j] = hbb[j] > 0 ? std::sqrt(std::max(rr[j], 0.0) / hbb[j]) : 0.0;
        int m = it[j];
        std::vector<double> d(m), e(m > 0 ? m - 1 : 0);
        for (int i = 0; i < m; ++i) {
          double a = ha[(size_t)i * nr + j];
          d[i] = 1.0 / a;
          if (i > 0) {
            double ap = ha[(size_t)(i - 1) * nr + j], bp = hb[(size_t)(i - 1) * nr + j];
            d[i] += bp / ap;
            e[i - 1] = std::sqrt(std::max(bp, 0.0)) / ap;
          }
        }
        double lo = 1, hi = 1;
        tridiag_extremes(d, e, lo, hi);
        stats->lambda_min[j] = lo;
        stats->lambda_max[j] = hi;
        stats->kappa[j] = hi / lo;
      }
    }
    if (breakdown) return set_err(BDDCSO_EBREAKDOWN, "PCG breakdown (p^T A p <= 0 or r^T z <= 0)");
    if (noconv) return set_err(BDDCSO_ENOCONV, "maxit reached before rtol");
  } catch (const HipFail& f) {
    return set_err(BDDCSO_EHIP, f.where + ": " + hipGetErrorString(f.e));
  }
  return BDDCSO_OK;
}

// The static scratch of the allocation-free solve (each device holds its own
// copy from module load until the process ends).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's scratch, looked up once per device (the
// array's host-side name is not a device address).
bddcso_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return set_err(BDDCSO_EHIP, "hipGetDevice failed or device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_err(BDDCSO_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return BDDCSO_OK;
}

}  // namespace

extern "C" {

bddcso_status bddcso_solve(bddcso_precond* pc, const double* b, double* x, int nrhs, bddcso_stats* stats,
                           void* stream) {
  if (!pc || !b || !x) return set_err(BDDCSO_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > pc->max_nrhs) return set_err(BDDCSO_EINVAL, "nrhs must be in 1..max_nrhs");
  if (b == x) return set_err(BDDCSO_EINVAL, "b and x must be distinct");
  return solve_impl(pc, precond_krylov(pc), b, x, nrhs, stats, stream);
}

bddcso_status bddcso_solve_noalloc(bddcso_precond* pc, const double* b, double* x, int nrhs, bddcso_stats* stats,
                                   void* stream) {
  if (!pc || !b || !x) return set_err(BDDCSO_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > pc->max_nrhs) return set_err(BDDCSO_EINVAL, "nrhs must be in 1..max_nrhs");
  if (b == x) return set_err(BDDCSO_EINVAL, "b and x must be distinct");
  const int maxit = std::max(pc->opt.maxit, pc->opt.fixed_iters);
  const size_t need = carve_krylov(nullptr, pc->geo.n_free, nrhs, pc->dot_blocks, maxit, nullptr);
  if (need > kNoAllocScratchBytes)
    return set_err(BDDCSO_EINVAL, "solve state of " + std::to_string(need) + " bytes exceeds the " +
                                      std::to_string(kNoAllocScratchBytes) +
                                      "-byte static scratch (about n_free * nrhs <= 1.39e6)");
  void* base = nullptr;
  bddcso_status st = scratch_address(&base);
  if (st != BDDCSO_OK) return st;
  Krylov K;
  carve_krylov((char*)base, pc->geo.n_free, nrhs, pc->dot_blocks, maxit, &K);
  return solve_impl(pc, K, b, x, nrhs, stats, stream);
}

bddcso_status bddcso_element_grad(const bddcso_precond* pc, const double* u, const double* lam, double* g,
                                  int nrhs, void* stream) {
  if (!pc || !u || !lam || !g) return set_err(BDDCSO_EINVAL, "null argument");
  if (nrhs < 1) return set_err(BDDCSO_EINVAL, "nrhs must be >= 1");
  launch_element_grad(pc->geo, pc->khat, pc->rho, u, lam, g, nrhs, as_stream(stream));
  if (hipGetLastError() != hipSuccess) return set_err(BDDCSO_EHIP, "element grad launch failed");
  return BDDCSO_OK;
}

bddcso_status bddcso_box_filter(const bddcso_problem* p, const double* in, double* out, int transpose,
                                void* stream) {
  if (!p || !in || !out) return set_err(BDDCSO_EINVAL, "null argument");
  if (in == out) return set_err(BDDCSO_EINVAL, "in and out must be distinct");
  Geo g{};
  g.dim = p->c.dim;
  for (int a = 0; a < 3; ++a) {
    g.ne[a] = (int)p->c.ne[a];
    g.nf[a] = (int)p->c.nf[a];
  }
  g.n_free = p->c.n_free;
  g.n_elem = p->c.n_elem;
  launch_box_filter(g, in, out, transpose ? 1 : 0, as_stream(stream));
  if (hipGetLastError() != hipSuccess) return set_err(BDDCSO_EHIP, "box filter launch failed");
  return BDDCSO_OK;
}

bddcso_status bddcso_coef_from_log(const bddcso_problem* p, const double* theta, double* rho, void* stream) {
  if (!p || !theta || !rho) return set_err(BDDCSO_EINVAL, "null argument");
  if (theta == rho) return set_err(BDDCSO_EINVAL, "theta and rho must be distinct");
  Geo g{};
  g.dim = p->c.dim;
  for (int a = 0; a < 3; ++a) {
    g.ne[a] = (int)p->c.ne[a];
    g.nf[a] = (int)p->c.nf[a];
  }
  g.n_free = p->c.n_free;
  g.n_elem = p->c.n_elem;
  launch_box_filter(g, theta, rho, 2, as_stream(stream));
  if (hipGetLastError() != hipSuccess) return set_err(BDDCSO_EHIP, "box filter launch failed");
  return BDDCSO_OK;
}

bddcso_status bddcso_precond_generation(const bddcso_precond* pc, int64_t* generation) {
  if (!pc || !generation) return set_err(BDDCSO_EINVAL, "null argument");
  *generation = pc->generation;
  return BDDCSO_OK;
}

bddcso_status bddcso_autotune(bddcso_problem* p, const double* rho_dev, const bddcso_options* base,
                              const double* b_dev, int nrhs, void* stream, bddcso_options* best,
                              bddcso_tune_report* report) {
  if (!p || !rho_dev || !b_dev || !best) return set_err(BDDCSO_EINVAL, "null argument");
  bddcso_options o0;
  if (base) o0 = *base;
  else bddcso_default_options(&o0);
  if (nrhs < 1 || nrhs > BDDCSO_MAX_RHS) return set_err(BDDCSO_EINVAL, "nrhs must be in 1..64");
  o0.max_nrhs = std::max(o0.max_nrhs, nrhs);
  // the knobs' defaults made explicit, so no variant repeats the base
  if (o0.sweep_reg_rows == 0) o0.sweep_reg_rows = kRegSweepMaxRows;
  if (o0.mr_min_rhs == 0) o0.mr_min_rhs = 4;
  if (o0.block_target == 0) o0.block_target = 192;
  if (o0.update_tile == 0) o0.update_tile = 64;
  hipStream_t s = as_stream(stream);
  bddcso_tune_report R;
  std::memset(&R, 0, sizeof(R));
  double* x = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMalloc((void**)&x, sizeof(double) * (size_t)p->c.n_free * nrhs) != hipSuccess)
    return set_err(BDDCSO_ENOMEM, "autotune: device allocation failed");
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipFree(x);
    return set_err(BDDCSO_EHIP, "autotune: event creation failed");
  }
  const double inf = std::numeric_limits<double>::infinity();
  // one trial: a preconditioner for these options, an untimed step, then a
  // step (numeric setup + solve) timed with events on the stream
  auto trial = [&](const bddcso_options& o) -> double {
    if (R.n_trials >= BDDCSO_TUNE_MAX) return inf;
    const int t = R.n_trials++;
    R.tried[t] = o;
    R.step_ms[t] = inf;
    bddcso_precond* pc = nullptr;
    bddcso_status st = bddcso_setup(p, rho_dev, &o, nullptr, 0, stream, &pc);
    if (st == BDDCSO_OK) st = bddcso_solve(pc, b_dev, x, nrhs, nullptr, stream);
    if (st == BDDCSO_OK || st == BDDCSO_ENOCONV) {
      st = BDDCSO_OK;
      bool ok = hipEventRecord(e0, s) == hipSuccess;
      bddcso_status s1 = bddcso_refactor(pc, rho_dev, stream);
      bddcso_status s2 = s1 == BDDCSO_OK ? bddcso_solve(pc, b_dev, x, nrhs, nullptr, stream) : s1;
      ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
      float ms = 0.f;
      if (ok && (s2 == BDDCSO_OK || s2 == BDDCSO_ENOCONV) && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
        R.step_ms[t] = ms;
      else
        st = s2 != BDDCSO_OK ? s2 : BDDCSO_EHIP;
    }
    if (pc) bddcso_precond_destroy(pc);
    R.status[t] = st;
    return R.step_ms[t];
  };
  bddcso_options cur = o0;
  double best_ms = trial(cur);
  R.best = 0;
  // a variant replaces the current choice only when it is more than 1% faster
  auto knob = [&](int bddcso_options::*field, std::initializer_list<int> values) {
    for (int v : values) {
      if (cur.*field == v) continue;
      bddcso_options cand = cur;
      cand.*field = v;
      const double ms = trial(cand);
      if (ms < 0.99 * best_ms) {
        best_ms = ms;
        cur = cand;
        R.best = R.n_trials - 1;
      }
    }
  };
  knob(&bddcso_options::update_tile, {64, 128});
  knob(&bddcso_options::slab_width, {0, 192, 96});
  knob(&bddcso_options::slab_lookahead, {0, 1, 2});
  knob(&bddcso_options::sweep_reg_rows, {kRegSweepMaxRows, 272});
  knob(&bddcso_options::block_target, {192, 128, 256});
  if (nrhs > 1) knob(&bddcso_options::mr_min_rhs, {4, 2, 8, BDDCSO_MAX_RHS + 1});
  knob(&bddcso_options::graph, {0, 1});
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(x);
  if (!(best_ms < inf)) {
    if (report) *report = R;
    return set_err(R.status[0] != BDDCSO_OK ? (bddcso_status)R.status[0] : BDDCSO_EHIP,
                   "autotune: no variant completed a step");
  }
  *best = cur;
  if (report) *report = R;
  return BDDCSO_OK;
}

bddcso_status bddcso_plan_info(bddcso_problem* p, const bddcso_options* opts, bddcso_plan_stats* out) {
  if (!p || !out) return set_err(BDDCSO_EINVAL, "null argument");
  bddcso_options o;
  if (opts) o = *opts;
  else bddcso_default_options(&o);
  Error err;
  std::shared_ptr<Plan> plan;
  try {
    plan = get_plan(p, o, err);
  } catch (const std::bad_alloc&) {
    return set_err(BDDCSO_ENOMEM, "host allocation failed while planning");
  }
  if (!plan) return set_err(BDDCSO_EINVAL, err.msg);
  const Plan& pl = *plan;
  std::memset(out, 0, sizeof(*out));
  out->n_coarse = pl.n_coarse;
  out->n_fronts = (int64_t)pl.fronts.size();
  out->levels = (int64_t)pl.level_fronts.size() - 1;
  for (const FrontDev& F : pl.fronts) {
    out->max_front = std::max<int64_t>(out->max_front, F.n);
    out->max_front_pivots = std::max<int64_t>(out->max_front_pivots, F.p);
    out->coarse_factor_entries += (double)F.n * F.p;
    out->coarse_sweep_flops += (double)F.n * F.n * F.p;
  }
  out->n_blocks = (int64_t)pl.blocks.size();
  out->max_block = pl.max_block;
  for (const BlockDev& B : pl.blocks) out->local_sweep_flops += (double)B.size * B.size * B.size;
  for (const SubDev& S : pl.subs) out->local_sweep_flops += (double)S.n_a * S.n_a * S.n_a;
  bddcso_precond* tmp = nullptr;
  size_t need = 0;
  bddcso_status st = create_precond(p, &o, DevMem::COUNT, nullptr, 0, nullptr, &tmp, &need);
  if (st != BDDCSO_OK) return st;
  out->device_bytes = (double)need;
  return BDDCSO_OK;
}

bddcso_status bddcso_profile(bddcso_precond* pc, int class_mask) {
  if (!pc) return set_err(BDDCSO_EINVAL, "null precond");
  if (class_mask < 0 || class_mask > (1 << (kNumClasses + 1)) - 2)
    return set_err(BDDCSO_EINVAL, "class mask must use bits 1..8");
  pc->prof.reset(class_mask);
  return BDDCSO_OK;
}

bddcso_status bddcso_profile_read(bddcso_precond* pc, int kernel_class, int64_t* launches, double* total_ms,
                                  double* flops, double* bytes) {
  if (!pc) return set_err(BDDCSO_EINVAL, "null precond");
  if (kernel_class < 1 || kernel_class > kNumClasses) return set_err(BDDCSO_EINVAL, "kernel class must be in 1..8");
  auto& R = pc->prof.rec[kernel_class];
  double ms = 0.0;
  for (size_t i = 0; i + 1 < R.used; i += 2) {
    if (hipEventSynchronize(R.ev[i + 1]) != hipSuccess) return set_err(BDDCSO_EHIP, "event sync failed");
    float t = 0.f;
    if (hipEventElapsedTime(&t, R.ev[i], R.ev[i + 1]) != hipSuccess)
      return set_err(BDDCSO_EHIP, "event timing failed");
    ms += t;
  }
  if (launches) *launches = R.launches;
  if (total_ms) *total_ms = ms;
  if (flops) *flops = R.flops;
  if (bytes) *bytes = R.bytes;
  return BDDCSO_OK;
}

bddcso_status bddcso_profile_reference(const bddcso_precond* pc, int kernel_class, double* flops, double* bytes) {
  if (!pc) return set_err(BDDCSO_EINVAL, "null precond");
  if (kernel_class < 1 || kernel_class > kNumClasses) return set_err(BDDCSO_EINVAL, "kernel class must be in 1..8");
  const auto& R = pc->prof.rec[kernel_class];
  if (flops) *flops = R.ref_flops;
  if (bytes) *bytes = R.ref_bytes;
  return BDDCSO_OK;
}

bddcso_status bddcso_copy_probe(const void* src_dev, void* dst_dev, int64_t bytes, void* stream) {
  if (!src_dev || !dst_dev || bytes < 0 || bytes % 16) return set_err(BDDCSO_EINVAL, "bytes must be a multiple of 16");
  launch_copy16(src_dev, dst_dev, bytes / 16, as_stream(stream));
  if (hipGetLastError() != hipSuccess) return set_err(BDDCSO_EHIP, "copy launch failed");
  return BDDCSO_OK;
}

bddcso_status bddcso_precond_info(const bddcso_precond* pc, int64_t* n_coarse, int64_t* n_fronts,
                                  int64_t* device_bytes, int64_t* coarse_factor_entries) {
  if (!pc) return set_err(BDDCSO_EINVAL, "null precond");
  if (n_coarse) *n_coarse = pc->plan->n_coarse;
  if (n_fronts) *n_fronts = (int64_t)pc->plan->fronts.size();
  if (device_bytes) *device_bytes = pc->mem.bytes;
  if (coarse_factor_entries) {
    int64_t t = 0;
    for (auto& F : pc->plan->fronts) t += (int64_t)F.n * F.p;
    *coarse_factor_entries = t;
  }
  return BDDCSO_OK;
}

bddcso_status bddcso_local_coarse(const bddcso_precond* pc, int sub, double* kc, int64_t* ids, int64_t cap_nc,
                                  int64_t* nc, void* stream) {
  if (!pc || !kc || !ids || !nc) return set_err(BDDCSO_EINVAL, "null argument");
  const Plan& pl = *pc->plan;
  if (sub < 0 || sub >= (int)pl.subs.size()) return set_err(BDDCSO_EINVAL, "subdomain out of range");
  const SubDev& S = pl.subs[sub];
  *nc = S.n_c;
  if (S.n_c > cap_nc) return set_err(BDDCSO_EINVAL, "output buffers too small");
  hipStream_t s = as_stream(stream);
  const size_t cnt = (size_t)S.n_c * S.n_c;
  if (pc->precision == 1) {
    std::vector<float> tmp(cnt);
    if (cnt && hipMemcpyAsync(tmp.data(), pc->nf.Kc + S.Kc_off, cnt * sizeof(float), hipMemcpyDeviceToHost, s))
      return set_err(BDDCSO_EHIP, "copy failed");
    if (hipStreamSynchronize(s) != hipSuccess) return set_err(BDDCSO_EHIP, "sync failed");
    for (size_t i = 0; i < cnt; ++i) kc[i] = tmp[i];
  } else {
    if (cnt && hipMemcpyAsync(kc, pc->nd.Kc + S.Kc_off, cnt * sizeof(double), hipMemcpyDeviceToHost, s))
      return set_err(BDDCSO_EHIP, "copy failed");
    if (hipStreamSynchronize(s) != hipSuccess) return set_err(BDDCSO_EHIP, "sync failed");
  }
  for (int k = 0; k < S.n_c; ++k) ids[k] = pl.c_glob[S.c_off + k];
  return BDDCSO_OK;
}

}  // extern "C"
