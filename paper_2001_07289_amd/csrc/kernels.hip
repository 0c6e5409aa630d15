// HIP kernels for gfx950 (CDNA4): the BDDC-SO setup, the preconditioner
// application, the Q1 operator and the PCG vector work.
//
// Dense contractions (the rank-k updates of the block inversions and the
// batched GEMMs of the setup) run on MFMA: v_mfma_f64_16x16x4_f64 in FP64,
// v_mfma_f32_16x16x4_f32 in FP32, 64x64 tiles per 256-thread workgroup (four
// 64-wide waves, 32x32 each).  Everything else is HBM-bound streaming:
// coalesced along the fastest index, reductions in fixed order (no
// floating-point atomics), so results are bitwise repeatable.
#include <hip/hip_runtime.h>
#include <utility>

#include <algorithm>
#include <cstdio>

#include "kernels.h"

namespace bddcso {

namespace {

constexpr int TILE = 64;
constexpr int BK = 16;
constexpr int PAD = 4;
constexpr int SWEEP_NB = kSweepNB;  // pivots per panel

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Inputs of both 16x16x4 forms: lane l holds A[l%16][l/16] and B[l/16][l%16].
// Outputs: lane l, register r holds D[row(l/16, r)][l%16]; the FP64 form
// interleaves the rows (l/16 + 4r), the FP32 form blocks them (4(l/16) + r).
template <>
struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int r) { return kq + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int r) { return 4 * kq + r; }
};

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
inline int64_t hmin(int64_t a, int64_t b) { return a < b ? a : b; }
inline int64_t hmax(int64_t a, int64_t b) { return a > b ? a : b; }

// ---------------------------------------------------------------------------
// geometry helpers

__device__ __forceinline__ void loc_coords(const SubDev& S, int l, int c[3]) {
  c[0] = l % S.m[0];
  c[1] = (l / S.m[0]) % S.m[1];
  c[2] = l / (S.m[0] * S.m[1]);
}

__device__ __forceinline__ int loc_index(const SubDev& S, const int c[3]) {
  if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= S.m[0] || c[1] >= S.m[1] || c[2] >= S.m[2])
    return -1;
  return c[0] + S.m[0] * (c[1] + S.m[1] * c[2]);
}

// Free-node index of local node l of S.
__device__ __forceinline__ int64_t free_of_local(const SubDev& S, const Geo& g, int l) {
  int c[3];
  loc_coords(S, l, c);
  return (int64_t)(S.lo[0] + c[0] - 1) +
         (int64_t)g.nf[0] * ((int64_t)(S.lo[1] + c[1] - 1) + (int64_t)g.nf[1] * (S.lo[2] + c[2] - 1));
}

// Entry of the local stiffness matrix K_i between two local nodes (local
// coordinates ca, cb, at most one step apart per axis): the sum over the
// elements of this subdomain that contain both of rho_e K^_e[a, b].
__device__ __forceinline__ double kloc(const SubDev& S, const Geo& g, const double* __restrict__ rho,
                                       const double* __restrict__ khat, const int ca[3],
                                       const int cb[3]) {
  int ga[3], gb[3], lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ga[a] = S.lo[a] + ca[a];
    gb[a] = S.lo[a] + cb[a];
    lo[a] = max(max(ga[a], gb[a]) - 1, S.elo[a]);
    hi[a] = min(min(ga[a], gb[a]), S.ehi[a] - 1);
  }
  double s = 0.0;
  for (int ez = lo[2]; ez <= hi[2]; ++ez)
    for (int ey = lo[1]; ey <= hi[1]; ++ey)
      for (int ex = lo[0]; ex <= hi[0]; ++ex) {
        int64_t e = ex + (int64_t)g.ne[0] * (ey + (int64_t)g.ne[1] * ez);
        int ia = (ga[0] - ex) + 2 * (ga[1] - ey) + 4 * (ga[2] - ez);
        int ib = (gb[0] - ex) + 2 * (gb[1] - ey) + 4 * (gb[2] - ez);
        s += rho[e] * khat[ia * 8 + ib];
      }
  return s;
}

// t-th neighbour (t < 9 in 3D, < 3 in 2D) of c in the adjacent plane c[pa]+dir.
__device__ __forceinline__ bool plane_nbr(const SubDev& S, int dim, const int c[3], int dir, int t,
                                          int out[3]) {
  out[0] = c[0];
  out[1] = c[1];
  out[2] = c[2];
  if (dim == 3) {
    out[2] += dir;
    out[0] += t % 3 - 1;
    out[1] += t / 3 - 1;
  } else {
    if (t >= 3) return false;
    out[1] += dir;
    out[0] += t - 1;
  }
  return out[0] >= 0 && out[1] >= 0 && out[2] >= 0 && out[0] < S.m[0] && out[1] < S.m[1] &&
         out[2] < S.m[2];
}

__device__ __forceinline__ const int32_t* set_loc_of(const PlanDev& P, const SubDev& S, int setR) {
  return setR ? P.r_loc + S.r_off : P.I_loc + S.I_off;
}
__device__ __forceinline__ const int32_t* loc_set_of(const PlanDev& P, const SubDev& S, int setR) {
  return (setR ? P.loc_r : P.loc_I) + S.loc_off;
}

// ---------------------------------------------------------------------------
// elementwise

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_f32_to_f64(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) b[i] = (double)a[i];
}

// Plain streaming copy (16 B per thread and step), used to calibrate the
// hardware byte counters against a known traffic.
__global__ void k_copy16(const int4* __restrict__ a, int4* __restrict__ b, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) b[i] = a[i];
}

__global__ void k_sub(const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ o, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) o[i] = a[i] - b[i];
}

// ---------------------------------------------------------------------------
// global Q1 operator: y = A x, one thread per free node (and right-hand side).
// Each row sums the 2^dim surrounding elements' contributions; boundary
// nodes carry zero.  Reads x and rho through the cache: about 24 B per dof
// of HBM traffic.

__global__ __launch_bounds__(256) void k_q1_apply(Geo g, const double* __restrict__ khat,
                                                  const double* __restrict__ rho,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ y) {
  __shared__ double kh[64];
  if (threadIdx.x < 64) kh[threadIdx.x] = khat[threadIdx.x];
  __syncthreads();
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int rhs = blockIdx.y;
  if (f >= g.n_free) return;
  const double* xr = x + rhs * g.n_free;
  int gx = (int)(f % g.nf[0]) + 1;
  int64_t t = f / g.nf[0];
  int gy = (int)(t % g.nf[1]) + 1;
  int gz = g.dim == 3 ? (int)(t / g.nf[1]) + 1 : 1;
  const int nz_el = g.dim == 3 ? 2 : 1;
  double acc = 0.0;
  for (int cz = 0; cz < nz_el; ++cz) {
    int ez = g.dim == 3 ? gz - 1 + cz : 0;
    for (int cy = 0; cy < 2; ++cy) {
      int ey = gy - 1 + cy;
      for (int cx = 0; cx < 2; ++cx) {
        int ex = gx - 1 + cx;
        int64_t e = ex + (int64_t)g.ne[0] * (ey + (int64_t)g.ne[1] * ez);
        int a = (gx - ex) + 2 * (gy - ey) + 4 * (gz - ez);
        double s = 0.0;
        for (int b = 0; b < (g.dim == 3 ? 8 : 4); ++b) {
          int nx = ex + (b & 1), ny = ey + ((b >> 1) & 1);
          int nzc = g.dim == 3 ? ez + ((b >> 2) & 1) : 1;
          if (nx < 1 || ny < 1 || nx > g.nf[0] || ny > g.nf[1]) continue;
          if (g.dim == 3 && (nzc < 1 || nzc > g.nf[2])) continue;
          int64_t fb = (nx - 1) + (int64_t)g.nf[0] * ((ny - 1) + (int64_t)g.nf[1] * (nzc - 1));
          int bb = g.dim == 3 ? b : (b | 4);
          s += kh[a * 8 + bb] * xr[fb];
        }
        acc += rho[e] * s;
      }
    }
  }
  y[rhs * g.n_free + f] = acc;
}

// 3D operator by tiles of QX x QY x QZ nodes: the tile's x values with a
// one-node halo and its elements' rho are staged in LDS once (coalesced rows
// along x), then each thread sums the 8 elements around each of its QZ nodes
// from LDS.  Tiles are dealt so that consecutive tiles (which share halo
// planes) run on one XCD and its L2.  Nodes outside the free range read 0.
constexpr int QX = 32, QY = 8, QZ = 4;

__global__ __launch_bounds__(256) void k_q1_apply3(Geo g, const double* __restrict__ khat,
                                                   const double* __restrict__ rho,
                                                   const double* __restrict__ x, double* __restrict__ y,
                                                   int tx_n, int ty_n, int ntile) {
  __shared__ double kh[64];
  __shared__ double xs[QZ + 2][QY + 2][QX + 2];
  __shared__ double rs[QZ + 1][QY + 1][QX + 1];
  // gridDim.x is a multiple of 8: XCD k (blocks k, k + 8, ...) takes the
  // logical tiles k * per .. (k + 1) * per - 1
  const int per = gridDim.x / 8;
  const int logical = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (logical >= ntile) return;
  const int tid = threadIdx.x;
  if (tid < 64) kh[tid] = khat[tid];
  const int tx = logical % tx_n, ty = (logical / tx_n) % ty_n, tz = logical / (tx_n * ty_n);
  const int X0 = 1 + tx * QX, Y0 = 1 + ty * QY, Z0 = 1 + tz * QZ;  // first node (free coordinates)
  const int nfx = g.nf[0], nfy = g.nf[1], nfz = g.nf[2];
  const double* xr = x + (int64_t)blockIdx.y * g.n_free;
  // x at nodes X0-1 .. X0+QX (0 outside 1..nf)
  for (int i = tid; i < (QZ + 2) * (QY + 2) * (QX + 2); i += 256) {
    const int ix = i % (QX + 2), iy = (i / (QX + 2)) % (QY + 2), iz = i / ((QX + 2) * (QY + 2));
    const int gx = X0 - 1 + ix, gy = Y0 - 1 + iy, gz = Z0 - 1 + iz;
    double v = 0.0;
    if (gx >= 1 && gx <= nfx && gy >= 1 && gy <= nfy && gz >= 1 && gz <= nfz)
      v = xr[(gx - 1) + nfx * ((gy - 1) + nfy * (gz - 1))];
    xs[iz][iy][ix] = v;
  }
  // rho at elements X0-1 .. X0+QX-1 (0 outside the mesh)
  for (int i = tid; i < (QZ + 1) * (QY + 1) * (QX + 1); i += 256) {
    const int ix = i % (QX + 1), iy = (i / (QX + 1)) % (QY + 1), iz = i / ((QX + 1) * (QY + 1));
    const int ex = X0 - 1 + ix, ey = Y0 - 1 + iy, ez = Z0 - 1 + iz;
    double v = 0.0;
    if (ex < g.ne[0] && ey < g.ne[1] && ez < g.ne[2]) v = rho[ex + g.ne[0] * (ey + g.ne[1] * ez)];
    rs[iz][iy][ix] = v;
  }
  __syncthreads();
  const int lx = tid % QX, ly = tid / QX;
  const int gx = X0 + lx, gy = Y0 + ly;
  if (gx > nfx || gy > nfy) return;
  double* yr = y + (int64_t)blockIdx.y * g.n_free;
#pragma unroll
  for (int lz = 0; lz < QZ; ++lz) {
    const int gz = Z0 + lz;
    if (gz > nfz) break;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
      const int a = (1 - cx) + 2 * (1 - cy) + 4 * (1 - cz);  // this node's corner of the element
      double sum = 0.0;
#pragma unroll
      for (int b = 0; b < 8; ++b)
        sum += kh[a * 8 + b] * xs[lz + cz + (b >> 2)][ly + cy + ((b >> 1) & 1)][lx + cx + (b & 1)];
      acc += rs[lz + cz][ly + cy][lx + cx] * sum;
    }
    yr[(gx - 1) + nfx * ((gy - 1) + nfy * (gz - 1))] = acc;
  }
}

// ---------------------------------------------------------------------------
// weights (eq. W / Remark 4)

__global__ void k_alpha(PlanDev P, int n_ss, const double* __restrict__ rho, int weighting,
                        double* __restrict__ alpha) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_ss) return;
  if (!weighting) {
    alpha[j] = 1.0;
    return;
  }
  double s = 0.0;
  int b = P.ss_eptr[j], e = P.ss_eptr[j + 1];
  for (int k = b; k < e; ++k) s += rho[P.ss_elem[k]];
  alpha[j] = s / (double)(e - b);
}

__global__ void k_delta(PlanDev P, const double* __restrict__ alpha, double* __restrict__ delta) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= P.tot_g) return;
  int q = P.g_gam[e];
  int sub = P.g_sub[e];
  double num = 0.0, den = 0.0;
  for (int k = P.gam_kptr[q]; k < P.gam_kptr[q + 1]; ++k) {
    int j = P.gam_key[k];
    double a = alpha[j];
    den += a;
    if (P.ss_parent[j] == sub) num += a;
  }
  delta[e] = num / den;
}

// Plane-coupling coefficients A[i, j] between a block's boundary-plane node i
// and its (up to 9) neighbours j in the adjacent plane, from rho, and for a
// first-plane row also the entries A[i, j] of its in-plane neighbours of
// rank at most its own (the part of A_kk the Schur coupling adds).  One
// thread per row decodes the node once; the rank tables are read and the
// coefficients written through LDS, so that they move as contiguous runs.
constexpr int CPL_ROWS = 256;

__global__ __launch_bounds__(CPL_ROWS) void k_coupling_coefs(PlanDev P, Geo g, const double* __restrict__ rho,
                                                             double* __restrict__ coef, double* __restrict__ icoef) {
  __shared__ double cf[CPL_ROWS * 9];
  __shared__ int rk[CPL_ROWS * 9];
  const int64_t row0 = (int64_t)blockIdx.x * CPL_ROWS;
  const int nr = (int)min((int64_t)CPL_ROWS, P.n_cpl - row0);
  const int64_t e0 = row0 * 9;
  for (int e = threadIdx.x; e < nr * 9; e += CPL_ROWS) rk[e] = P.cpl_rank[e0 + e];
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    const int64_t row = row0 + threadIdx.x;
    const SubDev S = P.subs[P.cpl_sub[row]];
    const int dir = P.cpl_dir[row];
    int c[3], cn[3];
    loc_coords(S, P.cpl_loc[row], c);
    for (int t = 0; t < 9; ++t) {
      double v = 0.0;
      if (rk[threadIdx.x * 9 + t] >= 0) {
        plane_nbr(S, g.dim, c, dir, t, cn);
        v = kloc(S, g, rho, P.khat, c, cn);
      }
      cf[threadIdx.x * 9 + t] = v;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nr * 9; e += CPL_ROWS) coef[e0 + e] = cf[e];
  // the in-plane entries, through the same LDS
  const int64_t f0 = row0 * 5;
  __syncthreads();
  for (int e = threadIdx.x; e < nr * 5; e += CPL_ROWS) rk[e] = P.ipl_rank[f0 + e];
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    const int64_t row = row0 + threadIdx.x;
    const SubDev S = P.subs[P.cpl_sub[row]];
    int c[3], cn[3];
    loc_coords(S, P.cpl_loc[row], c);
    for (int t = 0; t < 5; ++t) {
      double v = 0.0;
      if (rk[threadIdx.x * 5 + t] >= 0) {
        cn[0] = c[0] + kInPlaneLower[t][0];
        cn[1] = c[1] + (g.dim == 3 ? kInPlaneLower[t][1] : 0);
        cn[2] = c[2];
        v = kloc(S, g, rho, P.khat, c, cn);
      }
      cf[threadIdx.x * 5 + t] = v;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nr * 5; e += CPL_ROWS) icoef[f0 + e] = cf[e];
}

// ---------------------------------------------------------------------------
// local matrices: dense diagonal blocks of K_II / K_rr (entries within a block)
//
// Only the lower triangles are formed: k_block_zero_lower clears them (a
// wave per column, lanes along i), then k_block_assemble writes the stencil
// entries with j <= i.  The upper triangles are left as they are: the sweeps
// read only the lower triangle and write both.  The first-plane corner of a
// block coupled to the previous one is left out of both: the Schur coupling
// writes its whole lower triangle, stencil entries included.

typedef int i4v __attribute__((ext_vector_type(4)));

template <typename T>
__global__ __launch_bounds__(256) void k_block_zero_lower(PlanDev P, int setR, T* __restrict__ G) {
  // one workgroup per block
  const int sub = blockIdx.y, k = blockIdx.x;
  const SubDev S = P.subs[sub];
  if (k >= (setR ? S.nbR : S.nbI)) return;
  const BlockDev B = P.blocks[(setR ? S.bR_off : S.bI_off) + k];
  T* Gb = G + B.G_off;
  // wave w clears the columns j = w, w + 4, ...: from the start of the
  // 16-row group holding row j to the end of the column, in 16-byte stores
  // of whole 64/128-byte lines.  Columns start on 16-entry boundaries and
  // ld is a multiple of 16, so the stores stay inside the column; the
  // entries above row j they also clear are upper-triangle entries or
  // padding, which nothing reads before the sweep writes them.
  // The first-plane corner of a block coupled to the previous one is written
  // whole (lower triangle) by the Schur coupling, A_kk included: skipped.
  constexpr int per = 16 / (int)sizeof(T);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int fc = B.cf_off >= 0 ? B.first_n : 0;
  for (int j = wave; j < B.size; j += 4) {
    const int start = j < fc ? fc : j;
    if (start >= B.size) continue;
    const int i0 = start & ~15;
    i4v* col = reinterpret_cast<i4v*>(Gb + (int64_t)B.ld * j + i0);
    const int nv = (B.size - i0 + per - 1) / per;
    for (int q = lane; q < nv; q += 64) col[q] = i4v{0, 0, 0, 0};
  }
}

template <typename T>
__global__ void k_block_assemble(PlanDev P, Geo g, const double* __restrict__ rho, int setR,
                                 T* __restrict__ G) {
  const int sub = blockIdx.y;
  const SubDev S = P.subs[sub];
  const int nset = setR ? S.n_r : S.n_I;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nset) return;
  const int32_t* sl = set_loc_of(P, S, setR);
  const int32_t* ls = loc_set_of(P, S, setR);
  const int nb = setR ? S.nbR : S.nbI;
  const BlockDev* blk = P.blocks + (setR ? S.bR_off : S.bI_off);
  const int pa = g.dim - 1;
  int c[3];
  loc_coords(S, sl[i], c);
  int k = 0;
  while (k < nb && !(c[pa] >= blk[k].plane_lo && c[pa] < blk[k].plane_hi)) ++k;
  if (k == nb) return;
  const BlockDev B = blk[k];
  // a first-plane node of a coupled block: its neighbours of lower rank in
  // the block lie in the same plane, the corner the Schur coupling writes
  if (B.cf_off >= 0 && i - B.start < B.first_n) return;
  const int zr = g.dim == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int cn[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
        int ln = loc_index(S, cn);
        if (ln < 0) continue;
        int j = ls[ln];
        if (j < 0) continue;
        if (cn[pa] < B.plane_lo || cn[pa] >= B.plane_hi || j > i) continue;
        // the first-plane corner of a coupled block: the Schur coupling's
        if (B.cf_off >= 0 && i - B.start < B.first_n && j - B.start < B.first_n) continue;
        G[B.G_off + (int64_t)(i - B.start) + (int64_t)B.ld * (j - B.start)] =
            (T)kloc(S, g, rho, P.khat, c, cn);
      }
}

// Block Schur update S_k = A_kk - A_{k,k-1} G_{k-1} A_{k-1,k} of the
// block-tridiagonal factorization, restricted to the first-plane rows and
// columns of block k (the only ones the plane coupling reaches), on and
// below the diagonal.  This corner is not assembled in the matrix: A_kk's
// entries there (the in-plane stencil) come from the coupling table.  One workgroup per (subdomain, chunk of SC_COLS
// columns j'):
//   W[l', j'] = sum_m Gs[l', m] A[m, j']  over the last plane of block k-1,
//   S_k[i', j'] += sum_l A[i', l] W[l, j'],
// with Gs = -G_{k-1} the swept block, so the sum adds -A G A.  W stays in LDS.
constexpr int SC_COLS = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_schur_couple(PlanDev P, int setR, int k, T* __restrict__ G, int nch) {
  extern __shared__ char smem_raw[];
  T(*W)[SC_COLS + 1] = reinterpret_cast<T(*)[SC_COLS + 1]>(smem_raw);  // [last_n][cols]
  __shared__ int crk[SC_COLS][9];
  __shared__ double ccf[SC_COLS][9];
  // XCD-aware order: workgroups go round-robin over the 8 XCDs, so the nch
  // chunks of one subdomain (which gather the same G_{k-1}) are given
  // consecutive logical indices on one XCD and share its L2
  const int nblk = gridDim.x, lin = blockIdx.x;
  const int logical = (lin % 8) * (nblk / 8) + lin / 8;
  if (logical >= nch * P.n_sub) return;
  const int sub = logical / nch, chunk = logical % nch;
  const SubDev S = P.subs[sub];
  const int nb = setR ? S.nbR : S.nbI;
  if (k >= nb || k == 0) return;
  const BlockDev* blk = P.blocks + (setR ? S.bR_off : S.bI_off);
  const BlockDev Bp = blk[k - 1], B = blk[k];
  if (B.cf_off < 0) return;
  const int c0 = chunk * SC_COLS;
  if (c0 >= B.first_n) return;
  const int cols = min(SC_COLS, B.first_n - c0);
  __shared__ int mlo, mhi;
  if constexpr (sizeof(T) == 4) {
    if (threadIdx.x == 0) {
      mlo = INT32_MAX;
      mhi = -1;
    }
    __syncthreads();
  }
  // coupling rows of this chunk's columns (first-plane rows of block k), and
  // (FP32) the range of G_{k-1} columns their taps reach
  for (int e = threadIdx.x; e < SC_COLS * 9; e += blockDim.x) {
    const int c = e / 9, t = e % 9;
    const int64_t row = B.cf_off + c0 + c;
    const int m = c < cols ? P.cpl_rank[row * 9 + t] : -1;
    crk[c][t] = m >= 0 ? m - Bp.start : -1;
    ccf[c][t] = m >= 0 ? P.cpl_coef[row * 9 + t] : 0.0;
    if (sizeof(T) == 4 && m >= 0) {
      atomicMin(&mlo, m - Bp.start);
      atomicMax(&mhi, m - Bp.start);
    }
  }
  __syncthreads();
  const T* Gr = G + Bp.G_off + (Bp.size - Bp.last_n);
  if constexpr (sizeof(T) == 4) {
    // FP32 blocks: W = Gs[:, lo..hi] A_c on MFMA, A_c the chunk's coupling
    // columns over the taps' range (nine nonzeros per column, formed in the
    // B operand from the tap table), so each element of Gs in the range is
    // loaded once, 16 consecutive rows per load (measured: the gathers
    // below are the slower form in FP32, the faster one in FP64)
    typedef typename Mfma<T>::acc_t acc_t;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kq = lane >> 4, rr = lane & 15;
    const int lo = mlo, hi = mhi;
    const int ks = hi >= lo ? (hi - lo + 4) >> 2 : 0;
    int tm[9];
    T tc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      tm[t] = crk[rr][t];
      tc[t] = (T)ccf[rr][t];
    }
    const int nrt = (Bp.last_n + 15) >> 4;
    for (int rt = wave; rt < nrt; rt += 4) {
      const int row = rt * 16 + rr;
      acc_t acc = acc_t{0, 0, 0, 0};
      for (int s0 = 0; s0 < ks; s0 += 8) {
        T av[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int m = lo + 4 * (s0 + u) + kq;
          av[u] = (s0 + u < ks && row < Bp.last_n && m <= hi) ? Gr[row + (int64_t)Bp.ld * m] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (s0 + u >= ks) break;
          const int m = lo + 4 * (s0 + u) + kq;
          T b = (T)0;
#pragma unroll
          for (int t = 0; t < 9; ++t) b = tm[t] == m ? tc[t] : b;
          acc = Mfma<T>::mac(av[u], b, acc);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = rt * 16 + Mfma<T>::row(kq, r);
        if (lr < Bp.last_n) W[lr][rr] = acc[r];
      }
    }
  } else {
    // FP64 blocks: W[l'][c] = sum_t Gs[l', m_t] a_t, four columns' gathers
    // in flight at a time
    for (int lp = threadIdx.x; lp < Bp.last_n; lp += blockDim.x) {
      for (int cb = 0; cb < SC_COLS; cb += 4) {
        T gv[4][9];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc)
#pragma unroll
          for (int t = 0; t < 9; ++t) {
            const int m = crk[cb + cc][t];
            gv[cc][t] = m >= 0 ? Gr[lp + (int64_t)Bp.ld * m] : (T)0;
          }
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          double acc = 0.0;
#pragma unroll
          for (int t = 0; t < 9; ++t) acc += (double)gv[cc][t] * ccf[cb + cc][t];
          W[lp][cb + cc] = (T)acc;
        }
      }
    }
  }
  __syncthreads();
  // S_k[i'][c] += sum_t A[i', l_t] W[l_t][c], all of the row's columns at
  // once, on and below the diagonal only (the sweep of block k reads only
  // its lower triangle): rows i' >= c0 + c
  const int base = Bp.start + Bp.size - Bp.last_n;
  T* Gk = G + B.G_off + (int64_t)B.ld * c0;
  for (int ip = c0 + threadIdx.x; ip < B.first_n; ip += blockDim.x) {
    const int64_t row = B.cf_off + ip;
    double a[9];
    int l[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int r = P.cpl_rank[row * 9 + t];
      a[t] = r >= 0 ? P.cpl_coef[row * 9 + t] : 0.0;
      l[t] = r >= 0 ? r - base : 0;
    }
    const int cl = min(cols, ip - c0 + 1);  // columns c < cl lie on or below the diagonal
    // A_kk on this row within the chunk: its in-plane stencil entries of
    // rank at most its own (the corner is not assembled in the matrix)
    int jr[5];
    T jv[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      jr[q] = P.ipl_rank[row * 5 + q];
      jv[q] = (T)P.ipl_coef[row * 5 + q];
    }
    T old[SC_COLS];
#pragma unroll
    for (int c = 0; c < SC_COLS; ++c) {
      T v = (T)0;
#pragma unroll
      for (int q = 0; q < 5; ++q) v = jr[q] == c0 + c ? jv[q] : v;
      old[c] = v;
    }
#pragma unroll
    for (int c = 0; c < SC_COLS; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) acc += a[t] * (double)W[l[t]][c];
      if (c < cl) Gk[ip + (int64_t)B.ld * c] = old[c] + (T)acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Batched symmetric sweep (Gauss-Jordan on an SPD matrix, in place).
// Sweeping pivot set Q of a symmetric matrix M replaces M_QQ by -M_QQ^{-1},
// M_iQ by M_iQ M_QQ^{-1} and M_ij by M_ij - M_iQ M_QQ^{-1} M_Qj.  A full
// sweep gives -M^{-1}; sweeping the first p pivots of a front gives
// -F_PP^{-1}, F_BP F_PP^{-1} and the Schur complement F_BB - F_BP F_PP^{-1} F_PB.
// Pivots are swept in panels of SWEEP_NB: k_sweep_panel (one workgroup per
// matrix) writes back the previous panel, inverts the new pivot block in LDS
// and forms CD = M_{:,Q} D^{-1}; k_sweep_update applies the rank-NB update
// to every entry outside the panel on MFMA.

// Scratch per problem and panel parity: CD (n x NB, ld n) then Dinv (NB x NB).
template <typename T>
__device__ __forceinline__ T* sweep_slot(T* scratch, int64_t scr_stride, int prob, int j0) {
  return scratch + prob * scr_stride + ((j0 / SWEEP_NB) & 1) * (scr_stride / 2);
}

// Wave-uniform broadcast of lane l's value (l a compile-time or uniform index).
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

// 1/x by the hardware reciprocal refined with two Newton steps
// (r <- r + r (1 - x r)), accurate to the last bit or one ulp.
__device__ __forceinline__ double recip_f64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Lane l of a wave reads lane 16 G + (l mod 16): row G of 16 lanes copied to
// all four (two register swaps of gfx950: v_permlane16_swap exchanges the odd
// rows of its first operand with the even rows of its second, and
// v_permlane32_swap the upper half of the first with the lower half of the
// second).  No LDS traffic.
template <int G>
__device__ __forceinline__ int rowgroup_bcast_i32(int x) {
  const auto a = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // rows (x0 x0 x2 x2), (x1 x1 x3 x3)
  const int h = (G & 1) ? (int)a[1] : (int)a[0];
  const auto b = __builtin_amdgcn_permlane32_swap(h, h, false, false);  // rows (h0 h1 h0 h1), (h2 h3 h2 h3)
  return (G & 2) ? (int)b[1] : (int)b[0];
}

template <int G>
__device__ __forceinline__ double rowgroup_bcast_f64(double x) {
  return __hiloint2double(rowgroup_bcast_i32<G>(__double2hiint(x)), rowgroup_bcast_i32<G>(__double2loint(x)));
}

// Lane l of a wave reads lane Q of its own row of 16 lanes (DPP row
// broadcast; every lane is written, so the destination needs no fill)
template <int Q>
__device__ __forceinline__ double row_bcast_f64(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x150 + Q, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x150 + Q, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Lane l of a wave reads lane l ^ M (M = 1, 2, 4, 8, 16 or 32), the value
// __shfl_xor returns, without LDS traffic: DPP within rows of 16 lanes (xor 1
// and 2 by quad permutes, 4 by the half-row mirror followed by a quad
// reversal, 8 by a row rotation), register swaps across rows (xor 16 and 32).
template <int M>
__device__ __forceinline__ int xor_lane_i32(int x) {
  static_assert(M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32, "lane xor mask");
  if constexpr (M == 1) {
    return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
  } else if constexpr (M == 2) {
    return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
  } else if constexpr (M == 4) {
    const int h = __builtin_amdgcn_mov_dpp(x, 0x141, 0xf, 0xf, false);  // i -> 7 - i in each 8
    return __builtin_amdgcn_mov_dpp(h, 0x1B, 0xf, 0xf, false);           // quad_perm [3,2,1,0]
  } else if constexpr (M == 8) {
    return __builtin_amdgcn_mov_dpp(x, 0x128, 0xf, 0xf, false);  // row_ror:8
  } else if constexpr (M == 16) {
    const auto a = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // rows (x0 x0 x2 x2), (x1 x1 x3 x3)
    return (threadIdx.x & 16) ? (int)a[0] : (int)a[1];
  } else {
    const auto a = __builtin_amdgcn_permlane32_swap(x, x, false, false);  // rows (x0 x1 x0 x1), (x2 x3 x2 x3)
    return (threadIdx.x & 32) ? (int)a[0] : (int)a[1];
  }
}

template <int M>
__device__ __forceinline__ double xor_lane_f64(double x) {
  return __hiloint2double(xor_lane_i32<M>(__double2hiint(x)), xor_lane_i32<M>(__double2loint(x)));
}

// One pivot step of the 16x16 sweep below, as the rank-1 form
// X <- X0 - u v^T  (X0: X with row and column q zeroed; u = column q with -1
// at q; v = row q / d with -1/d at q).
template <int Q>
__device__ __forceinline__ void sweep16_step(double m[4], int jb, int kq, int rr, bool& bad) {
  const double dq = readlane_f64(m[Q & 3], (Q >> 2) * 16 + Q);     // X[Q][Q]
  const double rowq = rowgroup_bcast_f64<(Q >> 2)>(m[Q & 3]);     // X[Q][rr]
  bad |= (Q < jb) & !(dq > 0.0);
  const double inv = recip_f64(dq > 0.0 ? dq : 1.0);
  const bool qcol = rr == Q;
  const double v = qcol ? -inv : rowq * inv;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double colq = row_bcast_f64<Q>(m[t]);                   // X[4kq+t][Q]
    const bool qrow = t == (Q & 3) && kq == (Q >> 2);
    const double u = qrow ? -1.0 : colq;
    const double mz = (qrow || qcol) ? 0.0 : m[t];
    m[t] = fma(-u, v, mz);
  }
}

template <int... Qs>
__device__ __forceinline__ void sweep16_all(double m[4], int jb, int kq, int rr, bool& bad,
                                            std::integer_sequence<int, Qs...>) {
  (sweep16_step<Qs>(m, jb, kq, rr, bad), ...);
}

// A wave holds a 16x16 symmetric block X as m[t] = X[4 kq + t][rr]
// (kq = lane/16, rr = lane%16).  Sweeps pivots 0..15 (pivots >= jb are
// identity padding).  Per pivot q: X[q][q] comes by a wave-uniform
// broadcast, the pivot column X[4 kq + t][q] from lane q of the lane's own
// row of 16 (DPP), the pivot row X[q][rr] from row q / 4 of the wave by two
// register swaps (no LDS traffic).  On return m holds the swept block
// (-X^{-1} on the pivots).  Returns true on a pivot <= 0.
__device__ __forceinline__ bool quad_sweep16(double m[4], int jb, int lane) {
  bool bad = false;
  sweep16_all(m, jb, lane >> 4, lane & 15, bad, std::make_integer_sequence<int, 16>{});
  return bad;
}

// Sweeps a 32x32 symmetric block held in LDS at D (row i at D + i*ld; jb
// used pivots, the rest padded with the identity) by one wave, as two 16x16
// pivot sweeps and 16x16 MFMA products:
//   N11 = -D11^{-1};  T = D21 D11^{-1};  S = D22 - T D21^T;  N22 = -S^{-1};
//   V = N22 T;  result [N11 + T^T V, -V^T; -V, N22]  (= -D^{-1}).
// T points to 32 x 33 doubles of LDS scratch.  No workgroup barrier: LDS
// accesses of one wave are ordered.  Returns true on a pivot <= 0.
__device__ bool sweep32_fast(double* D, int ld, double* T, int jb, int lane) {
  typedef Mfma<double>::acc_t acc_t;
  const int kq = lane >> 4, rr = lane & 15;
  auto at = [&](int i, int j) -> double& { return D[i * ld + j]; };
  auto tt = [&](int i, int j) -> double& { return T[i * 33 + j]; };
  bool bad = false;
  double m[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) m[t] = at(4 * kq + t, rr);
  bad |= quad_sweep16(m, min(jb, 16), lane);
#pragma unroll
  for (int t = 0; t < 4; ++t) at(4 * kq + t, rr) = m[t];  // N11
  __builtin_amdgcn_wave_barrier();
  // T = D21 (-N11)
  acc_t c = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) c = Mfma<double>::mac(at(16 + rr, 4 * s4 + kq), -at(4 * s4 + kq, rr), c);
#pragma unroll
  for (int r = 0; r < 4; ++r) tt(Mfma<double>::row(kq, r), rr) = c[r];
  __builtin_amdgcn_wave_barrier();
  // S = D22 - T D21^T, written over D22
  c = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) c = Mfma<double>::mac(tt(rr, 4 * s4 + kq), at(16 + rr, 4 * s4 + kq), c);
  double sv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) sv[r] = at(16 + Mfma<double>::row(kq, r), 16 + rr) - c[r];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < 4; ++r) at(16 + Mfma<double>::row(kq, r), 16 + rr) = sv[r];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int t = 0; t < 4; ++t) m[t] = at(16 + 4 * kq + t, 16 + rr);
  bad |= quad_sweep16(m, max(jb - 16, 0), lane);
#pragma unroll
  for (int t = 0; t < 4; ++t) at(16 + 4 * kq + t, 16 + rr) = m[t];  // N22
  __builtin_amdgcn_wave_barrier();
  // V = N22 T, into T's rows 16..31
  c = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) c = Mfma<double>::mac(at(16 + rr, 16 + 4 * s4 + kq), tt(4 * s4 + kq, rr), c);
#pragma unroll
  for (int r = 0; r < 4; ++r) tt(16 + Mfma<double>::row(kq, r), rr) = c[r];
  __builtin_amdgcn_wave_barrier();
  // D11 = N11 + T^T V;  D21 = -V, D12 = -V^T
  acc_t w = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) w = Mfma<double>::mac(tt(4 * s4 + kq, rr), tt(16 + 4 * s4 + kq, rr), w);
  double n11[4], vv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = Mfma<double>::row(kq, r);
    n11[r] = at(i, rr);
    vv[r] = tt(16 + i, rr);
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = Mfma<double>::row(kq, r);
    at(i, rr) = n11[r] + w[r];
    at(16 + i, rr) = -vv[r];
    at(rr, 16 + i) = -vv[r];
  }
  __builtin_amdgcn_wave_barrier();
  return bad;
}

// Sweeps a 32x32 block (jb <= 32 used entries) held in LDS at D (row i at
// D + i*ld) by one wave, in registers: lane l keeps column l%32, rows
// 16*(l/32) .. +15.  Each pivot step takes the pivot row and column through
// cross-lane shuffles; no barriers.  Entries beyond jb are padded with the
// identity.  On return the block holds -B^{-1}.  Returns true on a pivot <= 0.
__device__ __forceinline__ bool wave_sweep32(double* D, int ld, int jb, int lane) {
  const int j = lane & 31, h = lane >> 5;
  double m[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int i = h * 16 + t;
    m[t] = (i < jb && j < jb) ? D[i * ld + j] : (i == j ? 1.0 : 0.0);
  }
  bool bad = false;
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    const int qh = q >> 4, qt = q & 15;
    const double rowq = __shfl(m[qt], j + 32 * qh, 64);  // B[q][j]
    double dq = __shfl(m[qt], q + 32 * qh, 64);          // B[q][q]
    if (!(dq > 0.0)) {
      bad = true;
      dq = 1.0;
    }
    const double inv = 1.0 / dq;
    double colq[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) colq[t] = __shfl(m[t], q + 32 * h, 64);  // B[16h+t][q]
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int i = h * 16 + t;
      double v;
      if (i == q && j == q) v = -inv;
      else if (i == q) v = rowq * inv;
      else if (j == q) v = colq[t] * inv;
      else v = m[t] - colq[t] * rowq * inv;
      m[t] = v;
    }
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) D[(h * 16 + t) * ld + j] = m[t];
  return bad;
}

// Sweeps the full SWEEP_NB x SWEEP_NB pivot block in LDS (entries beyond jb
// padded with the identity): the first 32 pivots by one wave, the Schur
// complement of the other 32 by GEMM-like updates over the workgroup, then
// its 32 pivots by one wave, then the first block's correction.  Sweeping
// two pivot sets in turn equals sweeping their union.  Every thread of the
// workgroup must call it.  tmp holds 32 x 33 doubles.
__device__ bool block_sweep(double (*D)[SWEEP_NB + 1], double (*tmp)[33], int jb, int tid, int nthreads) {
  constexpr int ld = SWEEP_NB + 1;
  bool bad = false;
  if (tid < 64) bad |= sweep32_fast(&D[0][0], ld, &tmp[0][0], min(jb, 32), tid);
  __syncthreads();
  if (jb > 32) {
    // T21 = D21 D11^{-1} = -D21 * (swept D11)
    for (int idx = tid; idx < 32 * 32; idx += nthreads) {
      const int i = idx / 32, j = idx % 32;
      double s = 0.0;
      for (int k = 0; k < 32; ++k) s -= D[32 + i][k] * D[k][j];
      tmp[i][j] = s;
    }
    __syncthreads();
    // D22 -= T21 D12 (D12 = D21^T, still unchanged)
    for (int idx = tid; idx < 32 * 32; idx += nthreads) {
      const int i = idx / 32, j = idx % 32;
      double s = 0.0;
      for (int k = 0; k < 32; ++k) s += tmp[i][k] * D[32 + j][k];
      D[32 + i][32 + j] -= s;
    }
    __syncthreads();
    for (int idx = tid; idx < 32 * 32; idx += nthreads) {
      const int i = idx / 32, j = idx % 32;
      D[32 + i][j] = tmp[i][j];
      D[j][32 + i] = tmp[i][j];
    }
    __syncthreads();
    if (tid < 64) bad |= wave_sweep32(&D[32][32], ld, jb - 32, tid);
    __syncthreads();
    // U = D12 S^{-1} = -D12 * (swept D22)
    for (int idx = tid; idx < 32 * 32; idx += nthreads) {
      const int i = idx / 32, j = idx % 32;
      double s = 0.0;
      for (int k = 0; k < 32; ++k) s -= D[i][32 + k] * D[32 + k][32 + j];
      tmp[i][j] = s;
    }
    __syncthreads();
    // D11 -= U D21
    for (int idx = tid; idx < 32 * 32; idx += nthreads) {
      const int i = idx / 32, j = idx % 32;
      double s = 0.0;
      for (int k = 0; k < 32; ++k) s += tmp[i][k] * D[32 + k][j];
      D[i][j] -= s;
    }
    __syncthreads();
    for (int idx = tid; idx < 32 * 32; idx += nthreads) {
      const int i = idx / 32, j = idx % 32;
      D[i][32 + j] = tmp[i][j];
      D[32 + j][i] = tmp[i][j];
    }
    __syncthreads();
  }
  return bad;
}

// One workgroup per (chunk of SWEEP_ROWS rows, matrix).  Only the lower
// triangle is kept current during the sweep (the update is symmetric); a
// final pass mirrors it.
//  1. writes back the previous panel for its rows, into the lower triangle;
//  2. loads the new pivot block and sweeps it in LDS (every workgroup of the
//     matrix does this redundantly; it is NB x NB, one barrier per pivot);
//  3. stages its rows of the column panel in LDS and forms CD = C D^{-1}.
// Rows of the previous panel read their column-panel values from the
// previous scratch slot, so no workgroup depends on another's writeback.
constexpr int SWEEP_ROWS = 256;

template <typename T>
__global__ __launch_bounds__(256) void k_sweep_panel(const SweepDesc* __restrict__ desc, T* pool,
                                                     int j0, int prev_j0, T* scratch,
                                                     int64_t scr_stride, int* status,
                                                     int status_code) {
  __shared__ double D[1][SWEEP_NB][SWEEP_NB + 1];
  __shared__ double tmp[32][33];
  extern __shared__ char smem_raw[];
  T(*Cl)[SWEEP_NB + 1] = reinterpret_cast<T(*)[SWEEP_NB + 1]>(smem_raw);  // [chunk rows][NB+1]
  const SweepDesc d = desc[blockIdx.y];
  const int n = d.n, p = d.p, ld = d.ld;
  const int r0 = blockIdx.x * SWEEP_ROWS;
  if (r0 >= n) return;
  const int rows = min(SWEEP_ROWS, n - r0);
  T* A = pool + d.off;
  const int tid = threadIdx.x;
  const bool have_prev = prev_j0 >= 0 && prev_j0 < p;
  const T* CDp = have_prev ? sweep_slot(scratch, scr_stride, blockIdx.y, prev_j0) : nullptr;
  const int pb = have_prev ? min(SWEEP_NB, p - prev_j0) : 0;
  // Each phase issues PU independent loads per thread before it stores any of
  // them, so the latency of one HBM round trip is paid per PU elements.
  constexpr int NT = 256, PU = 8;
  if (have_prev) {
    const T* Dip = CDp + (int64_t)n * SWEEP_NB;
    const int tot = rows * pb;
    for (int base = tid; base < tot; base += NT * PU) {
      T v[PU];
      int64_t dst[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int idx = base + u * NT;
        dst[u] = -1;
        if (idx < tot) {
          const int i = r0 + idx % rows, q = idx / rows;
          const int col = prev_j0 + q;
          if (i >= prev_j0 && i < prev_j0 + pb) {
            v[u] = -Dip[(i - prev_j0) + SWEEP_NB * q];
            dst[u] = i + (int64_t)ld * col;
          } else {
            v[u] = CDp[i + (int64_t)n * q];
            dst[u] = i > col ? i + (int64_t)ld * col : col + (int64_t)ld * i;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < PU; ++u)
        if (dst[u] >= 0) A[dst[u]] = v[u];
    }
  }
  if (j0 < 0 || j0 >= p) return;
  const int jb = min(SWEEP_NB, p - j0);
  {
    double dv[SWEEP_NB * SWEEP_NB / NT];
#pragma unroll
    for (int u = 0; u < SWEEP_NB * SWEEP_NB / NT; ++u) {
      const int idx = tid + u * NT;
      const int i = idx % SWEEP_NB, j = idx / SWEEP_NB;
      const int gi = max(i, j), gj = min(i, j);
      dv[u] = (i < jb && j < jb) ? (double)A[(j0 + gi) + (int64_t)ld * (j0 + gj)] : (i == j ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < SWEEP_NB * SWEEP_NB / NT; ++u) {
      const int idx = tid + u * NT;
      D[0][idx % SWEEP_NB][idx / SWEEP_NB] = dv[u];
    }
  }
  // stage this chunk's rows of the column panel (rows above the panel from
  // the lower-triangle mirror, previous-panel rows from its scratch slot)
  const bool above = r0 + rows <= j0;  // whole chunk above the panel: read the row panel along t
  {
    const int tot = rows * jb;
    for (int base = tid; base < tot; base += NT * PU) {
      T v[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int idx = base + u * NT;
        v[u] = 0;
        if (idx < tot) {
          const int t = above ? idx % jb : idx / rows, r = above ? idx / jb : idx % rows;
          const int i = r0 + r;
          if (have_prev && i >= prev_j0 && i < prev_j0 + pb) v[u] = CDp[(j0 + t) + (int64_t)n * (i - prev_j0)];
          else if (i < j0) v[u] = A[(j0 + t) + (int64_t)ld * i];
          else if (i >= j0 + jb) v[u] = A[i + (int64_t)ld * (j0 + t)];
        }
      }
#pragma unroll
      for (int u = 0; u < PU; ++u) {
        const int idx = base + u * NT;
        if (idx < tot) {
          const int t = above ? idx % jb : idx / rows, r = above ? idx / jb : idx % rows;
          Cl[r][t] = v[u];
        }
      }
    }
  }
  __syncthreads();
  const int cur = 0;
  if (block_sweep(D[0], tmp, jb, tid, blockDim.x)) atomicMax(status, status_code);
  // D[cur] holds -D^{-1}
  T* CD = sweep_slot(scratch, scr_stride, blockIdx.y, j0);
  T* Dinv = CD + (int64_t)n * SWEEP_NB;
  if (blockIdx.x == 0)
    for (int idx = tid; idx < jb * jb; idx += blockDim.x) {
      const int i = idx % jb, j = idx / jb;
      Dinv[i + SWEEP_NB * j] = (T)(-D[cur][i][j]);
    }
  // CD = C D^{-1} on MFMA: each wave takes 16-row tiles of the chunk and
  // computes CD^T[q][r] = sum_t Dinv[q][t] C[r][t] (D is symmetric), so the
  // lanes run along the rows and the stores are coalesced.
  {
    typedef typename Mfma<T>::acc_t acc_t;
    const int wave = tid >> 6, lane = tid & 63;
    const int kq = lane >> 4, rr = lane & 15;
    const int rtiles = (rows + 15) / 16;
    for (int rt = wave; rt < rtiles; rt += blockDim.x >> 6) {
      constexpr int QB = SWEEP_NB / 16;
      acc_t acc[QB];
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) acc[qb] = acc_t{0, 0, 0, 0};
      const int r = rt * 16 + rr;
#pragma unroll
      for (int ks = 0; ks < SWEEP_NB / 4; ++ks) {
        const int t = ks * 4 + kq;
        const T b = (r < rows && t < jb) ? Cl[r][t] : (T)0;
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
          const int q = qb * 16 + rr;
          const T a = (q < jb && t < jb) ? (T)(-D[cur][q][t]) : (T)0;
          acc[qb] = Mfma<T>::mac(a, b, acc[qb]);
        }
      }
#pragma unroll
      for (int qb = 0; qb < QB; ++qb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int q = qb * 16 + Mfma<T>::row(kq, e);
          const int i = r0 + rt * 16 + rr;
          if (q < jb && rt * 16 + rr < rows && !(i >= j0 && i < j0 + jb)) CD[i + (int64_t)n * q] = acc[qb][e];
        }
    }
  }
}

// Rank-NB update of the lower triangle outside the panel:
// A_ij -= CD_i . C_j for i >= j (tiles on or below the diagonal).  C_j comes
// from the lower triangle: the column panel below it, its mirror (the row
// panel) above it.  The MFMA takes C as its A operand and CD as its B
// operand, so each lane's output runs along i and the stores are coalesced.
template <typename T>
__global__ __launch_bounds__(256) void k_sweep_update(const SweepDesc* __restrict__ desc, T* pool,
                                                      int j0, const T* __restrict__ scratch,
                                                      int64_t scr_stride, int ntri, int nprob) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T As[SWEEP_NB][TILE + PAD];  // CD rows i
  __shared__ T Bs[SWEEP_NB][TILE + PAD];  // C rows j
  const int64_t nblk = gridDim.x;
  const int64_t glin = blockIdx.x;
  const int64_t logical = (glin % 8) * (nblk / 8) + glin / 8;  // XCD-aware, as in k_gemm
  if (logical >= (int64_t)nprob * ntri) return;
  const int prob = (int)(logical / ntri);
  const SweepDesc d = desc[prob];
  const int n = d.n, p = d.p, ld = d.ld;
  if (j0 >= p) return;
  const int jb = min(SWEEP_NB, p - j0);
  // linear index -> lower-triangular tile (ti >= tj)
  const int lin = (int)(logical % ntri);
  int ti = (int)((sqrt(8.0 * lin + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= lin) ++ti;
  while (ti * (ti + 1) / 2 > lin) --ti;
  const int tj = lin - ti * (ti + 1) / 2;
  const int i0 = ti * TILE, c0 = tj * TILE;
  if (i0 >= n || c0 >= n) return;
  T* A = pool + d.off;
  const T* CD = sweep_slot(const_cast<T*>(scratch), scr_stride, prob, j0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < TILE * SWEEP_NB; idx += 256) {
    const int r = idx % TILE, q = idx / TILE;
    const int i = i0 + r;
    T a = 0;
    if (q < jb && i < n && !(i >= j0 && i < j0 + jb)) a = CD[i + (int64_t)n * q];
    As[q][r] = a;
  }
  for (int idx = tid; idx < TILE * SWEEP_NB; idx += 256) {
    int r, q;
    if (c0 + TILE <= j0) {  // whole tile above the panel: read the row panel, coalesced along q
      q = idx % SWEEP_NB;
      r = idx / SWEEP_NB;
    } else {
      r = idx % TILE;
      q = idx / TILE;
    }
    const int j = c0 + r;
    T b = 0;
    if (q < jb && j < n) {
      if (j < j0) b = A[(j0 + q) + (int64_t)ld * j];
      else if (j >= j0 + jb) b = A[j + (int64_t)ld * (j0 + q)];
    }
    Bs[q][r] = b;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  const int wi = (wave & 1) * 32, wj = (wave >> 1) * 32;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  const int kq = lane >> 4, rr = lane & 15;
  const int ksteps = (jb + 3) / 4;
  for (int ks = 0; ks < ksteps; ++ks) {
    const int kk = ks * 4 + kq;
    T av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = As[kk][wi + a * 16 + rr];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = Bs[kk][wj + b * 16 + rr];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::mac(bv[b], av[a], acc[a][b]);
  }
  // read every old value of the wave's 32x32 block first, then write
  T old[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = c0 + wj + b * 16 + Mfma<T>::row(kq, r);
        const int i = i0 + wi + a * 16 + rr;
        const bool on = i < n && j <= i && !(i >= j0 && i < j0 + jb) && !(j >= j0 && j < j0 + jb);
        old[a][b][r] = on ? A[i + (int64_t)ld * j] : (T)0;
      }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = c0 + wj + b * 16 + Mfma<T>::row(kq, r);
        const int i = i0 + wi + a * 16 + rr;
        if (i < n && j <= i && !(i >= j0 && i < j0 + jb) && !(j >= j0 && j < j0 + jb))
          A[i + (int64_t)ld * j] = old[a][b][r] - acc[a][b][r];
      }
}

// Mirrors the lower triangle of the pivot block (the leading p x p) into its
// upper one after a sweep, by 32x32 tiles through LDS so both the read and
// the write run along columns.  Outside the pivot block only the lower
// triangle is kept: a front's border rows and update block are read there
// (the products with -F_PP^{-1} read whole pivot columns).
template <typename T>
__global__ void k_symmetrize(const SweepDesc* __restrict__ desc, T* pool, int ntri) {
  __shared__ T tile[32][33];
  const SweepDesc d = desc[blockIdx.y];
  T* A = pool + d.off;
  const int nt = (d.p + 31) / 32;
  for (int lin = blockIdx.x; lin < nt * (nt + 1) / 2; lin += gridDim.x) {
    int ti = (int)((sqrt(8.0 * lin + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= lin) ++ti;
    while (ti * (ti + 1) / 2 > lin) --ti;
    const int tj = lin - ti * (ti + 1) / 2;  // tile (ti, tj) of the lower triangle, ti >= tj
    __syncthreads();
    for (int idx = threadIdx.x; idx < 32 * 32; idx += blockDim.x) {
      const int r = idx % 32, c = idx / 32;
      const int i = ti * 32 + r, j = tj * 32 + c;
      tile[c][r] = (i < d.p && j < d.p) ? A[i + (int64_t)d.ld * j] : (T)0;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 32 * 32; idx += blockDim.x) {
      const int r = idx % 32, c = idx / 32;   // upper entry (tj*32 + r, ti*32 + c) = lower (ti*32 + c, tj*32 + r)
      const int i = tj * 32 + r, j = ti * 32 + c;
      if (i < d.p && j < d.p && i < j) A[i + (int64_t)d.ld * j] = tile[r][c];
    }
  }
  (void)ntri;
}

// ---------------------------------------------------------------------------
// Register-resident sweep for matrices of at most 16*MT rows: one workgroup
// of RS_WAVES waves per matrix holds its lower triangle as 16x16 MFMA
// accumulator tiles (tile t = wave + RS_WAVES * slot), so the matrix is read
// from HBM once and written once.  Pivots go in panels of 16 (one tile
// column).  Per panel:
//   1. the owners of the panel's tiles stage its column C (n x 16, with the
//      row panel mirrored) and the 16x16 pivot block D in LDS;
//   2. every wave sweeps D in registers (the same arithmetic in each wave,
//      so all hold the same -D^{-1});
//   3. the waves form CD = C D^{-1} on MFMA, one 16-row tile at a time;
//   4. every tile takes the rank-16 update M_ij -= CD_i C_j^T on MFMA, and the
//      panel's own entries become CD (rows or columns in the panel) or
//      -D^{-1} (the pivot block).
// Only the lower triangle is read; both triangles are written.
constexpr int RS_MAX_TILES = kRegSweepMaxRows / 16;  // largest matrix: 304 rows
constexpr int SLAB = kSlab;       // pivots per slab of the large-matrix sweep
// Flops of a slab's trailing update below which its pivot-block sweep of the
// next slab stays on the main stream (about 250 us of update at the 35-37
// TFLOP/s these updates reach; the sweep takes about 100 us).
constexpr double kSlabInlineFlops = 9e9;

template <typename T, int MT, int RS_WAVES>
__global__ __launch_bounds__(RS_WAVES * 64) void k_sweep_reg(const SweepDesc* __restrict__ desc, T* pool,
                                                             int* status, int status_code, int slab_j0,
                                                             int sl = SLAB) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int NTILE = MT * (MT + 1) / 2;
  constexpr int TPW = (NTILE + RS_WAVES - 1) / RS_WAVES;
  __shared__ T Cs[MT * 16][17];     // panel column C (rows of the pivot columns), 0 on the pivot rows
  __shared__ T CDs[MT * 16][17];    // C D^{-1}
  __shared__ double Ds[16][17];     // pivot block before the sweep
  __shared__ double Dw[16][17];     // swept pivot block (-D^{-1})
  __shared__ int tab[NTILE];
  const SweepDesc d = desc[blockIdx.x];
  // slab mode (slab_j0 >= 0): the diagonal block of pivots slab_j0 ..
  // slab_j0 + sl - 1 of the matrix (sl <= 16 MT), swept completely
  const int ld = d.ld;
  const int n = slab_j0 < 0 ? d.n : min(sl, d.p - slab_j0);
  const int p = slab_j0 < 0 ? d.p : n;
  if (slab_j0 >= 0 && n <= 0) return;
  T* A = pool + d.off + (slab_j0 < 0 ? 0 : (int64_t)slab_j0 * (ld + 1));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kq = lane >> 4, rr = lane & 15;
  for (int t = tid; t < NTILE; t += RS_WAVES * 64) {
    int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    tab[t] = (ti << 8) | (t - ti * (ti + 1) / 2);
  }
  __syncthreads();
  const int nt = (n + 15) >> 4;
  // wave-uniform tile coordinates of each slot (ti = -1: no tile)
  int sti[TPW], stj[TPW];
#pragma unroll
  for (int sl = 0; sl < TPW; ++sl) {
    const int t = wave + RS_WAVES * sl;
    const int code = t < NTILE ? __builtin_amdgcn_readfirstlane(tab[t]) : -1;
    sti[sl] = (code >= 0 && (code >> 8) < nt) ? (code >> 8) : -1;
    stj[sl] = code & 255;
  }
  acc_t acc[TPW];
  // load the lower triangle (padding beyond n is 0), branch-free per element
#pragma unroll
  for (int sl = 0; sl < TPW; ++sl) {
    acc[sl] = acc_t{0, 0, 0, 0};
    if (sti[sl] < 0) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * sti[sl] + Mfma<T>::row(kq, r), j = 16 * stj[sl] + rr;
      const int hi = min(max(i, j), n - 1), lo = min(min(i, j), n - 1);
      // uniform base + 32-bit byte offset: no 64-bit address registers
      const T v = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(A) +
                                              (uint32_t)(lo * ld + hi) * (uint32_t)sizeof(T));
      acc[sl][r] = (i < n && j < n) ? v : (T)0;
    }
  }
  bool bad = false;
  const int npan = (p + 15) >> 4;
  for (int tq = 0; tq < npan; ++tq) {
    // an opaque scalar zero added to the slots' tile coordinates: the LDS
    // addresses derived from them are recomputed each panel instead of being
    // hoisted out of the loop and held in registers for every slot
    int oz;
    asm volatile("s_mov_b32 %0, 0" : "=s"(oz));
    const int j0 = 16 * tq, jb = min(16, p - j0);
    __syncthreads();  // the previous panel's readers of Cs / CDs / Dw are done
    // 1. stage C and D from the tiles of tile row / column tq
#pragma unroll
    for (int sl = 0; sl < TPW; ++sl) {
      const int ti = sti[sl] + oz, tj = stj[sl] + oz;
      if (ti < 0) continue;
      if (ti == tq && tj == tq) {  // pivot rows carry no C
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = Mfma<T>::row(kq, r);
          const T v = acc[sl][r];
          if (a < jb && rr < jb) Ds[a][rr] = (double)v;
          Cs[j0 + a][rr] = (a >= jb && rr < jb) ? v : (T)0;
        }
      } else if (tj == tq) {        // column panel, rows 16 ti + a
#pragma unroll
        for (int r = 0; r < 4; ++r) Cs[16 * ti + Mfma<T>::row(kq, r)][rr] = rr < jb ? acc[sl][r] : (T)0;
      } else if (ti == tq) {        // row panel: M[j0 + a][16 tj + b] = C[16 tj + b][a]
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = Mfma<T>::row(kq, r);
          Cs[16 * tj + rr][a] = a < jb ? acc[sl][r] : (T)0;
        }
      }
    }
    __syncthreads();
    // 2. wave 0 sweeps the pivot block
    if (wave == 0) {
      double m[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = 4 * kq + t;
        m[t] = (i < jb && rr < jb) ? Ds[i][rr] : (i == rr ? 1.0 : 0.0);
      }
      bad |= quad_sweep16(m, jb, lane);
#pragma unroll
      for (int t = 0; t < 4; ++t) Dw[4 * kq + t][rr] = m[t];
    }
    __syncthreads();
    // 3. CD = C D^{-1} with D^{-1} = -Dw
    for (int ti = wave; ti < nt; ti += RS_WAVES) {
      acc_t c = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
        c = Mfma<T>::mac(Cs[16 * ti + rr][4 * s4 + kq], (T)(-Dw[4 * s4 + kq][rr]), c);
#pragma unroll
      for (int r = 0; r < 4; ++r) CDs[16 * ti + Mfma<T>::row(kq, r)][rr] = c[r];
    }
    __syncthreads();
    // 4. rank-16 update and the panel's new entries
#pragma unroll
    for (int sl = 0; sl < TPW; ++sl) {
      const int ti = sti[sl] + oz, tj = stj[sl] + oz;
      if (ti < 0) continue;
      acc_t c = acc[sl];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
        c = Mfma<T>::mac(-CDs[16 * ti + rr][4 * s4 + kq], Cs[16 * tj + rr][4 * s4 + kq], c);
      if (ti == tq || tj == tq) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * ti + Mfma<T>::row(kq, r), j = 16 * tj + rr;
          const bool iq = i >= j0 && i < j0 + jb, jq = j >= j0 && j < j0 + jb;
          const T dv = (T)Dw[(i - j0) & 15][(j - j0) & 15];
          const T c1 = CDs[i][(j - j0) & 15], c2 = CDs[j][(i - j0) & 15];
          c[r] = (iq && jq) ? dv : jq ? c1 : iq ? c2 : c[r];
        }
      }
      acc[sl] = c;
      // keep each slot's operand loads next to its MFMAs (register pressure)
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (bad && lane == 0) atomicMax(status, status_code);
  // write both triangles
#pragma unroll
  for (int sl = 0; sl < TPW; ++sl) {
    const int ti = sti[sl], tj = stj[sl];
    if (ti < 0) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * ti + Mfma<T>::row(kq, r), j = 16 * tj + rr;
      if (i < n && j < n) {
        char* base = reinterpret_cast<char*>(A);
        *reinterpret_cast<T*>(base + (uint32_t)(i * ld + j) * (uint32_t)sizeof(T)) = acc[sl][r];
        if (ti != tj) *reinterpret_cast<T*>(base + (uint32_t)(j * ld + i) * (uint32_t)sizeof(T)) = acc[sl][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Sweep of matrices above 272 rows, by slabs of SLAB pivots S = j0..j0+sb-1.
// Sweeping S at once equals sweeping its pivots in turn, so per slab:
//   1. k_sweep_reg (slab mode) replaces M_SS by -M_SS^{-1} in place;
//   2. k_slab_cd forms CD = M_{:,S} M_SS^{-1} for the rows outside S;
//   3. k_slab_update applies M_ij -= CD_i M_{j,S}^T to the lower triangle
//      outside S (rank-sb, on MFMA; M_{j,S} still holds the old values);
//   4. k_slab_writeback stores CD into the slab's rows and columns.
// Only the lower triangle is kept current; k_symmetrize mirrors it at the end.
// CD lives in scratch, n x SLAB per matrix (column-major, ld n).

// C[i][t] = M[i][j0 + t] from the lower triangle (the row panel above j0).
template <typename T>
__device__ __forceinline__ T slab_c(const T* A, int ld, int j0, int i, int t) {
  return i >= j0 ? A[i + (int64_t)ld * (j0 + t)] : A[(j0 + t) + (int64_t)ld * i];
}

// Element e of an array with a wave-uniform base, addressed by a 32-bit byte
// offset (matrices here stay far below 4 GB): no 64-bit address registers.
template <typename T>
__device__ __forceinline__ T ld32(const T* base, uint32_t e) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + e * (uint32_t)sizeof(T));
}
// slab_c through 32-bit offsets
template <typename T>
__device__ __forceinline__ T slab_c32(const T* A, int ld, int j0, int i, int t) {
  return ld32(A, i >= j0 ? (uint32_t)(i + ld * (j0 + t)) : (uint32_t)((j0 + t) + ld * i));
}

// 2. CD[i][q] = -sum_t C[i][t] W[t][q], W = M_SS after step 1 (= -M_SS^{-1}).
// One workgroup per (64-row tile, 64-column tile of the slab, matrix).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_slab_cd(const SweepDesc* __restrict__ desc, const T* __restrict__ pool,
                                                 int j0, T* __restrict__ scratch, int64_t scr_stride, int sl) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T As[32][TILE + PAD];  // C rows i, K chunk
  __shared__ T Bs[32][TILE + PAD];  // W columns q, K chunk
  const SweepDesc d = desc[blockIdx.z];
  const int n = d.n, ld = d.ld;
  const int sb = min(sl, d.p - j0);
  if (sb <= 0) return;
  const int i0 = blockIdx.x * TILE, q0 = blockIdx.y * TILE;
  if (i0 >= n || q0 >= sb) return;
  const T* A = pool + d.off;
  T* CD = scratch + (int64_t)blockIdx.z * scr_stride;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int kq = lane >> 4, rr = lane & 15;
  const int wi = (wave & 1) * 32, wq = (wave >> 1) * 32;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  // the next K chunk is loaded into registers while this one is multiplied
  T av[8], bv[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = tid + u * 256;
      const int r = idx % TILE, t = idx / TILE;   // 64 rows x 32 K
      const int i = i0 + r, kk = k0 + t;
      const bool ok = i < n && kk < sb && !(i >= j0 && i < j0 + sb);
      av[u] = ok ? slab_c32(A, ld, j0, i, kk) : (T)0;
      const int q = q0 + r;                        // W[kk][q] = M[j0+q][j0+kk] (both triangles valid)
      bv[u] = (q < sb && kk < sb) ? ld32(A, (uint32_t)((j0 + q) + ld * (j0 + kk))) : (T)0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < sb; k0 += 32) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = tid + u * 256;
      As[idx / TILE][idx % TILE] = av[u];
      Bs[idx / TILE][idx % TILE] = bv[u];
    }
    __syncthreads();
    if (k0 + 32 < sb) load(k0 + 32);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int kk = ks * 4 + kq;
      T x[2], y[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) x[a] = As[kk][wi + a * 16 + rr];
#pragma unroll
      for (int b = 0; b < 2; ++b) y[b] = Bs[kk][wq + b * 16 + rr];
      // output tile transposed (W as the A operand) so lanes run along i
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::mac(y[b], x[a], acc[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = q0 + wq + b * 16 + Mfma<T>::row(kq, r);
        const int i = i0 + wi + a * 16 + rr;
        if (i < n && q < sb && !(i >= j0 && i < j0 + sb)) CD[i + (int64_t)n * q] = -acc[a][b][r];
      }
}

// 3. Lower-triangle tiles outside S: M_ij -= sum_q CD[i][q] C[j][q].
// region: 0 every tile; 1 only the tiles of the next slab's pivot block;
// 2 every tile but those (the two halves of the update, for the look-ahead).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_slab_update(const SweepDesc* __restrict__ desc, T* pool, int j0,
                                                     const T* __restrict__ scratch, int64_t scr_stride,
                                                     int ntri, int nprob, int region, int sl) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T As[32][TILE + PAD];  // CD rows i
  __shared__ T Bs[32][TILE + PAD];  // C rows j
  const int64_t nblk = gridDim.x;
  const int64_t glin = blockIdx.x;
  const int64_t logical = (glin % 8) * (nblk / 8) + glin / 8;  // XCD-aware
  if (logical >= (int64_t)nprob * ntri) return;
  const int prob = (int)(logical / ntri);
  const SweepDesc d = desc[prob];
  const int n = d.n, ld = d.ld;
  const int sb = min(sl, d.p - j0);
  if (sb <= 0) return;
  const int lin = (int)(logical % ntri);
  int ti = (int)((sqrt(8.0 * lin + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= lin) ++ti;
  while (ti * (ti + 1) / 2 > lin) --ti;
  const int tj = lin - ti * (ti + 1) / 2;
  const int i0 = ti * TILE, c0 = tj * TILE;
  if (i0 >= n || c0 >= n) return;
  // tiles wholly inside the slab rows or columns take no update
  if ((i0 >= j0 && i0 + TILE <= j0 + sb) || (c0 >= j0 && c0 + TILE <= j0 + sb)) return;
  if (region) {
    const int j1 = j0 + sb, sbn = min(sl, d.p - j1);  // next slab's pivots
    const bool nextd = sbn > 0 && i0 + TILE > j1 && i0 < j1 + sbn && c0 + TILE > j1 && c0 < j1 + sbn;
    if ((region == 1) != nextd) return;
  }
  T* A = pool + d.off;
  const T* CD = scratch + (int64_t)prob * scr_stride;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int kq = lane >> 4, rr = lane & 15;
  const int wi = (wave & 1) * 32, wj = (wave >> 1) * 32;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  // the next K chunk is loaded into registers while this one is multiplied
  T av[8], bv[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = tid + u * 256;
      const int r = idx % TILE, q = idx / TILE;
      const int i = i0 + r, j = c0 + r, kk = k0 + q;
      av[u] = (i < n && kk < sb && !(i >= j0 && i < j0 + sb)) ? ld32(CD, (uint32_t)(i + n * kk)) : (T)0;
      bv[u] = (j < n && kk < sb && !(j >= j0 && j < j0 + sb)) ? slab_c32(A, ld, j0, j, kk) : (T)0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < sb; k0 += 32) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = tid + u * 256;
      As[idx / TILE][idx % TILE] = av[u];
      Bs[idx / TILE][idx % TILE] = bv[u];
    }
    __syncthreads();
    if (k0 + 32 < sb) load(k0 + 32);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int kk = ks * 4 + kq;
      T x[2], y[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) x[a] = As[kk][wi + a * 16 + rr];
#pragma unroll
      for (int b = 0; b < 2; ++b) y[b] = Bs[kk][wj + b * 16 + rr];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::mac(y[b], x[a], acc[a][b]);
    }
  }
  T old[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = c0 + wj + b * 16 + Mfma<T>::row(kq, r);
        const int i = i0 + wi + a * 16 + rr;
        const bool on = i < n && j <= i && !(i >= j0 && i < j0 + sb) && !(j >= j0 && j < j0 + sb);
        old[a][b][r] = on ? A[i + (int64_t)ld * j] : (T)0;
      }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = c0 + wj + b * 16 + Mfma<T>::row(kq, r);
        const int i = i0 + wi + a * 16 + rr;
        if (i < n && j <= i && !(i >= j0 && i < j0 + sb) && !(j >= j0 && j < j0 + sb))
          A[i + (int64_t)ld * j] = old[a][b][r] - acc[a][b][r];
      }
}

// 3'. The same trailing update by 128 x 128 tiles: each of the four waves
// owns a 64 x 64 quarter (4 x 4 MFMA tiles), so every operand element staged
// in LDS feeds four MFMAs per wave and a tile moves half the operand bytes
// per flop of the 64 x 64 form (about 10 flop/B from L2 instead of 6).
constexpr int UT = 128, UK = 16;

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_slab_update128(
    const SweepDesc* __restrict__ desc, T* pool, int j0, const T* __restrict__ scratch, int64_t scr_stride,
    int ntri, int nprob, int region, int sl) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T As[UK][UT + PAD];  // CD rows i
  __shared__ T Bs[UK][UT + PAD];  // slab columns of rows j
  const int64_t nblk = gridDim.x;
  const int64_t glin = blockIdx.x;
  const int64_t logical = (glin % 8) * (nblk / 8) + glin / 8;  // XCD-aware
  if (logical >= (int64_t)nprob * ntri) return;
  const int prob = (int)(logical / ntri);
  const SweepDesc d = desc[prob];
  const int n = d.n, ld = d.ld;
  const int sb = min(sl, d.p - j0);
  if (sb <= 0) return;
  const int lin = (int)(logical % ntri);
  int ti = (int)((sqrt(8.0 * lin + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= lin) ++ti;
  while (ti * (ti + 1) / 2 > lin) --ti;
  const int tj = lin - ti * (ti + 1) / 2;
  const int i0 = ti * UT, c0 = tj * UT;
  if (i0 >= n || c0 >= n) return;
  if ((i0 >= j0 && i0 + UT <= j0 + sb) || (c0 >= j0 && c0 + UT <= j0 + sb)) return;
  if (region) {
    const int j1 = j0 + sb, sbn = min(sl, d.p - j1);  // next slab's pivots
    const bool nextd = sbn > 0 && i0 + UT > j1 && i0 < j1 + sbn && c0 + UT > j1 && c0 < j1 + sbn;
    if ((region == 1) != nextd) return;
  }
  T* A = pool + d.off;
  const T* CD = scratch + (int64_t)prob * scr_stride;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int kq = lane >> 4, rr = lane & 15;
  const int wi = (wave & 1) * 64, wj = (wave >> 1) * 64;
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  T av[8], bv[8];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = tid + u * 256;
      const int r = idx % UT, q = idx / UT;
      const int i = i0 + r, j = c0 + r, kk = k0 + q;
      av[u] = (i < n && kk < sb && !(i >= j0 && i < j0 + sb)) ? ld32(CD, (uint32_t)(i + n * kk)) : (T)0;
      bv[u] = (j < n && kk < sb && !(j >= j0 && j < j0 + sb)) ? slab_c32(A, ld, j0, j, kk) : (T)0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < sb; k0 += UK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = tid + u * 256;
      As[idx / UT][idx % UT] = av[u];
      Bs[idx / UT][idx % UT] = bv[u];
    }
    __syncthreads();
    if (k0 + UK < sb) load(k0 + UK);
#pragma unroll
    for (int ks = 0; ks < UK / 4; ++ks) {
      const int kk = ks * 4 + kq;
      T x[4], y[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) x[a] = As[kk][wi + a * 16 + rr];
#pragma unroll
      for (int b = 0; b < 4; ++b) y[b] = Bs[kk][wj + b * 16 + rr];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<T>::mac(y[b], x[a], acc[a][b]);
    }
  }
  // per tile row: read the old values of its four MFMA tiles, then write
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    T old[4][4];
    const int i = i0 + wi + a * 16 + rr;
    const bool irow = i < n && !(i >= j0 && i < j0 + sb);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = c0 + wj + b * 16 + Mfma<T>::row(kq, r);
        const bool on = irow && j <= i && !(j >= j0 && j < j0 + sb);
        old[b][r] = on ? A[i + (int64_t)ld * j] : (T)0;
      }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = c0 + wj + b * 16 + Mfma<T>::row(kq, r);
        if (irow && j <= i && !(j >= j0 && j < j0 + sb)) A[i + (int64_t)ld * j] = old[b][r] - acc[a][b][r];
      }
  }
}

// 4. The slab's rows and columns outside S become CD (lower triangle).
template <typename T>
__global__ void k_slab_writeback(const SweepDesc* __restrict__ desc, T* pool, int j0, const T* __restrict__ scratch,
                                 int64_t scr_stride, int sl) {
  const SweepDesc d = desc[blockIdx.y];
  const int n = d.n, ld = d.ld;
  const int sb = min(sl, d.p - j0);
  if (sb <= 0) return;
  T* A = pool + d.off;
  const T* CD = scratch + (int64_t)blockIdx.y * scr_stride;
  const int tot = n * sb;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += gridDim.x * blockDim.x) {
    const int i = idx % n, q = idx / n;
    if (i >= j0 && i < j0 + sb) continue;
    const T v = CD[i + (int64_t)n * q];
    if (i > j0) A[i + (int64_t)ld * (j0 + q)] = v;
    else A[(j0 + q) + (int64_t)ld * i] = v;
  }
}

// ---------------------------------------------------------------------------
// Batched GEMM on MFMA: C = beta C + alpha op(A) op(B), column-major, with one
// descriptor per problem (uneven sizes).  grid = (tiles of the largest
// problem, problems); out-of-range tiles exit at once.  The MFMA computes the
// transposed tile (op(B) as its A operand) so each lane's outputs run down a
// column of C and the stores are coalesced.

constexpr int GBK = 32;  // K chunk of the batched GEMM

template <typename T, int TA, int TB>
__global__ __launch_bounds__(256) void k_gemm(const GemmDesc* __restrict__ desc,
                                              const T* __restrict__ Ap, const T* __restrict__ Bp,
                                              T* __restrict__ Cp, T alpha, T beta, int tiles_m, int tiles_n,
                                              int nprob) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T As[1][GBK][TILE + PAD];
  __shared__ T Bs[1][GBK][TILE + PAD];
  // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs,
  // so consecutive logical tiles (one problem's) are given to one XCD and
  // share its L2.
  const int64_t nblk = gridDim.x;
  const int64_t lin = blockIdx.x;
  const int64_t logical = (lin % 8) * (nblk / 8) + lin / 8;
  const int tiles = tiles_m * tiles_n;
  if (logical >= (int64_t)nprob * tiles) return;
  const int prob = (int)(logical / tiles), tile = (int)(logical % tiles);
  const GemmDesc d = desc[prob];
  const int ti = tile % tiles_m, tj = tile / tiles_m;
  const int m0 = ti * TILE, n0 = tj * TILE;
  if (m0 >= d.m || n0 >= d.n) return;
  const T* A = Ap + d.a;
  const T* B = Bp + d.b;
  T* C = Cp + d.c;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  const int kq = lane >> 4, rr = lane & 15;
  constexpr int PER = TILE * GBK / 256;  // elements per thread per operand
  T ra[PER], rb[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + 256 * u;
      int r, q;
      if (TA) {
        q = idx % GBK;
        r = idx / GBK;
      } else {
        r = idx % TILE;
        q = idx / TILE;
      }
      const int i = m0 + r, kk = k0 + q;
      ra[u] = (i < d.m && kk < d.k) ? (TA ? A[kk + (int64_t)d.lda * i] : A[i + (int64_t)d.lda * kk]) : (T)0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + 256 * u;
      int r, q;
      if (TB) {
        r = idx % TILE;
        q = idx / TILE;
      } else {
        q = idx % GBK;
        r = idx / GBK;
      }
      const int j = n0 + r, kk = k0 + q;
      rb[u] = (j < d.n && kk < d.k) ? (TB ? B[j + (int64_t)d.ldb * kk] : B[kk + (int64_t)d.ldb * j]) : (T)0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + 256 * u;
      int r, q;
      if (TA) {
        q = idx % GBK;
        r = idx / GBK;
      } else {
        r = idx % TILE;
        q = idx / TILE;
      }
      As[buf][q][r] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + 256 * u;
      int r, q;
      if (TB) {
        r = idx % TILE;
        q = idx / TILE;
      } else {
        q = idx % GBK;
        r = idx / GBK;
      }
      Bs[buf][q][r] = rb[u];
    }
  };
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  load(0);
  store(0);
  __syncthreads();
  const int cur = 0;
  // 16x16 sub-tiles of this wave that hold any output (the rest are padding)
  const bool ra0 = m0 + wr < d.m, ra1 = m0 + wr + 16 < d.m;
  const bool rb0 = n0 + wc < d.n, rb1 = n0 + wc + 16 < d.n;
  for (int k0 = 0; k0 < d.k; k0 += GBK) {
    const bool more = k0 + GBK < d.k;
    if (more) load(k0 + GBK);  // next chunk in flight while this one is multiplied
    const int ksteps = min(GBK / 4, (d.k - k0 + 3) / 4);
    if (ra0 && rb0) {
#pragma unroll
      for (int ks = 0; ks < GBK / 4; ++ks) {
        if (ks >= ksteps) break;
        const int kk = ks * 4 + kq;
        T av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = As[cur][kk][wr + a * 16 + rr];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Bs[cur][kk][wc + b * 16 + rr];
        acc[0][0] = Mfma<T>::mac(bv[0], av[0], acc[0][0]);
        if (rb1) acc[0][1] = Mfma<T>::mac(bv[1], av[0], acc[0][1]);
        if (ra1) acc[1][0] = Mfma<T>::mac(bv[0], av[1], acc[1][0]);
        if (ra1 && rb1) acc[1][1] = Mfma<T>::mac(bv[1], av[1], acc[1][1]);
      }
    }    __syncthreads();
    if (more) store(0);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = m0 + wr + a * 16 + rr;
        int j = n0 + wc + b * 16 + Mfma<T>::row(kq, r);
        if (i < d.m && j < d.n) {
          T* c = C + i + (int64_t)d.ldc * j;
          T v = alpha * acc[a][b][r];
          *c = beta == (T)0 ? v : beta * *c + v;
        }
      }
}

// Batched GEMM for problems with at most 176 output rows (non-transposed
// operands): one workgroup of 16 waves per (problem, 128 output columns)
// holds its output block in registers, so every A element is read from
// memory once per 128 columns and every B element once.  The waves form a
// 4 x 4 grid; wave (wr, wc) owns the row tiles wr + 4i and the column tiles
// wc + 4j (16 x 16 each).  K goes in chunks of GF_KC through LDS with the
// next chunk prefetched into registers.  The LDS tiles are zero-padded to
// 192 rows and to whole chunks, so every wave runs the same branch-free
// k-steps (three row tiles, one to three column tiles by a wave-uniform
// choice made once) and the products of padding are never stored.  Two
// shapes: 128 columns per workgroup with K chunks of 32, and for 129 to 192
// columns one workgroup per problem (the 128-column form would need a second
// round of workgroups for the last columns) with K chunks of 16, which keeps
// the nine accumulator tiles per wave within 128 VGPRs.
constexpr int GF_KC = 32;
constexpr int GF_M = 176, GF_N = 128, GF_MP = 192, GF_N3 = 192, GF_KC3 = 16;

template <typename T, int NB, int KC, int GN>
__device__ __forceinline__ void gf_main(const GemmDesc& d, const T* __restrict__ A, const T* __restrict__ B,
                                        T* __restrict__ C, int nn, T alpha, T beta, T (*As)[GF_MP + 4],
                                        T (*Bs)[GN + 4]) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int kq = lane >> 4, rr = lane & 15;
  const int wr = wave & 3, wc = wave >> 2;
  constexpr int PA = (GF_MP * KC) / 1024, PB = GN * KC / 1024;
  T ra[PA], rb[PB];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PA; ++u) {
      const int idx = tid + 1024 * u, i = idx % GF_MP, q = idx / GF_MP;
      ra[u] = (i < d.m && k0 + q < d.k) ? A[i + (int64_t)d.lda * (k0 + q)] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int idx = tid + 1024 * u, q = idx % KC, j = idx / KC;
      rb[u] = (j < nn && k0 + q < d.k) ? B[(k0 + q) + (int64_t)d.ldb * j] : (T)0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < PA; ++u) {
      const int idx = tid + 1024 * u, i = idx % GF_MP, q = idx / GF_MP;
      As[q][i] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int idx = tid + 1024 * u, q = idx % KC, j = idx / KC;
      Bs[q][j] = rb[u];
    }
  };
  acc_t acc[3][NB > 0 ? NB : 1];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < (NB > 0 ? NB : 1); ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  // row tiles of this wave that hold output rows (wave-uniform): a 169-row
  // block needs 11 of the 12 row tiles
  const int na = __builtin_amdgcn_readfirstlane((wr + 8) * 16 < d.m ? 3 : (wr + 4) * 16 < d.m ? 2 : 1);
  load(0);
  for (int k0 = 0; k0 < d.k; k0 += KC) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + KC < d.k) load(k0 + KC);
    // K steps of 4 that reach a valid index of this chunk (the tail chunk of
    // a 169-deep product has 9 of 32)
    const int kv = min(KC, d.k - k0);
    if (NB > 0) {
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        if (ks * 4 >= kv) break;
        const int kk = ks * 4 + kq;
        T av[3], bv[NB > 0 ? NB : 1];
#pragma unroll
        for (int a = 0; a < 3; ++a) av[a] = As[kk][(wr + 4 * a) * 16 + rr];
#pragma unroll
        for (int b = 0; b < NB; ++b) bv[b] = Bs[kk][(wc + 4 * b) * 16 + rr];
        // transposed product (B as the A operand) so each lane's outputs run down a column
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (a >= na) break;
#pragma unroll
          for (int b = 0; b < NB; ++b) acc[a][b] = Mfma<T>::mac(bv[b], av[a], acc[a][b]);
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = (wr + 4 * a) * 16 + rr;
        const int j = (wc + 4 * b) * 16 + Mfma<T>::row(kq, r);
        if (i < d.m && j < nn) {
          T* c = C + i + (int64_t)d.ldc * j;
          const T v = alpha * acc[a][b][r];
          *c = beta == (T)0 ? v : beta * *c + v;
        }
      }
}

template <typename T, int KC, int GN>
__global__ __launch_bounds__(1024) void k_gemm_full(const GemmDesc* __restrict__ desc,
                                                    const T* __restrict__ Ap, const T* __restrict__ Bp,
                                                    T* __restrict__ Cp, T alpha, T beta) {
  __shared__ T As[KC][GF_MP + 4];
  __shared__ T Bs[KC][GN + 4];
  const GemmDesc d = desc[blockIdx.x];
  const int n0 = blockIdx.y * GN;
  if (d.m <= 0 || n0 >= d.n) return;
  const int nn = min(GN, d.n - n0);
  const T* A = Ap + d.a;
  const T* B = Bp + d.b + (int64_t)d.ldb * n0;
  T* C = Cp + d.c + (int64_t)d.ldc * n0;
  // column tiles wc, wc + 4 of this wave that hold output (wave-uniform);
  // every wave runs the same chunk loop and barriers
  const int wc = (threadIdx.x >> 6) >> 2;
  const int nb = __builtin_amdgcn_readfirstlane((wc + 8) * 16 < nn && GN > 128 ? 3
                                                 : (wc + 4) * 16 < nn                ? 2
                                                 : wc * 16 < nn                      ? 1
                                                                                     : 0);
  if (nb == 3) gf_main<T, (GN > 128 ? 3 : 2), KC, GN>(d, A, B, C, nn, alpha, beta, As, Bs);
  else if (nb == 2) gf_main<T, 2, KC, GN>(d, A, B, C, nn, alpha, beta, As, Bs);
  else if (nb == 1) gf_main<T, 1, KC, GN>(d, A, B, C, nn, alpha, beta, As, Bs);
  else gf_main<T, 0, KC, GN>(d, A, B, C, nn, alpha, beta, As, Bs);
}

// ---------------------------------------------------------------------------
// constrained Neumann setup: right-hand sides [C_r^T | -K_rv], couplings

template <typename T>
__global__ void k_rhs_fill(PlanDev P, Geo g, const double* __restrict__ rho, T* __restrict__ Z) {
  const int sub = blockIdx.y;
  const SubDev S = P.subs[sub];
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= S.n_a + S.n_v) return;
  T* z = Z + S.Z_off + (int64_t)S.n_r * P.z_col[S.c_off + col];  // stored in the order the forward solve reaches
  if (col < S.n_a) {
    const int b = P.a_ptr[S.a_off + col], e = P.a_ptr[S.a_off + col + 1];
    const T w = (T)(1.0 / (double)(e - b));
    for (int t = b; t < e; ++t) z[P.a_r[t]] = w;
  } else {
    const int v = col - S.n_a;
    const int lv = P.v_loc[S.v_off + v];
    int cv[3];
    loc_coords(S, lv, cv);
    const int32_t* lr = P.loc_r + S.loc_off;
    const int zr = g.dim == 3 ? 1 : 0;
    for (int dz = -zr; dz <= zr; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int cn[3] = {cv[0] + dx, cv[1] + dy, cv[2] + dz};
          int ln = loc_index(S, cn);
          if (ln < 0) continue;
          int j = lr[ln];
          if (j < 0) continue;
          z[j] = (T)(-kloc(S, g, rho, P.khat, cn, cv));
        }
  }
}

// fwd (fwd = 1): tmp = Z[block k, :] - A_{k,k-1} Z[last plane of k-1, :]
// bwd (fwd = 0): tmp[0:last_n, :] = A_{k,k+1} Z[first plane of k+1, :]
// One workgroup per (column chunk of CPL_COLS, subdomain sub0 + blockIdx.y): the source plane's
// rows of the chunk are staged in LDS once, then every output row takes its
// (up to) 9 neighbours from LDS.
constexpr int CPL_COLS = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_couple_multi(PlanDev P, int k, int fwd, T* __restrict__ Z,
                                                      T* __restrict__ tmp, int64_t tmp_stride, int sub0) {
  extern __shared__ char smem_raw[];
  T(*src)[CPL_COLS + 1] = reinterpret_cast<T(*)[CPL_COLS + 1]>(smem_raw);
  const int sub = sub0 + blockIdx.y;
  const SubDev S = P.subs[sub];
  const int nb = S.nbR;
  const int ncols = S.n_a + S.n_v;
  if (fwd ? k >= nb : k + 1 >= nb) return;
  const int c0 = blockIdx.x * CPL_COLS;
  if (c0 >= ncols) return;
  const int nc = min(CPL_COLS, ncols - c0);
  const BlockDev B = P.blocks[S.bR_off + k];
  // forward: columns the right-hand sides have not reached yet stay zero
  if (fwd && c0 >= B.za) return;
  const int64_t roff = fwd ? B.cf_off : B.cb_off;
  const bool couple = fwd ? (k > 0 && roff >= 0) : roff >= 0;
  if (!fwd && !couple) return;
  const T* z = Z + S.Z_off;
  int sbase = 0;
  if (couple) {
    const BlockDev O = P.blocks[S.bR_off + (fwd ? k - 1 : k + 1)];
    sbase = fwd ? O.start + O.size - O.last_n : O.start;  // first rank of the source plane
    const int sn = fwd ? O.last_n : O.first_n;
    for (int b0 = 0; b0 < sn * nc; b0 += 8 * 256) {  // 8 loads in flight per thread
      T vv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = b0 + threadIdx.x + 256 * u, r = idx % sn, c = idx / sn;
        vv[u] = idx < sn * nc ? z[sbase + r + (int64_t)S.n_r * (c0 + c)] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = b0 + threadIdx.x + 256 * u, r = idx % sn, c = idx / sn;
        if (idx < sn * nc) src[r][c] = vv[u];
      }
    }
    __syncthreads();
  }
  // forward: the whole block's right-hand side, coupled on its first plane;
  // backward: the coupling of the last plane only
  const int rows = fwd ? B.size : B.last_n;
  const int crow = fwd ? B.first_n : B.last_n;   // rows that take a coupling
  const int ld = fwd ? B.size : B.last_n;
  T* tp = tmp + sub * tmp_stride;
  for (int i = threadIdx.x; i < rows; i += blockDim.x) {
    double a[9];
    int l[9];
    const bool ci = couple && i < crow;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int rk = ci ? P.cpl_rank[(roff + i) * 9 + t] : -1;
      a[t] = rk >= 0 ? P.cpl_coef[(roff + i) * 9 + t] : 0.0;
      l[t] = rk >= 0 ? rk - sbase : 0;
    }
    T zin[CPL_COLS];  // the block's right-hand side, all columns' loads in flight at once
#pragma unroll
    for (int c = 0; c < CPL_COLS; ++c)
      zin[c] = (fwd && c < nc) ? z[B.start + i + (int64_t)S.n_r * (c0 + c)] : (T)0;
#pragma unroll
    for (int c = 0; c < CPL_COLS; ++c) {
      if (c >= nc) break;
      double acc = 0.0;
      if (ci) {
#pragma unroll
        for (int t = 0; t < 9; ++t) acc += a[t] * (double)src[l[t]][c];
      }
      tp[i + (int64_t)ld * (c0 + c)] = fwd ? zin[c] - (T)acc : (T)acc;
    }
  }
}

// X at the selected rows, S_c = C_r X (lower triangle) and
// T = C_r Y - [0 I], in one pass over Z's columns.  The column space is
// S_c's n_a columns (X's columns) followed by T's n_c columns; a workgroup
// takes C of them and stages each one's values at the selected rows in LDS
// (X's column b for S_c column b, also stored as XG's column b, 0 at a Gamma
// entry that is a primal vertex; the vertex's column of Y' for a vertex
// column of T; an average column of T is -e_a and reads nothing).  C_r
// takes the mean of a column over each average's nodes, which are Gamma
// entries, so selected rows (a_g over the ranges a_ptr[a]..a_ptr[a+1]);
// every mean is summed from LDS in node order.  S_c = C_r K_rr^{-1} C_r^T is
// symmetric and its sweep reads only the lower triangle, so only a >= b is
// formed there.  T's vertex columns are stored packed (n_a x n_v, ld n_a,
// column v for vertex v): its average columns -e_a are not stored, since
// Lambda's average columns are columns of the swept S_c (k_lam_assemble).
// A vertex's column of Y' is also stored at the selected rows
// as Phi's column of that vertex (the product then adds -X Lambda_v), with
// the unit entry of the vertex's coarse dof in the rows of Gamma entries
// that are primal vertices, and its Gamma rows as YG, for the
// preconditioner's application.
template <typename T, int C>
__global__ __launch_bounds__(256) void k_object_means(PlanDev P, const T* __restrict__ Z, T* __restrict__ XG,
                                                      T* __restrict__ Sc, T* __restrict__ Tv,
                                                      T* __restrict__ PhiG, T* __restrict__ YG, int ld) {
  extern __shared__ unsigned char om_smem[];
  T* zs = (T*)om_smem;                                    // [C][ld]: the columns at the selected rows
  int* ag = (int*)(om_smem + (size_t)C * ld * sizeof(T));  // selected row of each average node
  const int sub = blockIdx.y;
  const SubDev S = P.subs[sub];
  const int na = S.n_a, ncol = na + S.n_c, ns = S.n_s;
  const int j0 = blockIdx.x * C;
  if (j0 >= ncol) return;
  const int a0 = P.a_ptr[S.a_off], nar = P.a_ptr[S.a_off + na] - a0;
  int zc[C];  // Z column staged for each local column, -1: none
  int vx[C];  // the vertex of a vertex column of T, -1: none
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int jj = j0 + j;
    zc[j] = -1;
    vx[j] = -1;
    if (jj < na) {
      zc[j] = P.z_col[S.c_off + jj];
    } else if (jj < ncol) {
      const int kind = P.c_kind[S.c_off + jj - na];
      if (kind >= 0) {
        zc[j] = P.z_col[S.c_off + na + kind];
        vx[j] = kind;
      }
    }
  }
  for (int t = threadIdx.x; t < nar; t += blockDim.x) ag[t] = P.a_g[a0 + t];
  const T* z = Z + S.Z_off;
  // four rows per thread at a time: their row indices first, then all the
  // gathers (4 C loads in flight)
  for (int t0 = 0; t0 < ns; t0 += 4 * (int)blockDim.x) {
    int r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + threadIdx.x + u * blockDim.x;
      r[u] = t < ns ? P.sel_r[S.sel_off + t] : -1;
    }
    T v[4][C];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < C; ++j) v[u][j] = (zc[j] >= 0 && r[u] >= 0) ? z[r[u] + S.n_r * (int64_t)zc[j]] : (T)0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + threadIdx.x + u * blockDim.x;
      if (t >= ns) continue;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        if (zc[j] < 0) continue;
        zs[j * ld + t] = v[u][j];
        if (j0 + j < na) XG[S.XG_off + t + (int64_t)ns * (j0 + j)] = v[u][j];
        if (vx[j] >= 0) {
          const T y = r[u] >= 0 ? v[u][j] : (P.g_v[S.g_off + t] == vx[j] ? (T)1 : (T)0);
          PhiG[S.PhiG_off + t + (int64_t)ns * vx[j]] = y;
          if (t < S.n_g) YG[S.YG_off + t + (int64_t)S.n_g * vx[j]] = y;
        }
      }
    }
  }
  __syncthreads();
  const int nj = min(C, ncol - j0);
  for (int e = threadIdx.x; e < nj * na; e += blockDim.x) {
    const int j = e / na, a = e - j * na, jj = j0 + j;
    if (jj < na && a < jj) continue;  // S_c: lower triangle only
    int zcj = -1, vxj = -1;
#pragma unroll
    for (int q = 0; q < C; ++q)
      if (q == j) {
        zcj = zc[q];
        vxj = vx[q];
      }
    if (zcj < 0) continue;  // an average column of T: -e_a, never stored
    const int pb = P.a_ptr[S.a_off + a] - a0, pe = P.a_ptr[S.a_off + a + 1] - a0;
    const T* col = zs + j * ld;
    double acc = 0.0;
    for (int t = pb; t < pe; ++t) acc += (double)col[ag[t]];
    const double v = acc / (double)(pe - pb);
    if (jj < na)
      Sc[S.Sc_off + a + (int64_t)na * jj] = (T)v;
    else
      Tv[S.T_off + a + (int64_t)na * vxj] = (T)v;
  }
}

// Lambda = -S_c^{-1} T in coarse order.  The swept S_c holds -S_c^{-1} (both
// triangles), and T's average column of average a' is -e_a', so Lambda's
// column there is the swept S_c's column a'; the vertex columns are the
// product's output, packed (n_a x n_v, ld n_a).
template <typename T>
__global__ void k_lam_assemble(PlanDev P, const T* __restrict__ Sc, const T* __restrict__ LV, T* __restrict__ Lam) {
  const int sub = blockIdx.y;
  const SubDev S = P.subs[sub];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= S.n_a * S.n_c) return;
  const int a = idx % S.n_a, c = idx / S.n_a;
  const int kind = P.c_kind[S.c_off + c];
  Lam[S.T_off + idx] = kind < 0 ? Sc[S.Sc_off + a + (int64_t)S.n_a * (-kind - 1)] : LV[S.T_off + a + (int64_t)S.n_a * kind];
}

// Local coarse matrix from the equations that define Phi.  With the
// saddle-point system K_rr Phi_r + K_rv Phi_v + C_r^T Lambda = 0 and
// C_r Phi_r = [0 I], (K Phi)_r = -C_r^T Lambda, so Phi^T K Phi has the rows
// (K Phi)_v at vertex dofs and -Lambda at average dofs.  The two triangles
// are averaged so the result is symmetric to the last bit.
// Stencil rows of the primal vertices: for vertex v of a subdomain and its
// 27 neighbour offsets, the coefficient K[v, j] and a code: the selected-row index of j,
// or -(c+1) when j is the vertex of local coarse dof c, or INT32_MIN when j
// is not a local node.  Filled once per setup.
__global__ void k_vertex_stencil(PlanDev P, Geo g, const double* __restrict__ rho, int64_t* __restrict__ vcode_unused,
                                 double* __restrict__ vcoef, int32_t* __restrict__ vcode) {
  (void)vcode_unused;
  const int sub = blockIdx.y;
  const SubDev S = P.subs[sub];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= S.n_v * 27) return;
  const int v = idx / 27, t = idx % 27;
  const int lv = P.v_loc[S.v_off + v];
  int cv[3];
  loc_coords(S, lv, cv);
  const int dz = g.dim == 3 ? t / 9 - 1 : 0, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  int cn[3] = {cv[0] + dx, cv[1] + dy, cv[2] + dz};
  const int64_t out = (S.v_off + v) * 27 + t;
  const int ln = (g.dim == 2 && t >= 9) ? -1 : loc_index(S, cn);
  if (ln < 0) {
    vcode[out] = INT32_MIN;
    vcoef[out] = 0.0;
    return;
  }
  const int r = P.loc_r[S.loc_off + ln];
  vcode[out] = r >= 0 ? P.loc_sel[S.loc_off + ln] : -(P.v_c[S.v_off + P.g_v[S.g_off + P.loc_g[S.loc_off + ln]]] + 1);
  vcoef[out] = kloc(S, g, rho, P.khat, cv, cn);
}

// K_c's vertex rows in its vertex columns, from the rows' equations: one
// workgroup per (chunk of vertex columns, subdomain).  The chunk's vertex
// columns of Phi (all selected rows) and the subdomain's vertex stencils are staged
// in LDS with coalesced loads; an entry is then a 27-term sum over LDS.  The
// entries in an average row or column are -Lambda (taken by
// k_kc_symmetrize), so only the vertex columns of Phi are staged.
template <typename T>
__global__ __launch_bounds__(256) void k_kc_identity(PlanDev P, const T* __restrict__ PhiR,
                                                     const double* __restrict__ vcoef,
                                                     const int32_t* __restrict__ vcode, T* __restrict__ Kc,
                                                     int kc_cols, int stage_stencils) {
  extern __shared__ double phs[];  // [kc_cols][n_s] Phi, then [n_v][27] coefficients, then [n_v][27] codes
  __shared__ int vcol[8];          // the chunk's columns (local coarse indices of its vertices)
  const SubDev S = P.subs[blockIdx.y];
  const int v0 = blockIdx.x * kc_cols;
  if (v0 >= S.n_v) return;
  const int nc = min(kc_cols, S.n_v - v0), ns = S.n_s, nv27 = stage_stencils ? S.n_v * 27 : 0;
  double* lcoef = phs + (int64_t)kc_cols * P.max_ns;
  int32_t* lcode = reinterpret_cast<int32_t*>(lcoef + (int64_t)27 * P.max_nv);
  const double* scoef = stage_stencils ? lcoef : vcoef + S.v_off * 27;
  const int32_t* scode = stage_stencils ? lcode : vcode + S.v_off * 27;
  if ((int)threadIdx.x < nc) vcol[threadIdx.x] = P.v_c[S.v_off + v0 + threadIdx.x];
  __syncthreads();
  // each column is contiguous (ld n_s): 8 loads in flight per thread
  const T* src = PhiR + S.PhiG_off;
  const int tot = ns * nc;
  for (int b0 = 0; b0 < tot; b0 += 8 * 256) {
    T r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = b0 + threadIdx.x + 256 * u;
      r[u] = i < tot ? src[(int64_t)ns * (v0 + i / ns) + i % ns] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = b0 + threadIdx.x + 256 * u;
      if (i < tot) phs[i] = (double)r[u];
    }
  }
  for (int b0 = 0; b0 < nv27; b0 += 4 * 256) {
    double cf[4];
    int32_t cd[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = b0 + threadIdx.x + 256 * u;
      cf[u] = i < nv27 ? vcoef[S.v_off * 27 + i] : 0.0;
      cd[u] = i < nv27 ? vcode[S.v_off * 27 + i] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = b0 + threadIdx.x + 256 * u;
      if (i < nv27) {
        lcoef[i] = cf[u];
        lcode[i] = cd[u];
      }
    }
  }
  __syncthreads();
  // thread (v, j): row v_c[v], column vcol[j]
  for (int idx = threadIdx.x; idx < S.n_v * nc; idx += blockDim.x) {
    const int v = idx % S.n_v, j = idx / S.n_v, c2 = vcol[j];
    double acc = 0.0;
    for (int t = 0; t < 27; ++t) {
      const int code = scode[v * 27 + t];
      if (code == INT32_MIN) continue;
      const double phi = code >= 0 ? phs[j * ns + code] : (-code - 1 == c2 ? 1.0 : 0.0);
      acc += scoef[v * 27 + t] * phi;
    }
    Kc[S.Kc_off + P.v_c[S.v_off + v] + (int64_t)S.n_c * c2] = (T)acc;
  }
}

// K_c <- its symmetric part, by pairs of 32 x 32 tiles (ti >= tj) staged in
// LDS, so reads and writes run along columns.  Each one-sided entry (i, j)
// (row i's equation) comes from where it was formed: -Lambda on an average
// row (K_c = -Lambda there); on a vertex row, the transposed entry in an
// average column (K_c is symmetric) and the stencil sum of k_kc_identity in
// a vertex column.
template <typename T>
__global__ void k_kc_symmetrize(PlanDev P, const T* __restrict__ Lam, T* __restrict__ Kc) {
  __shared__ double ta[32][33], tb[32][33];
  __shared__ int ki[32], kj[32];
  const SubDev S = P.subs[blockIdx.y];
  const int n = S.n_c, nt = (n + 31) / 32;
  int lin = blockIdx.x, ti = 0;
  if (lin >= nt * (nt + 1) / 2) return;
  while (lin > ti) lin -= ++ti;
  const int tj = lin;
  T* K = Kc + S.Kc_off;
  const T* L = Lam + S.T_off;
  if (threadIdx.x < 32) {
    const int i = ti * 32 + threadIdx.x, j = tj * 32 + threadIdx.x;
    ki[threadIdx.x] = i < n ? P.c_kind[S.c_off + i] : 0;
    kj[threadIdx.x] = j < n ? P.c_kind[S.c_off + j] : 0;
  }
  __syncthreads();
  // one-sided entry (i, j) with kinds a (row) and b (column)
  auto side = [&](int i, int j, int a, int b) -> double {
    if (a < 0) return -(double)L[(-a - 1) + (int64_t)S.n_a * j];
    if (b < 0) return -(double)L[(-b - 1) + (int64_t)S.n_a * i];
    return (double)K[i + (int64_t)n * j];
  };
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int r = e % 32, q = e / 32;
    const int i = ti * 32 + r, j = tj * 32 + q;        // tile (ti, tj)
    ta[r][q] = (i < n && j < n) ? side(i, j, ki[r], kj[q]) : 0.0;
    const int i2 = tj * 32 + r, j2 = ti * 32 + q;      // tile (tj, ti)
    tb[r][q] = (i2 < n && j2 < n) ? side(i2, j2, kj[r], ki[q]) : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int r = e % 32, q = e / 32;
    const double v = 0.5 * (ta[r][q] + tb[q][r]);       // entry (ti*32 + r, tj*32 + q)
    const int i = ti * 32 + r, j = tj * 32 + q;
    if (i < n && j < n) K[i + (int64_t)n * j] = (T)v;
    const double w = 0.5 * (tb[r][q] + ta[q][r]);       // entry (tj*32 + r, ti*32 + q)
    const int i2 = tj * 32 + r, j2 = ti * 32 + q;
    if (ti != tj && i2 < n && j2 < n) K[i2 + (int64_t)n * j2] = (T)w;
  }
}

template <typename T>
__global__ void k_kc_to_front(PlanDev P, const int32_t* __restrict__ subs_c, const T* __restrict__ Kc,
                              double* __restrict__ fpool) {
  const int sub = subs_c[blockIdx.y];
  const SubDev S = P.subs[sub];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= S.n_c * S.n_c) return;
  const int a = idx % S.n_c, b = idx / S.n_c;
  const FrontDev F = P.fronts[S.front];
  const int pa = P.sub_fmap[S.c_off + a], pb = P.sub_fmap[S.c_off + b];
  // the fronts' lower triangles only (the sweeps read nothing else); K_c,i is
  // symmetric, so each lower entry takes (a, b) or its mirror exactly once
  if (pa < pb) return;
  fpool[F.off + pa + (int64_t)F.n * pb] += (double)Kc[S.Kc_off + idx];
}

// Zero the lower triangle of every front (all that is summed into and read
// by the sweeps): one workgroup per (front, 32 columns).
__global__ __launch_bounds__(256) void k_front_zero_lower(PlanDev P, const int32_t* __restrict__ fr,
                                                          double* __restrict__ fpool) {
  const FrontDev F = P.fronts[fr[blockIdx.y]];
  const int j0 = blockIdx.x * 32;
  if (j0 >= F.n) return;
  double* M = fpool + F.off;
  for (int j = j0; j < min(j0 + 32, F.n); ++j)
    for (int i = j + threadIdx.x; i < F.n; i += 256) M[i + (int64_t)F.n * j] = 0.0;
}

// Assembly of a front's lower triangle from its sources, each entry written
// once (no zeroing pass, no read-modify-write, no atomics): the update
// blocks of its children (swept at the level below) and the local coarse
// matrices of the subdomains it splits off, summed in source order.  One
// wave per column j, lanes down the rows i >= j, four rows in flight.
template <typename T>
__global__ __launch_bounds__(256) void k_front_gather(PlanDev P, const int32_t* __restrict__ fr,
                                                      const T* __restrict__ Kc, double* __restrict__ fpool) {
  const FrontDev F = P.fronts[fr[blockIdx.y]];
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= F.n) return;
  const int ns = F.nsrc;
  const int32_t* mp[2];
  const double* cb[2];  // a child's update block (lower triangle, leading dimension ld)
  const T* kb[2];       // a subdomain's local coarse matrix (full, symmetric)
  int mj[2], ld[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    mp[q] = nullptr;
    cb[q] = nullptr;
    kb[q] = nullptr;
    mj[q] = -1;
    ld[q] = 0;
    if (q >= ns) continue;
    mp[q] = P.front_imap + F.src_map[q];
    mj[q] = mp[q][j];
    if (F.src[q] >= 0) {
      const FrontDev C = P.fronts[F.src[q]];
      cb[q] = fpool + C.off + C.p + (int64_t)C.n * C.p;
      ld[q] = C.n;
    } else {
      const SubDev& S = P.subs[-F.src[q] - 1];
      kb[q] = Kc + S.Kc_off;
      ld[q] = S.n_c;
    }
  }
  double* __restrict__ dst = fpool + F.off + (int64_t)F.n * j;
  for (int i0 = j; i0 < F.n; i0 += 256) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 64 * u + lane;
      double acc = 0.0;
      if (i < F.n) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (mj[q] < 0) continue;
          const int mi = mp[q][i];
          if (mi < 0) continue;
          const int hi = max(mi, mj[q]), lo = min(mi, mj[q]);
          acc += cb[q] ? cb[q][hi + (int64_t)ld[q] * lo] : (double)kb[q][hi + (int64_t)ld[q] * lo];
        }
      }
      v[u] = acc;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 64 * u + lane;
      if (i < F.n) dst[i] = v[u];
    }
  }
}

// Extend-add of a child's update block into its parent: one wave per column
// b of the child's border, lanes down the rows a >= b (the lower triangle,
// read along columns).  Each lower entry goes once to the parent's lower
// triangle; the plan orders a child's border as its parent does, so rows
// stay in increasing order there too.  Four entries are read before any is
// added (child and parent fronts never overlap).
__global__ __launch_bounds__(256) void k_front_child_scatter(PlanDev P, const int32_t* __restrict__ children,
                                                             double* __restrict__ fpool) {
  const int ch = children[blockIdx.y];
  const FrontDev C = P.fronts[ch];
  const FrontDev F = P.fronts[C.parent];
  const int nb = C.n - C.p;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (b >= nb) return;
  const int32_t* __restrict__ pm = P.front_pmap + C.pmap_off;
  const int pb = pm[b];
  const double* __restrict__ src = fpool + C.off + (int64_t)C.n * (C.p + b) + C.p;
  double* __restrict__ dst = fpool + F.off;
  for (int a0 = b; a0 < nb; a0 += 256) {
    double v[4];
    int pa[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int a = a0 + 64 * u + lane;
      pa[u] = a < nb ? pm[a] : -1;
      v[u] = a < nb ? src[a] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (pa[u] >= 0) dst[max(pa[u], pb) + (int64_t)F.n * min(pa[u], pb)] += v[u];
  }
}

// ---------------------------------------------------------------------------
// per-iteration kernels

template <typename T>
__global__ void k_gather_I(PlanDev P, Geo g, const double* __restrict__ r, T* __restrict__ vI) {
  const int sub = blockIdx.y, rhs = blockIdx.z;
  const SubDev S = P.subs[sub];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n_I) return;
  vI[rhs * P.tot_I + S.I_off + i] = (T)r[rhs * g.n_free + free_of_local(S, g, P.I_loc[S.I_off + i])];
}

// Block-tridiagonal solve with explicitly inverted diagonal blocks, one
// workgroup per (subdomain, right-hand side):
//   forward  c_k = b_k - A_{k,k-1} xh_{k-1},  xh_k = G_k c_k
//   backward x_k = xh_k - G_k A_{k,k+1} x_{k+1}
// (G_k = -Gs_k, the swept block).  The couplings A_{k,k+-1} come from the
// coupling table.  G_k is symmetric, so only its lower triangle is read:
// each 16x16 lower tile T(r, q) adds T c_q to rows r and T^T c_r to rows q.
// The backward product G_k[:, base:] c (the last-plane columns) reads the
// band of lower rows >= base the same way.
//
// The steps form one chain per workgroup, so the kernel is built to keep
// HBM busy across it: the tiles of the next step's block (which do not
// depend on the solution) are loaded into registers as soon as the current
// step's tiles are consumed, and the next step's coupling terms and vector
// entries are loaded before that.  The neighbour block's values that the
// coupling reads stay in LDS from the step that produced them.  Waves take
// tiles round-robin, keep partial sums per wave in LDS and the waves' sums
// are added in fixed order, so the result is bitwise repeatable.
// Two shapes, both of 8 waves so that two workgroups share a CU: 5
// register-held tiles per wave for sets whose blocks have at most 40 tiles
// (up to 144 rows), 9 tiles for larger blocks.  Sixteen waves (one workgroup
// per CU) make the constrained Neumann solve faster alone but take compute
// units from the coarse solve that runs beside it.  The LDS size allows up
// to 16 waves.
constexpr int BS_WAVES_MAX = 16;

// Tile lin of the lower triangle restricted to tile rows >= t0: first the
// rectangle left of tile column t0, then the triangle of tile rows/columns >= t0.
__device__ __forceinline__ void bs_tile_rc(int lin, int t0, int nrow, int& tr, int& tc) {
  if (lin < nrow * t0) {
    tr = t0 + lin / t0;
    tc = lin % t0;
  } else {
    int l2 = lin - nrow * t0, q = 0;  // integer steps only, so wave-uniform inputs stay scalar
    while (l2 > q) l2 -= ++q;
    tr = t0 + q;
    tc = t0 + l2;
  }
}

// lane (a, g) loads the entries (16 tr + a, 16 tc + 4 g + u), u < 4, of the
// lower triangle; outside it or above row s / below row base it loads the
// block's first entry, which bs_tile_mul ignores.  The tile's
// origin is wave-uniform, so each load is a scalar base plus a 32-bit lane
// offset.
template <typename T>
__device__ __forceinline__ void bs_tile_load(const T* __restrict__ M, int s, int ld, int base, int tr, int tc, int a,
                                             int g, T (&L)[4]) {
  const int r = tr * 16 + a;
  const bool rok = r < s && r >= base;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = tc * 16 + 4 * g + u;
    const bool on = rok && q <= r;
    // every lane loads (entry 0 when off: bs_tile_mul masks it), from the
    // uniform block base plus a 32-bit byte offset; nothing touches the
    // value until it is used, so the load stays in flight
    const uint32_t byte = on ? (uint32_t)(q * ld + r) * (uint32_t)sizeof(T) : 0u;
    L[u] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(M) + byte);
  }
}

// y[r] += sum_{q >= base} T(r, q) x[q - base] (rows of the tile) and
// y[q] += T(r, q) x[r - base] for q < r (the mirrored upper entries).
template <typename T>
__device__ __forceinline__ void bs_tile_mul(const T (&L)[4], int s, int base, int tr, int tc, int a, int g,
                                            const T* __restrict__ x, double* __restrict__ y) {
  const int r = tr * 16 + a;
  const bool rok = r < s && r >= base;
  double t1 = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = tc * 16 + 4 * g + u;
    if (rok && q >= base && q <= r) t1 += (double)L[u] * (double)x[q - base];
  }
  t1 += xor_lane_f64<16>(t1);
  t1 += xor_lane_f64<32>(t1);
  if (g == 0 && rok) y[r] += t1;
  const double xr = rok ? (double)x[r - base] : 0.0;
  double p[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) p[u] = (rok && tc * 16 + 4 * g + u < r) ? (double)L[u] * xr : 0.0;
  // sum p[u] over the 16 lanes a by halving: after the exchange across
  // lane bit 3 a lane keeps two columns, after bit 2 one column
  // u = 2 (a>>3 & 1) + (a>>2 & 1), and bits 1 and 0 complete the sum
  const bool h8 = (a & 8) != 0, h4 = (a & 4) != 0;
  double k0 = h8 ? p[2] : p[0], k1 = h8 ? p[3] : p[1];
  k0 += xor_lane_f64<8>(h8 ? p[0] : p[2]);
  k1 += xor_lane_f64<8>(h8 ? p[1] : p[3]);
  double k2 = h4 ? k1 : k0;
  k2 += xor_lane_f64<4>(h4 ? k0 : k1);
  k2 += xor_lane_f64<2>(k2);
  k2 += xor_lane_f64<1>(k2);
  const int q = tc * 16 + 4 * g + (h8 ? 2 : 0) + (h4 ? 1 : 0);
  if ((a & 3) == 0 && q < s) y[q] += k2;
}

// A block descriptor read into scalar registers (the loads cannot be proven
// unclobbered by the kernel's vector stores, so the fields are made uniform
// explicitly and the tile addresses stay scalar).
__device__ __forceinline__ int64_t rfl64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ BlockDev block_uniform(const BlockDev* __restrict__ p) {
  BlockDev B = *p;
  B.start = __builtin_amdgcn_readfirstlane(B.start);
  B.size = __builtin_amdgcn_readfirstlane(B.size);
  B.plane_lo = __builtin_amdgcn_readfirstlane(B.plane_lo);
  B.plane_hi = __builtin_amdgcn_readfirstlane(B.plane_hi);
  B.first_n = __builtin_amdgcn_readfirstlane(B.first_n);
  B.last_n = __builtin_amdgcn_readfirstlane(B.last_n);
  B.ld = __builtin_amdgcn_readfirstlane(B.ld);
  B.G_off = rfl64(B.G_off);
  B.cf_off = rfl64(B.cf_off);
  B.cb_off = rfl64(B.cb_off);
  return B;
}

template <typename T, int BS_THREADS, int BS_PT, int BS_CP>
__global__ __launch_bounds__(BS_THREADS) void k_block_solve(PlanDev P, int setR, const T* __restrict__ G,
                                                            T* __restrict__ vec) {
  constexpr int BS_WAVES = BS_THREADS / 64;
  extern __shared__ char smem_raw[];
  const int mb = P.max_block;
  double* yp = reinterpret_cast<double*>(smem_raw);  // BS_WAVES x mb partial products
  double* prod = yp + (int64_t)BS_WAVES * mb;        // 9 x mb coupling terms
  T* cl = reinterpret_cast<T*>(prod + (int64_t)9 * mb);  // the step's right-hand side
  T* xs = cl + mb;                                   // final values of the last block solved
  const int sub = blockIdx.x, rhs = blockIdx.y;
  const SubDev S = P.subs[sub];
  const int nb = setR ? S.nbR : S.nbI;
  const BlockDev* blk = P.blocks + (setR ? S.bR_off : S.bI_off);
  T* v = vec + rhs * (setR ? P.tot_r : P.tot_I) + (setR ? S.r_off : S.I_off);
  const int tid = threadIdx.x, lane = tid & 63, a = lane & 15, g = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int i = tid; i < BS_WAVES * mb; i += BS_THREADS) yp[i] = 0.0;
  // steps 0..nb-1 forward over block t, then backward over block 2 nb - 2 - t
  // (blocks without a coupling to the next one have no backward step)
  const int nsteps = nb > 0 ? 2 * nb - 1 : 0;
  auto next_step = [&](int t) {
    ++t;
    while (t < nsteps && t >= nb && blk[2 * nb - 2 - t].cb_off < 0) ++t;
    return t;
  };
  auto step_block = [&](int t) { return t < nb ? t : 2 * nb - 2 - t; };
  // coupled rows and their table offset, base of the product
  auto step_shape = [&](int t, const BlockDev& B, int& nrows, int64_t& crow, int& base) {
    if (t < nb) {
      nrows = B.cf_off >= 0 ? B.first_n : 0;
      crow = B.cf_off;
      base = 0;
    } else {
      nrows = B.last_n;
      crow = B.cb_off;
      base = B.size - B.last_n;
    }
  };
  T L[BS_PT][4];
  int rk[BS_CP];
  double cf[BS_CP];
  T vin_next = (T)0;
  auto prefetch_small = [&](int t, const BlockDev& B) {  // coupling terms and v entries of step t
    int nrows, base;
    int64_t crow;
    step_shape(t, B, nrows, crow, base);
#pragma unroll
    for (int m = 0; m < BS_CP; ++m) {
      const int p = tid + BS_THREADS * m;
      const bool on = p < 9 * nrows;
      rk[m] = on ? P.cpl_rank[crow * 9 + p] : -1;
      cf[m] = on ? P.cpl_coef[crow * 9 + p] : 0.0;
    }
    vin_next = tid < B.size ? v[B.start + tid] : (T)0;
  };
  // tile u of step t into L[u]
  auto prefetch_tile = [&](int t, const BlockDev& B, int u) {
    int nrows, base;
    int64_t crow;
    step_shape(t, B, nrows, crow, base);
    const int nt = (B.size + 15) >> 4, t0 = base >> 4, nrow = nt - t0;
    const int ntiles = nrow * t0 + nrow * (nrow + 1) / 2;
    const int lin = wave + BS_WAVES * u;
    int tr = nt, tc = 0;  // past the last row: loads nothing
    if (lin < ntiles) bs_tile_rc(lin, t0, nrow, tr, tc);
    bs_tile_load(G + B.G_off, B.size, B.ld, base, tr, tc, a, g, L[u]);
  };
  auto prefetch_tiles = [&](int t, const BlockDev& B) {
#pragma unroll
    for (int u = 0; u < BS_PT; ++u) prefetch_tile(t, B, u);
  };
  if (nsteps > 0) {
    const BlockDev B0 = block_uniform(blk);
    prefetch_small(0, B0);
    prefetch_tiles(0, B0);
  }
  int xs_blk = -1, xs_start = 0;
  __syncthreads();
  for (int t = 0; t < nsteps;) {
    const int tn = next_step(t);
    const BlockDev Bn = block_uniform(blk + step_block(tn < nsteps ? tn : t));
    const bool fwd = t < nb;
    const int k = step_block(t);
    const BlockDev B = block_uniform(blk + k);
    const int s = B.size;
    int nrows, base;
    int64_t crow;
    step_shape(t, B, nrows, crow, base);
    const T vin = vin_next;  // vin_next is reloaded for the next step before C reads vin
    // A. coupling terms from the neighbour block's final values
    if (nrows > 0) {
      const int nbr = fwd ? k - 1 : k + 1;
      if (xs_blk != nbr) {  // its values are not in LDS (a skipped step before): read them
        const BlockDev Bx = block_uniform(blk + nbr);
        for (int i = tid; i < Bx.size; i += BS_THREADS) xs[i] = v[Bx.start + i];
        xs_blk = nbr;
        xs_start = Bx.start;
        __syncthreads();
      }
#pragma unroll
      for (int m = 0; m < BS_CP; ++m) {
        const int p = tid + BS_THREADS * m;
        if (p < 9 * nrows) prod[p] = rk[m] >= 0 ? cf[m] * (double)xs[rk[m] - xs_start] : 0.0;
      }
      for (int p = tid + BS_THREADS * BS_CP; p < 9 * nrows; p += BS_THREADS) {
        const int j = P.cpl_rank[crow * 9 + p];
        prod[p] = j >= 0 ? P.cpl_coef[crow * 9 + p] * (double)xs[j - xs_start] : 0.0;
      }
      __syncthreads();
    }
    for (int i = tid; i < (fwd ? s : nrows); i += BS_THREADS) {
      double acc = 0.0;
      if (i < nrows) {
#pragma unroll
        for (int u = 0; u < 9; ++u) acc += prod[9 * i + u];
      }
      if (fwd) {
        const T b = i == tid ? vin : v[B.start + i];
        cl[i] = b - (T)acc;
      } else {
        cl[i] = (T)acc;
      }
    }
    __syncthreads();
    // B. the block product.  The next step's loads are issued as the
    // registers free up: the small ones first (A waits for them), then each
    // tile's right after its product, so the step's HBM traffic runs beside
    // its arithmetic instead of after it.
    if (tn < nsteps) prefetch_small(tn, Bn);
    {
      const int nt = (s + 15) >> 4, t0 = base >> 4, nrow = nt - t0;
      const int ntiles = nrow * t0 + nrow * (nrow + 1) / 2;
      double* y = yp + (int64_t)wave * mb;
#pragma unroll
      for (int u = 0; u < BS_PT; ++u) {
        const int lin = wave + BS_WAVES * u;
        if (lin < ntiles) {
          int tr, tc;
          bs_tile_rc(lin, t0, nrow, tr, tc);
          bs_tile_mul(L[u], s, base, tr, tc, a, g, cl, y);
        }
        if (tn < nsteps) prefetch_tile(tn, Bn, u);
        __builtin_amdgcn_sched_barrier(0);  // one tile's temporaries at a time (register pressure)
      }
      for (int lin = wave + BS_WAVES * BS_PT; lin < ntiles; lin += BS_WAVES) {  // blocks above 192 rows
        int tr, tc;
        bs_tile_rc(lin, t0, nrow, tr, tc);
        T Lx[4];
        bs_tile_load(G + B.G_off, s, B.ld, base, tr, tc, a, g, Lx);
        bs_tile_mul(Lx, s, base, tr, tc, a, g, cl, y);
      }
    }
    __syncthreads();
    // C. sum the waves' partials in fixed order, clear them, store
    for (int i = tid; i < s; i += BS_THREADS) {
      double acc = 0.0;
#pragma unroll
      for (int w = 0; w < BS_WAVES; ++w) {
        acc += yp[(int64_t)w * mb + i];
        yp[(int64_t)w * mb + i] = 0.0;
      }
      T o;
      if (fwd) {
        o = -(T)acc;
      } else {
        const T xh = i == tid ? vin : v[B.start + i];
        o = xh + (T)acc;
      }
      v[B.start + i] = o;
      xs[i] = o;
    }
    xs_blk = k;
    xs_start = B.start;
    __syncthreads();
    t = tn;
  }
}

// The same block-tridiagonal solve for many right-hand sides at once: one
// workgroup per (subdomain, group of MR_COLS right-hand sides), so each G_k
// is streamed from HBM once per group.  The products G_k C (C: the block's
// right-hand sides, size x MR_COLS, staged in LDS) run on MFMA: a wave owns
// 16 rows of the output and all MR_COLS columns, and each A-operand load of
// G feeds MR_COLS / 16 MFMAs.
constexpr int MR_COLS = 32;
constexpr int MR_THREADS = 512;

template <typename T>
__device__ __forceinline__ void block_gemm_mr(const T* __restrict__ M, int s, int ncols, int nrows,
                                              const T (*cl)[MR_COLS + 1], T* __restrict__ v, int64_t vstride,
                                              int nr, bool accumulate, T sign, int wave, int lane) {
  // v[r][i] (+)= sign * sum_{j < ncols} M[i + s j] cl[j][r],  i < nrows, r < nr
  typedef typename Mfma<T>::acc_t acc_t;
  const int kq = lane >> 4, rr = lane & 15;
  for (int rt = wave; rt * 16 < nrows; rt += MR_THREADS / 64) {
    const int row = rt * 16 + rr;
    const bool rok = row < nrows;
    acc_t acc[MR_COLS / 16];
#pragma unroll
    for (int c = 0; c < MR_COLS / 16; ++c) acc[c] = acc_t{0, 0, 0, 0};
    int k0 = 0;
    for (; k0 + 16 <= ncols; k0 += 16) {
      T a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = rok ? M[row + (int64_t)s * (k0 + 4 * u + kq)] : (T)0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < MR_COLS / 16; ++c)
          acc[c] = Mfma<T>::mac(a[u], cl[k0 + 4 * u + kq][16 * c + rr], acc[c]);
    }
    for (; k0 < ncols; k0 += 4) {
      const int kk = k0 + kq;
      const T a = (rok && kk < ncols) ? M[row + (int64_t)s * kk] : (T)0;
#pragma unroll
      for (int c = 0; c < MR_COLS / 16; ++c)
        acc[c] = Mfma<T>::mac(a, kk < ncols ? cl[kk][16 * c + rr] : (T)0, acc[c]);
    }
    // lane holds D[row(kq, e)][rr] of each 16 x 16 output block
#pragma unroll
    for (int c = 0; c < MR_COLS / 16; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = rt * 16 + Mfma<T>::row(kq, e), r = 16 * c + rr;
        if (i < nrows && r < nr) {
          T* dst = v + (int64_t)r * vstride + i;
          *dst = accumulate ? *dst + sign * acc[c][e] : sign * acc[c][e];
        }
      }
  }
}

template <typename T>
__global__ __launch_bounds__(MR_THREADS) void k_block_solve_mr(PlanDev P, int setR, const T* __restrict__ G,
                                                               T* __restrict__ vec, int nrhs) {
  extern __shared__ char smem_raw[];
  T(*cl)[MR_COLS + 1] = reinterpret_cast<T(*)[MR_COLS + 1]>(smem_raw);  // [max_block][cols]
  const int sub = blockIdx.x, r0 = blockIdx.y * MR_COLS;
  const int nr = min(MR_COLS, nrhs - r0);
  const SubDev S = P.subs[sub];
  const int nb = setR ? S.nbR : S.nbI;
  const BlockDev* blk = P.blocks + (setR ? S.bR_off : S.bI_off);
  const int64_t vstride = setR ? P.tot_r : P.tot_I;
  T* v = vec + (int64_t)r0 * vstride + (setR ? S.r_off : S.I_off);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int k = 0; k < nb; ++k) {
    const BlockDev B = blk[k];
    for (int idx = tid; idx < B.size * MR_COLS; idx += MR_THREADS) {
      const int i = idx % B.size, r = idx / B.size;
      T c = 0;
      if (r < nr) {
        const T* vr = v + (int64_t)r * vstride;
        c = vr[B.start + i];
        if (B.cf_off >= 0 && i < B.first_n) {
          const int64_t row = B.cf_off + i;
          double acc = 0.0;
#pragma unroll
          for (int t = 0; t < 9; ++t) {
            const int j = P.cpl_rank[row * 9 + t];
            if (j >= 0) acc += P.cpl_coef[row * 9 + t] * (double)vr[j];
          }
          c -= (T)acc;
        }
      }
      cl[i][r] = c;
    }
    __syncthreads();
    block_gemm_mr(G + B.G_off, B.ld, B.size, B.size, cl, v + B.start, vstride, nr, false, (T)-1, wave, lane);
    __syncthreads();
  }
  for (int k = nb - 2; k >= 0; --k) {
    const BlockDev B = blk[k];
    if (B.cb_off < 0) continue;
    const int base = B.size - B.last_n;
    for (int idx = tid; idx < B.last_n * MR_COLS; idx += MR_THREADS) {
      const int i = idx % B.last_n, r = idx / B.last_n;
      double acc = 0.0;
      if (r < nr) {
        const T* vr = v + (int64_t)r * vstride;
        const int64_t row = B.cb_off + i;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const int j = P.cpl_rank[row * 9 + t];
          if (j >= 0) acc += P.cpl_coef[row * 9 + t] * (double)vr[j];
        }
      }
      cl[i][r] = (T)acc;
    }
    __syncthreads();
    block_gemm_mr(G + B.G_off + (int64_t)B.ld * base, B.ld, B.last_n, B.size, cl, v + B.start, vstride, nr,
                  true, (T)1, wave, lane);
    __syncthreads();
  }
}

// The K_{Gamma I} entries (the interior neighbours the plan lists for each
// Gamma entry): the neighbour's interior index and the stiffness entry (from
// rho).  One thread per entry.
__global__ void k_kgi_fill(PlanDev P, Geo g, const double* __restrict__ rho) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= P.n_kgi) return;
  const int64_t ge = P.kgi_own[k];
  const SubDev S = P.subs[P.g_sub[ge]];
  int c[3];
  loc_coords(S, P.g_loc[ge], c);
  const int t = P.kgi_t[k];
  const int cn[3] = {c[0] + t % 3 - 1, c[1] + (t / 3) % 3 - 1, c[2] + t / 9 - 1};
  P.kgi_col[k] = P.loc_I[S.loc_off + loc_index(S, cn)];
  P.kgi_val[k] = kloc(S, g, rho, P.khat, c, cn);
}

// q[e] = (K_{Gamma I} y_I)[e] for the Gamma entries of each subdomain, from
// the entries the setup stored.
template <typename T>
__global__ void k_gamma_kgi(PlanDev P, const T* __restrict__ vI, T* __restrict__ q) {
  const int sub = blockIdx.y, rhs = blockIdx.z;
  const SubDev S = P.subs[sub];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S.n_g) return;
  const T* y = vI + rhs * P.tot_I + S.I_off;
  const int64_t ge = S.g_off + e;
  double acc = 0.0;
  for (int k = P.kgi_ptr[ge]; k < P.kgi_ptr[ge + 1]; ++k) acc += P.kgi_val[k] * (double)y[P.kgi_col[k]];
  q[rhs * P.tot_g + ge] = (T)acc;
}

// t = r_Gamma - sum_i q_i (I - P)^T, then g_e = delta_e t (E^T).
template <typename T>
__global__ void k_gamma_t(PlanDev P, Geo g, const double* __restrict__ r, const T* __restrict__ q,
                          const double* __restrict__ delta, T* __restrict__ gv) {
  const int64_t qg = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (qg >= P.n_gam) return;
  double t = r[rhs * g.n_free + P.gam_node[qg]];
  const int b = P.gam_eptr[qg], e = P.gam_eptr[qg + 1];
  for (int k = b; k < e; ++k) t -= (double)q[rhs * P.tot_g + P.gam_ent[k]];
  for (int k = b; k < e; ++k) {
    int ent = P.gam_ent[k];
    gv[rhs * P.tot_g + ent] = (T)(delta[ent] * t);
  }
}

template <typename T>
__global__ void k_neumann_rhs(PlanDev P, const T* __restrict__ gv, T* __restrict__ vR) {
  const int sub = blockIdx.y, rhs = blockIdx.z;
  const SubDev S = P.subs[sub];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S.n_g) return;
  const int r = P.g_r[S.g_off + e];
  if (r >= 0) vR[rhs * P.tot_r + S.r_off + r] = gv[rhs * P.tot_g + S.g_off + e];
}

// mu = S_c^{-1} C_r u, one workgroup per (subdomain, rhs, 64 rows).  Sc holds the
// swept matrix -S_c^{-1}.
// Partial sums of y = M x (M: nrow x ncol, column-major with leading
// dimension ld; x in LDS), accumulated in A, by a 256-thread workgroup: lane
// l of wave w sums rows 64 k + l over the columns j = w mod 4 with four loads
// in flight, into part[w * stride + row] (LDS, stride >= nrow).  Ends with a
// barrier.
template <typename A, typename T, typename X>
__device__ __forceinline__ void gemv_split4(const T* __restrict__ M, int ld, int nrow, int ncol, const X* x,
                                            A* part, int stride) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r0 = 0; r0 < nrow; r0 += 64) {
    const int r = r0 + lane;
    if (r < nrow) {
      A a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      int j = w;
      for (; j + 12 < ncol; j += 16) {
        a0 += (A)M[r + (int64_t)ld * j] * (A)x[j];
        a1 += (A)M[r + (int64_t)ld * (j + 4)] * (A)x[j + 4];
        a2 += (A)M[r + (int64_t)ld * (j + 8)] * (A)x[j + 8];
        a3 += (A)M[r + (int64_t)ld * (j + 12)] * (A)x[j + 12];
      }
      for (; j < ncol; j += 4) a0 += (A)M[r + (int64_t)ld * j] * (A)x[j];
      part[w * stride + r] = (a0 + a1) + (a2 + a3);
    }
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_mu(PlanDev P, const T* __restrict__ vR, const T* __restrict__ Sc,
                                            T* __restrict__ mu) {
  extern __shared__ char smem_raw[];
  T* av = reinterpret_cast<T*>(smem_raw);
  const int sub = blockIdx.x, rhs = blockIdx.y;
  const SubDev S = P.subs[sub];
  const int r0 = blockIdx.z * 64;  // this workgroup's 64 rows of S_c
  if (r0 >= S.n_a) return;
  const int nr = min(64, S.n_a - r0);
  const T* u = vR + rhs * P.tot_r + S.r_off;
  for (int a = threadIdx.x; a < S.n_a; a += blockDim.x) {
    const int pb = P.a_ptr[S.a_off + a], pe = P.a_ptr[S.a_off + a + 1];
    double s = 0.0;
    for (int t = pb; t < pe; ++t) s += (double)u[P.a_r[t]];
    av[a] = (T)(s / (double)(pe - pb));
  }
  __syncthreads();
  // the product with this workgroup's 64 rows of S_c, the columns in four
  // groups (one per wave), partial sums combined in a fixed order
  const T* M = Sc + S.Sc_off + r0;
  T* part = av + P.max_na;
  gemv_split4<T>(M, S.n_a, nr, S.n_a, av, part, 64);
  for (int a = threadIdx.x; a < nr; a += blockDim.x)
    mu[rhs * P.tot_a + S.am_off + r0 + a] = -((part[a] + part[64 + a]) + (part[128 + a] + part[192 + a]));
}

// Sum over the wave (every lane gets it; lane 0's pairing is that of the
// shift-down tree), by register swaps and DPP: no LDS traffic.
__device__ __forceinline__ double wave_sum(double v) {
  v += xor_lane_f64<32>(v);
  v += xor_lane_f64<16>(v);
  v += xor_lane_f64<8>(v);
  v += xor_lane_f64<4>(v);
  v += xor_lane_f64<2>(v);
  v += xor_lane_f64<1>(v);
  return v;
}

// bci = Phi_Gamma^T g_Gamma.  Phi = Y' - X Lambda, and only its vertex
// columns are stored, so the products with g run over the n_a columns of X
// and the n_v vertex columns of Phi (n_c in all, as for Phi alone): a
// vertex column's product is its entry of bci; the products w = X_Gamma^T g
// (per average, in wv) become the average entries -Lambda^T w in
// k_coarse_rhs_avg.  One workgroup per (column chunk, subdomain, rhs), one
// wave per column.
constexpr int CRL_COLS = 16;

// Where product column q goes (X's column q < n_a to w, else the vertex
// q - n_a's entry of bci).
template <typename T>
__device__ __forceinline__ void crl_store(const PlanDev& P, const SubDev& S, int q, int rhs, T v, T* wv, T* bci) {
  if (q < S.n_a) wv[(int64_t)rhs * P.tot_a + S.am_off + q] = v;
  else bci[(int64_t)rhs * P.tot_c + S.c_off + P.v_c[S.v_off + q - S.n_a]] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_rhs_local(PlanDev P, const T* __restrict__ XG,
                                                          const T* __restrict__ PhiG,
                                                          const T* __restrict__ gv, T* __restrict__ wv,
                                                          T* __restrict__ bci) {
  extern __shared__ char smem_raw[];
  T* gl = reinterpret_cast<T*>(smem_raw);
  const int sub = blockIdx.y, rhs = blockIdx.z;
  const SubDev S = P.subs[sub];
  const int nq = S.n_a + S.n_v;
  const int cb = blockIdx.x * CRL_COLS;
  if (cb >= nq) return;
  const T* g = gv + rhs * P.tot_g + S.g_off;
  for (int e = threadIdx.x; e < S.n_g; e += blockDim.x) gl[e] = g[e];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int qend = min(nq, cb + CRL_COLS);
  auto column = [&](int q) {
    return q < S.n_a ? XG + S.XG_off + (int64_t)S.n_s * q : PhiG + S.PhiG_off + (int64_t)S.n_s * (q - S.n_a);
  };
  // two columns per wave at a time (q and q + nw), four loads in flight per
  // lane and column
  for (int q = cb + wave; q < qend; q += 2 * nw) {
    const int q2 = q + nw;
    const bool two = q2 < qend;
    const T* c1 = column(q);
    const T* c2 = two ? column(q2) : c1;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    int e = lane;
    for (; e + 192 < S.n_g; e += 256) {
      const T x0 = c1[e], x1 = c1[e + 64], x2 = c1[e + 128], x3 = c1[e + 192];
      const T y0 = c2[e], y1 = c2[e + 64], y2 = c2[e + 128], y3 = c2[e + 192];
      a0 += (double)(x0 * gl[e]);
      a1 += (double)(x1 * gl[e + 64]);
      a2 += (double)(x2 * gl[e + 128]);
      a3 += (double)(x3 * gl[e + 192]);
      b0 += (double)(y0 * gl[e]);
      b1 += (double)(y1 * gl[e + 64]);
      b2 += (double)(y2 * gl[e + 128]);
      b3 += (double)(y3 * gl[e + 192]);
    }
    for (; e < S.n_g; e += 64) {
      const T x0 = c1[e], y0 = c2[e];
      a0 += (double)(x0 * gl[e]);
      b0 += (double)(y0 * gl[e]);
    }
    const double acc1 = wave_sum((a0 + a1) + (a2 + a3));
    const double acc2 = wave_sum((b0 + b1) + (b2 + b3));
    if (lane == 0) {
      crl_store(P, S, q, rhs, (T)acc1, wv, bci);
      if (two) crl_store(P, S, q2, rhs, (T)acc2, wv, bci);
    }
  }
}

// The average entries of bci: -Lambda^T w with w = X_Gamma^T g, plus
// eps (sum of g over Gamma) on a pinned subdomain, whose Phi_r has the extra
// term 1 e^T / delta (eps = e / delta).  One workgroup per (chunk of 16
// averages, subdomain, rhs); each wave takes four columns of Lambda at once
// and loads w beside them (one round of loads).
constexpr int CRA_COLS = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_rhs_avg(PlanDev P, const T* __restrict__ Lam,
                                                        const double* __restrict__ eps, const T* __restrict__ gv,
                                                        const T* __restrict__ wv, T* __restrict__ bci) {
  __shared__ double red[256];
  const int sub = blockIdx.y, rhs = blockIdx.z;
  const SubDev S = P.subs[sub];
  const int na = S.n_a, j0 = blockIdx.x * CRA_COLS;
  if (j0 >= na) return;
  const T* ws = wv + (int64_t)rhs * P.tot_a + S.am_off;
  const bool pinned = S.pin >= 0;  // uniform over the workgroup
  double gsum = 0.0;
  if (pinned) {
    const T* g = gv + (int64_t)rhs * P.tot_g + S.g_off;
    double part = 0.0;
    for (int e = threadIdx.x; e < S.n_g; e += blockDim.x) part += (double)g[e];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    gsum = red[0];
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const T* L = Lam + S.T_off;
  int cc[4];
  double acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = j0 + 4 * wave + u;
    cc[u] = j < na ? P.a_c[S.am_off + j] : -1;
    acc[u] = 0.0;
  }
  for (int a = lane; a < na; a += 64) {
    T lv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) lv[u] = cc[u] >= 0 ? L[a + (int64_t)na * cc[u]] : (T)0;
    const double wa = (double)ws[a];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += (double)lv[u] * wa;
  }
  T* b = bci + (int64_t)rhs * P.tot_c + S.c_off;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double sum = wave_sum(acc[u]);
    if (lane == 0 && cc[u] >= 0) b[cc[u]] = (T)(pinned ? eps[S.am_off + cc[u]] * gsum - sum : -sum);
  }
}

// v2 on Gamma = v_Delta plus the coarse correction, u - X mu + Phi_Gamma u_c.
// With Phi = Y' - X Lambda this is u - X (mu + Lambda u_c) + Y' u_c, where
// Y' is nonzero only in the vertex columns: the rows of X and of Y' at the
// Gamma entries are read (n_a + n_v columns instead of n_a + n_c).  One
// workgroup per (chunk of 64 Gamma rows, subdomain, rhs): lane l of wave w
// takes row 64 chunk + l and the columns j = w mod 4, four loads in flight;
// wave 0 adds the four partial sums in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_v2(PlanDev P, const T* __restrict__ vR, const T* __restrict__ XG,
                                            const T* __restrict__ mu, const T* __restrict__ lu,
                                            const T* __restrict__ YG, const double* __restrict__ uc,
                                            T* __restrict__ v2) {
  extern __shared__ char smem_raw[];
  T* sh = reinterpret_cast<T*>(smem_raw);
  const int sub = blockIdx.y, rhs = blockIdx.z;
  const SubDev S = P.subs[sub];
  const int e0 = blockIdx.x * 64;
  if (e0 >= S.n_g) return;
  T* mul = sh;
  T* ucv = sh + P.max_na;
  T* part = ucv + P.max_nv + 1;  // [4][64]
  for (int a = threadIdx.x; a < S.n_a; a += blockDim.x)
    mul[a] = mu[rhs * P.tot_a + S.am_off + a] + lu[rhs * P.tot_a + S.am_off + a];
  for (int v = threadIdx.x; v < S.n_v; v += blockDim.x)
    ucv[v] = (T)uc[rhs * P.n_coarse + P.c_glob[S.c_off + P.v_c[S.v_off + v]]];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, e = e0 + lane;
  T acc = 0;
  if (e < S.n_g) {
    const T* X = XG + S.XG_off;
    const T* Y = YG + S.YG_off;
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int a = w;
    for (; a + 12 < S.n_a; a += 16) {
      a0 -= X[e + (int64_t)S.n_s * a] * mul[a];
      a1 -= X[e + (int64_t)S.n_s * (a + 4)] * mul[a + 4];
      a2 -= X[e + (int64_t)S.n_s * (a + 8)] * mul[a + 8];
      a3 -= X[e + (int64_t)S.n_s * (a + 12)] * mul[a + 12];
    }
    for (; a < S.n_a; a += 4) a0 -= X[e + (int64_t)S.n_s * a] * mul[a];
    for (int v = w; v < S.n_v; v += 4) a1 += Y[e + (int64_t)S.n_g * v] * ucv[v];
    acc = (a0 + a1) + (a2 + a3);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  if (w == 0 && e < S.n_g) {
    const T* u = vR + rhs * P.tot_r + S.r_off;
    const int r = P.g_r[S.g_off + e];
    const T base = r >= 0 ? u[r] : (T)0;
    v2[rhs * P.tot_g + S.g_off + e] = base + ((part[lane] + part[64 + lane]) + (part[128 + lane] + part[192 + lane]));
  }
}

// lu = Lambda u_c per subdomain and right-hand side: one workgroup per
// (subdomain, rhs, 64 rows of Lambda), the local coarse values staged in
// LDS, one lane per average row (Lambda read along its columns, four waves
// over the columns).
template <typename T>
__global__ __launch_bounds__(256) void k_lam_uc(PlanDev P, const T* __restrict__ Lam,
                                                const double* __restrict__ uc, T* __restrict__ lu) {
  extern __shared__ char smem_raw[];
  double* ucl = reinterpret_cast<double*>(smem_raw);
  const int sub = blockIdx.x, rhs = blockIdx.y;
  const SubDev S = P.subs[sub];
  const int r0 = blockIdx.z * 64;  // this workgroup's 64 rows of Lambda
  if (r0 >= S.n_a) return;
  const int nr = min(64, S.n_a - r0);
  for (int c = threadIdx.x; c < S.n_c; c += blockDim.x) ucl[c] = uc[rhs * P.n_coarse + P.c_glob[S.c_off + c]];
  __syncthreads();
  const T* L = Lam + S.T_off + r0;
  double* part = ucl + P.max_nc;
  gemv_split4<double>(L, S.n_a, nr, S.n_c, ucl, part, 64);
  for (int a = threadIdx.x; a < nr; a += blockDim.x)
    lu[rhs * P.tot_a + S.am_off + r0 + a] = (T)((part[a] + part[64 + a]) + (part[128 + a] + part[192 + a]));
}

// ---------------------------------------------------------------------------
// Pinned subdomains (floating, no primal point constraints; SubDev::pin).
// Their r-set leaves out one interior node, so K_rr is definite, and the
// local functions are w + c 1 with w = 0 at the pin: the constant c is one
// more unknown.  With d = C 1 (all ones: each average of the constant is 1),
// S = C_r K_rr^{-1} C_r^T, e = S^{-1} d and delta = d^T e, the constrained
// Neumann problem [K C^T; C 0] [v; mu] = [g; 0] has
//   mu = S^{-1} q + c e,  q = C_r K_rr^{-1} g_r,  c = (1^T g - d^T S^{-1} q) / delta,
//   v = K_rr^{-1} (g_r - C_r^T mu) + c 1,
// and the coarse basis (C Phi = I, minimal energy) has
//   Lambda = e e^T / delta - S^{-1},  Phi_r = -X Lambda + 1 e^T / delta,
// so K_c = Phi^T K Phi = -Lambda as with eliminated vertices.

// Setup, after Lambda = -S^{-1}: eps = e / delta, delta, Lambda += e e^T / delta.
template <typename T>
__global__ __launch_bounds__(256) void k_float_setup(PlanDev P, const T* __restrict__ Sc, T* __restrict__ Lam,
                                                     double* __restrict__ eps, double* __restrict__ fdelta) {
  extern __shared__ char smem_raw[];
  double* e = reinterpret_cast<double*>(smem_raw);
  __shared__ double red[256];
  const int sub = blockIdx.x;
  const SubDev S = P.subs[sub];
  if (S.pin < 0 || S.n_a == 0) return;
  const int na = S.n_a;
  // Sc holds -S^{-1} (both triangles) after its sweep
  double part = 0.0;
  for (int a = threadIdx.x; a < na; a += blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < na; ++b) acc -= (double)Sc[S.Sc_off + a + (int64_t)na * b];
    e[a] = acc;
    part += acc;
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double delta = red[0];
  for (int a = threadIdx.x; a < na; a += blockDim.x) eps[S.am_off + a] = e[a] / delta;
  if (threadIdx.x == 0) fdelta[sub] = delta;
  T* L = Lam + S.T_off;
  for (int idx = threadIdx.x; idx < na * na; idx += blockDim.x) {
    const int a = idx % na, c = idx / na;
    L[idx] = (T)((double)L[idx] + e[a] * e[c] / delta);
  }
}

// Apply, after mu = S^{-1} q: c = (1^T g - sum mu) / delta, mu += c e.
template <typename T>
__global__ __launch_bounds__(256) void k_float_mu(PlanDev P, const T* __restrict__ gv, T* __restrict__ mu,
                                                  const double* __restrict__ eps,
                                                  const double* __restrict__ fdelta, double* __restrict__ fc) {
  __shared__ double red[256];
  const int sub = blockIdx.x, rhs = blockIdx.y;
  const SubDev S = P.subs[sub];
  if (S.pin < 0) return;
  double part = 0.0;
  for (int e = threadIdx.x; e < S.n_g; e += blockDim.x) part += (double)gv[rhs * P.tot_g + S.g_off + e];
  T* m = mu + rhs * P.tot_a + S.am_off;
  for (int a = threadIdx.x; a < S.n_a; a += blockDim.x) part -= (double)m[a];
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double delta = fdelta[sub], c = red[0] / delta;
  for (int a = threadIdx.x; a < S.n_a; a += blockDim.x)
    m[a] = (T)((double)m[a] + c * delta * eps[S.am_off + a]);
  if (threadIdx.x == 0) fc[rhs * P.n_sub + sub] = c;
}

// Apply, after v2 on Gamma: add c + e^T u_c / delta (the constant of the
// Neumann solution and of Phi u_c).
template <typename T>
__global__ __launch_bounds__(256) void k_float_v2(PlanDev P, const double* __restrict__ uc,
                                                  const double* __restrict__ eps, const double* __restrict__ fc,
                                                  T* __restrict__ v2) {
  __shared__ double red[256];
  const int sub = blockIdx.x, rhs = blockIdx.y;
  const SubDev S = P.subs[sub];
  if (S.pin < 0) return;
  double part = 0.0;
  for (int a = threadIdx.x; a < S.n_a; a += blockDim.x)
    part += eps[S.am_off + a] * uc[rhs * P.n_coarse + P.c_glob[S.c_off + a]];
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double add = fc[rhs * P.n_sub + sub] + red[0];
  T* v = v2 + rhs * P.tot_g + S.g_off;
  for (int e = threadIdx.x; e < S.n_g; e += blockDim.x) v[e] = (T)((double)v[e] + add);
}

// The K_{I Gamma} entries (the Gamma neighbours the plan lists for each
// interior node): the neighbour's free index and the stiffness entry (from
// rho).  One thread per entry, so no thread walks a node's list.
__global__ void k_kig_fill(PlanDev P, Geo g, const double* __restrict__ rho) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= P.n_kig) return;
  const SubDev S = P.subs[P.kig_sub[e]];
  int c[3];
  loc_coords(S, P.I_loc[P.kig_own[e]], c);
  const int t = P.kig_t[e];
  const int cn[3] = {c[0] + t % 3 - 1, c[1] + (t / 3) % 3 - 1, c[2] + t / 9 - 1};
  P.kig_col[e] = (int32_t)free_of_local(S, g, loc_index(S, cn));
  P.kig_val[e] = kloc(S, g, rho, P.khat, c, cn);
}

// Interior right-hand side of the second Dirichlet solve: r_I - K_{I Gamma} w,
// from the entries the setup stored.
template <typename T>
__global__ void k_interior_rhs(PlanDev P, Geo g, const double* __restrict__ r, const double* __restrict__ w,
                               T* __restrict__ vI) {
  const int sub = blockIdx.y, rhs = blockIdx.z;
  const SubDev S = P.subs[sub];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n_I) return;
  const int64_t gi = S.I_off + i;
  const double* wr = w + rhs * g.n_free;
  double acc = r[rhs * g.n_free + free_of_local(S, g, P.I_loc[gi])];
  for (int e = P.kig_ptr[gi]; e < P.kig_ptr[gi + 1]; ++e) acc -= P.kig_val[e] * wr[P.kig_col[e]];
  vI[rhs * P.tot_I + gi] = (T)acc;
}

template <typename T>
__global__ void k_scatter_I(PlanDev P, Geo g, const T* __restrict__ vI, double* __restrict__ z) {
  const int sub = blockIdx.y, rhs = blockIdx.z;
  const SubDev S = P.subs[sub];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n_I) return;
  z[rhs * g.n_free + free_of_local(S, g, P.I_loc[S.I_off + i])] =
      (double)vI[rhs * P.tot_I + S.I_off + i];
}

// w = E v2 on Gamma (weighted sum over the subdomains sharing each node).
template <typename T>
__global__ void k_gamma_w(PlanDev P, Geo g, const T* __restrict__ v2, const double* __restrict__ delta,
                          double* __restrict__ z) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (q >= P.n_gam) return;
  double w = 0.0;
  for (int k = P.gam_eptr[q]; k < P.gam_eptr[q + 1]; ++k) {
    int ent = P.gam_ent[k];
    w += delta[ent] * (double)v2[rhs * P.tot_g + ent];
  }
  z[rhs * g.n_free + P.gam_node[q]] = w;
}

// ---- coarse multifrontal solve ------------------------------------------

// Forward-solve vectors of every front: a pivot's entry is the coarse
// right-hand side of its coarse dof, summed over the subdomains that share
// the dof (b_c = sum_i R_ci^T bci), the other entries 0.  Every coarse dof
// is the pivot of exactly one front.
template <typename T>
__global__ void k_front_vec_init(PlanDev P, const int32_t* __restrict__ fr, const T* __restrict__ bci,
                                 double* __restrict__ fvec, int64_t stride) {
  const FrontDev F = P.fronts[fr[blockIdx.y]];
  const int rhs = blockIdx.z;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= F.n) return;
  double v = 0.0;
  if (k < F.p) {
    const int c = P.front_idx[F.idx_off + k];
    for (int e = P.crs_eptr[c]; e < P.crs_eptr[c + 1]; ++e) v += (double)bci[rhs * P.tot_c + P.crs_ent[e]];
  }
  fvec[rhs * stride + F.voff + k] = v;
}

__global__ void k_front_vec_scatter(PlanDev P, const int32_t* __restrict__ ch, double* __restrict__ fvec,
                                    int64_t stride) {
  const FrontDev C = P.fronts[ch[blockIdx.y]];
  const FrontDev F = P.fronts[C.parent];
  const int rhs = blockIdx.z;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= C.n - C.p) return;
  fvec[rhs * stride + F.voff + P.front_pmap[C.pmap_off + k]] += fvec[rhs * stride + C.voff + C.p + k];
}

// z = F[:, :p] y_P; xh_P = -z_P (F_PP holds -G); y_B -= z_B (F_BP holds L~).
__global__ __launch_bounds__(256) void k_front_fwd(PlanDev P, const int32_t* __restrict__ fr,
                                                   const double* __restrict__ fpool,
                                                   double* __restrict__ fvec, double* __restrict__ xh,
                                                   int64_t stride) {
  __shared__ double yl[2048];
  const FrontDev F = P.fronts[fr[blockIdx.y]];
  const int rhs = blockIdx.z;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if ((int64_t)blockIdx.x * blockDim.x >= F.n || F.p == 0) return;
  const double* M = fpool + F.off;
  double* y = fvec + rhs * stride + F.voff;
  double acc = 0.0;
  for (int j0 = 0; j0 < F.p; j0 += 2048) {
    const int jn = min(2048, F.p - j0);
    __syncthreads();
    for (int j = threadIdx.x; j < jn; j += blockDim.x) yl[j] = y[j0 + j];
    __syncthreads();
    if (i < F.n)
      for (int j = 0; j < jn; ++j) acc += M[i + (int64_t)F.n * (j0 + j)] * yl[j];
  }
  __syncthreads();
  if (i >= F.n) return;
  if (i < F.p) xh[rhs * stride + F.voff + i] = -acc;
  else y[i] -= acc;
}

// Vector entry idx of one right-hand side (fv: its part of fvec) plus the
// children's border values it receives, added in slot order (the order of
// the scatter launches it replaces).
__device__ __forceinline__ double front_pulled(const PlanDev& P, const double* __restrict__ fv, int64_t idx) {
  double v = fv[idx];
  for (int j = 0; j < P.n_slot; ++j) {
    const int32_t src = P.front_pull[idx * P.n_slot + j];
    if (src >= 0) v += fv[src];
  }
  return v;
}

// The same forward step split over chunks of FK pivot columns, for one or a
// few right-hand sides: k_front_fwd_part writes the partial products of
// each chunk (64 rows x 4 column groups per workgroup, the groups summed in
// fixed order), k_front_fwd_fin sums the chunks in order and applies them.
// part[kc][rhs][front row] (kc-major, stride nrhs * stride per chunk).
constexpr int FK = 256;

// direct: every front of the launch has at most FK pivots (one chunk), and
// the chunk's sums are applied here as k_front_fwd_fin would (no part).
__global__ __launch_bounds__(256) void k_front_fwd_part(PlanDev P, const int32_t* __restrict__ fr,
                                                        const double* __restrict__ fpool,
                                                        double* __restrict__ fvec, int64_t stride, int nrhs,
                                                        double* __restrict__ part, int pull, int direct,
                                                        double* __restrict__ xh) {
  __shared__ double yl[FK];
  __shared__ double red[4][64];
  const FrontDev F = P.fronts[fr[blockIdx.z / nrhs]];
  const int rhs = blockIdx.z % nrhs;
  const int i0 = blockIdx.x * 64, kc = blockIdx.y, k0 = kc * FK;
  if (i0 >= F.n || k0 >= F.p) return;
  const int kn = min(FK, F.p - k0);
  const double* fv = fvec + rhs * stride;
  for (int j = threadIdx.x; j < FK; j += blockDim.x)
    yl[j] = j >= kn ? 0.0 : pull ? front_pulled(P, fv, F.voff + k0 + j) : fv[F.voff + k0 + j];
  __syncthreads();
  const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = i0 + r;
  double acc = 0.0;
  if (i < F.n) {
    const double* M = fpool + F.off + i + (int64_t)F.n * k0;
#pragma unroll 8
    for (int j = g; j < kn; j += 4) acc += M[(int64_t)F.n * j] * yl[j];
  }
  red[g][r] = acc;
  __syncthreads();
  if (g == 0 && i < F.n) {
    const double z = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
    if (direct) {
      const int64_t at = rhs * stride + F.voff + i;
      if (i < F.p) xh[at] = -z;
      else fvec[at] = (pull ? front_pulled(P, fvec + rhs * stride, F.voff + i) : fvec[at]) - z;
    } else {
      part[(int64_t)kc * nrhs * stride + rhs * stride + F.voff + i] = z;
    }
  }
}

__global__ __launch_bounds__(256) void k_front_fwd_fin(PlanDev P, const int32_t* __restrict__ fr,
                                                       double* __restrict__ fvec, double* __restrict__ xh,
                                                       int64_t stride, int nrhs, const double* __restrict__ part,
                                                       int pull) {
  const FrontDev F = P.fronts[fr[blockIdx.y]];
  const int rhs = blockIdx.z;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= F.n || F.p == 0) return;
  const int nkc = (F.p + FK - 1) / FK;
  double z = 0.0;
  for (int kc = 0; kc < nkc; ++kc) z += part[(int64_t)kc * nrhs * stride + rhs * stride + F.voff + i];
  const int64_t at = rhs * stride + F.voff + i;
  if (i < F.p) xh[at] = -z;
  else fvec[at] = (pull ? front_pulled(P, fvec + rhs * stride, F.voff + i) : fvec[at]) - z;
}

// x_P = xh_P - L~^T x_B, x_B from ancestors; one wave per pivot column.
__global__ __launch_bounds__(256) void k_front_bwd(PlanDev P, const int32_t* __restrict__ fr,
                                                   const double* __restrict__ fpool,
                                                   const double* __restrict__ xh, int64_t stride,
                                                   double* __restrict__ uc) {
  __shared__ double xb[2048];
  const FrontDev F = P.fronts[fr[blockIdx.y]];
  const int rhs = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = blockIdx.x * (blockDim.x >> 6) + wave;
  if ((int64_t)blockIdx.x * (blockDim.x >> 6) >= F.p) return;
  const int nb = F.n - F.p;
  const double* M = fpool + F.off;
  double acc = 0.0;
  for (int b0 = 0; b0 < nb; b0 += 2048) {
    const int bn = min(2048, nb - b0);
    __syncthreads();
    for (int b = threadIdx.x; b < bn; b += blockDim.x)
      xb[b] = uc[rhs * P.n_coarse + P.front_idx[F.idx_off + F.p + b0 + b]];
    __syncthreads();
    if (k < F.p)
      for (int b = lane; b < bn; b += 64) acc += M[(F.p + b0 + b) + (int64_t)F.n * k] * xb[b];
  }
  acc = wave_sum(acc);
  if (k < F.p && lane == 0)
    uc[rhs * P.n_coarse + P.front_idx[F.idx_off + k]] = xh[rhs * stride + F.voff + k] - acc;
}

// ---- products with many right-hand sides ----------------------------------
// The per-iteration products with the coarse basis rows (Phi_Gamma, X_Gamma)
// and with the coarse fronts, for groups of MR_COLS right-hand sides: one
// workgroup takes 64 output rows (4 waves x 16) and the group's columns; the
// right-hand sides are staged in LDS in chunks of MR_KC rows and each A
// element read from HBM feeds MR_COLS / 16 MFMAs.
constexpr int MR_KC = 128;

// acc[c] += sum_{k < kn} a(k) * Bs[k][16 c + rr]   (one wave, 16 output rows)
template <typename T, typename AF>
__device__ __forceinline__ void mr_accum(AF a_of, bool rok, int kn, const T (*Bs)[MR_COLS + 1],
                                         typename Mfma<T>::acc_t* acc, int kq, int rr) {
#pragma unroll 8
  for (int k4 = 0; k4 < MR_KC / 4; ++k4) {
    if (4 * k4 >= kn) break;
    const int k = 4 * k4 + kq;
    const T a = (rok && k < kn) ? a_of(k) : (T)0;
#pragma unroll
    for (int c = 0; c < MR_COLS / 16; ++c) acc[c] = Mfma<T>::mac(a, Bs[k][16 * c + rr], acc[c]);
  }
}

// The products of k_coarse_rhs_local for many right-hand sides: column q of
// [X_Gamma | Phi_Gamma's vertex columns] times g, stored by crl_store.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_rhs_local_mr(PlanDev P, const T* __restrict__ XG,
                                                             const T* __restrict__ PhiG,
                                                             const T* __restrict__ gv, T* __restrict__ wv,
                                                             T* __restrict__ bci, int nrhs) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T Bs[MR_KC][MR_COLS + 1];
  const int sub = blockIdx.y, r0 = blockIdx.z * MR_COLS, nr = min(MR_COLS, nrhs - r0);
  const SubDev S = P.subs[sub];
  const int nq = S.n_a + S.n_v;
  const int c0 = blockIdx.x * 64;
  if (c0 >= nq) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kq = lane >> 4, rr = lane & 15;
  const int qc = c0 + wave * 16 + rr;  // this lane's product column
  const bool rok = qc < nq;
  const T* M = !rok ? XG : qc < S.n_a ? XG + S.XG_off + (int64_t)S.n_s * qc
                                      : PhiG + S.PhiG_off + (int64_t)S.n_s * (qc - S.n_a);
  acc_t acc[MR_COLS / 16];
#pragma unroll
  for (int q = 0; q < MR_COLS / 16; ++q) acc[q] = acc_t{0, 0, 0, 0};
  for (int kb = 0; kb < S.n_g; kb += MR_KC) {
    const int kn = min(MR_KC, S.n_g - kb);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MR_KC * MR_COLS / 256; ++u) {
      const int idx = tid + u * 256, k = idx % MR_KC, r = idx / MR_KC;
      Bs[k][r] = (k < kn && r < nr) ? gv[(int64_t)(r0 + r) * P.tot_g + S.g_off + kb + k] : (T)0;
    }
    __syncthreads();
    mr_accum<T>([&](int k) { return M[kb + k]; }, rok, kn, Bs, acc, kq, rr);
  }
#pragma unroll
  for (int q = 0; q < MR_COLS / 16; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int cc = c0 + wave * 16 + Mfma<T>::row(kq, e), r = 16 * q + rr;
      if (cc < nq && r < nr) crl_store(P, S, cc, r0 + r, (T)acc[q][e], wv, bci);
    }
}

// v2 on Gamma = u - X_Gamma (mu + Lambda u_c) + Y'_Gamma u_c (as in k_v2),
// for 64 Gamma rows per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_v2_mr(PlanDev P, const T* __restrict__ vR, const T* __restrict__ XG,
                                               const T* __restrict__ mu, const T* __restrict__ lu,
                                               const T* __restrict__ YG, const double* __restrict__ uc,
                                               T* __restrict__ v2, int nrhs) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T Bs[MR_KC][MR_COLS + 1];
  const int sub = blockIdx.y, r0 = blockIdx.z * MR_COLS, nr = min(MR_COLS, nrhs - r0);
  const SubDev S = P.subs[sub];
  const int e0 = blockIdx.x * 64;
  if (e0 >= S.n_g) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kq = lane >> 4, rr = lane & 15;
  const int e = e0 + wave * 16 + rr;
  const bool rok = e < S.n_g;
  acc_t acc[MR_COLS / 16];
#pragma unroll
  for (int q = 0; q < MR_COLS / 16; ++q) acc[q] = acc_t{0, 0, 0, 0};
  for (int kb = 0; kb < S.n_v; kb += MR_KC) {   // + Y'_Gamma u_c (vertex columns)
    const int kn = min(MR_KC, S.n_v - kb);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MR_KC * MR_COLS / 256; ++u) {
      const int idx = tid + u * 256, k = idx % MR_KC, r = idx / MR_KC;
      Bs[k][r] = (k < kn && r < nr)
                     ? (T)uc[(int64_t)(r0 + r) * P.n_coarse + P.c_glob[S.c_off + P.v_c[S.v_off + kb + k]]]
                     : (T)0;
    }
    __syncthreads();
    const T* M = YG + S.YG_off + e + (int64_t)S.n_g * kb;
    mr_accum<T>([&](int k) { return M[(int64_t)S.n_g * k]; }, rok, kn, Bs, acc, kq, rr);
  }
  for (int kb = 0; kb < S.n_a; kb += MR_KC) {   // - X_Gamma (mu + Lambda u_c)
    const int kn = min(MR_KC, S.n_a - kb);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MR_KC * MR_COLS / 256; ++u) {
      const int idx = tid + u * 256, k = idx % MR_KC, r = idx / MR_KC;
      const int64_t at = (int64_t)(r0 + r) * P.tot_a + S.am_off + kb + k;
      Bs[k][r] = (k < kn && r < nr) ? -(mu[at] + lu[at]) : (T)0;
    }
    __syncthreads();
    const T* M = XG + S.XG_off + e + (int64_t)S.n_s * kb;
    mr_accum<T>([&](int k) { return M[(int64_t)S.n_s * k]; }, rok, kn, Bs, acc, kq, rr);
  }
#pragma unroll
  for (int q = 0; q < MR_COLS / 16; ++q)
#pragma unroll
    for (int ee = 0; ee < 4; ++ee) {
      const int row = e0 + wave * 16 + Mfma<T>::row(kq, ee), r = 16 * q + rr;
      if (row < S.n_g && r < nr) {
        const int rx = P.g_r[S.g_off + row];
        const T base = rx >= 0 ? vR[(int64_t)(r0 + r) * P.tot_r + S.r_off + rx] : (T)0;
        v2[(int64_t)(r0 + r) * P.tot_g + S.g_off + row] = base + acc[q][ee];
      }
    }
}

// Front forward step for many right-hand sides: z = F[:, :p] y_P; rows < p
// give xh_P = -z_P, rows >= p update y_B -= z_B.
__global__ __launch_bounds__(256) void k_front_fwd_mr(PlanDev P, const int32_t* __restrict__ fr,
                                                      const double* __restrict__ fpool, double* __restrict__ fvec,
                                                      double* __restrict__ xh, int64_t stride, int nrhs) {
  typedef Mfma<double>::acc_t acc_t;
  __shared__ double Bs[MR_KC][MR_COLS + 1];
  const FrontDev F = P.fronts[fr[blockIdx.y]];
  const int r0 = blockIdx.z * MR_COLS, nr = min(MR_COLS, nrhs - r0);
  const int i0 = blockIdx.x * 64;
  if (i0 >= F.n || F.p == 0) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kq = lane >> 4, rr = lane & 15;
  const int row = i0 + wave * 16 + rr;
  const bool rok = row < F.n;
  acc_t acc[MR_COLS / 16];
#pragma unroll
  for (int q = 0; q < MR_COLS / 16; ++q) acc[q] = acc_t{0, 0, 0, 0};
  for (int kb = 0; kb < F.p; kb += MR_KC) {
    const int kn = min(MR_KC, F.p - kb);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MR_KC * MR_COLS / 256; ++u) {
      const int idx = tid + u * 256, k = idx % MR_KC, r = idx / MR_KC;
      Bs[k][r] = (k < kn && r < nr) ? fvec[(int64_t)(r0 + r) * stride + F.voff + kb + k] : 0.0;
    }
    __syncthreads();
    const double* M = fpool + F.off + row + (int64_t)F.n * kb;
    mr_accum<double>([&](int k) { return M[(int64_t)F.n * k]; }, rok, kn, Bs, acc, kq, rr);
  }
  __syncthreads();  // every workgroup of this front reads rows < p only; rows >= p are written below
#pragma unroll
  for (int q = 0; q < MR_COLS / 16; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + wave * 16 + Mfma<double>::row(kq, e), r = 16 * q + rr;
      if (i < F.n && r < nr) {
        const int64_t at = (int64_t)(r0 + r) * stride + F.voff + i;
        if (i < F.p) xh[at] = -acc[q][e];
        else fvec[at] -= acc[q][e];
      }
    }
}

// Front backward step for many right-hand sides: x_P = xh_P - L~^T x_B with
// x_B (the ancestors' coarse unknowns) gathered from u_c.
__global__ __launch_bounds__(256) void k_front_bwd_mr(PlanDev P, const int32_t* __restrict__ fr,
                                                      const double* __restrict__ fpool,
                                                      const double* __restrict__ xh, int64_t stride,
                                                      double* __restrict__ uc, int nrhs) {
  typedef Mfma<double>::acc_t acc_t;
  __shared__ double Bs[MR_KC][MR_COLS + 1];
  const FrontDev F = P.fronts[fr[blockIdx.y]];
  const int r0 = blockIdx.z * MR_COLS, nr = min(MR_COLS, nrhs - r0);
  const int i0 = blockIdx.x * 64;
  if (i0 >= F.p) return;
  const int nb = F.n - F.p;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kq = lane >> 4, rr = lane & 15;
  const int row = i0 + wave * 16 + rr;   // pivot index
  const bool rok = row < F.p;
  acc_t acc[MR_COLS / 16];
#pragma unroll
  for (int q = 0; q < MR_COLS / 16; ++q) acc[q] = acc_t{0, 0, 0, 0};
  for (int kb = 0; kb < nb; kb += MR_KC) {
    const int kn = min(MR_KC, nb - kb);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MR_KC * MR_COLS / 256; ++u) {
      const int idx = tid + u * 256, k = idx % MR_KC, r = idx / MR_KC;
      Bs[k][r] = (k < kn && r < nr)
                     ? uc[(int64_t)(r0 + r) * P.n_coarse + P.front_idx[F.idx_off + F.p + kb + k]] : 0.0;
    }
    __syncthreads();
    // L~^T[row][b] = F[p + b][row]
    const double* M = fpool + F.off + F.p + kb + (int64_t)F.n * row;
    mr_accum<double>([&](int k) { return M[k]; }, rok, kn, Bs, acc, kq, rr);
  }
#pragma unroll
  for (int q = 0; q < MR_COLS / 16; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + wave * 16 + Mfma<double>::row(kq, e), r = 16 * q + rr;
      if (i < F.p && r < nr)
        uc[(int64_t)(r0 + r) * P.n_coarse + P.front_idx[F.idx_off + i]] =
            xh[(int64_t)(r0 + r) * stride + F.voff + i] - acc[q][e];
    }
}

// ---- PCG vectors ----------------------------------------------------------

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ a,
                                                     const double* __restrict__ b, int64_t n,
                                                     double* __restrict__ partial) {
  __shared__ double sh[4];
  const int rhs = blockIdx.y;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  const double* ar = a + rhs * n;
  const double* br = b + rhs * n;
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += ar[i] * br[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[rhs * gridDim.x + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ partial, int nb,
                                                   double* __restrict__ out) {
  __shared__ double sh[4];
  const int rhs = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[rhs * nb + i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[rhs] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void k_pcg_xr(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                         const double* __restrict__ q, const double* __restrict__ rz,
                         const double* __restrict__ pq, const int32_t* __restrict__ active, int64_t n) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  const double alpha = rz[rhs] / pq[rhs];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t k = rhs * n + i;
  x[k] += alpha * p[k];
  r[k] -= alpha * q[k];
}

__global__ void k_pcg_p(double* __restrict__ p, const double* __restrict__ z,
                        const double* __restrict__ num, const double* __restrict__ den,
                        const int32_t* __restrict__ active, int64_t n) {
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  const double beta = num[rhs] / den[rhs];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t k = rhs * n + i;
  p[k] = z[k] + beta * p[k];
}

// ---- gradient and filter ---------------------------------------------------

__global__ void k_element_grad(Geo g, const double* __restrict__ khat, const double* __restrict__ rho,
                               const double* __restrict__ u, const double* __restrict__ lam,
                               double* __restrict__ out, int nrhs) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= g.n_elem) return;
  const int ex = (int)(e % g.ne[0]);
  const int ey = (int)((e / g.ne[0]) % g.ne[1]);
  const int ez = (int)(e / ((int64_t)g.ne[0] * g.ne[1]));
  const int nn = g.dim == 3 ? 8 : 4;
  int64_t fid[8];
  for (int a = 0; a < nn; ++a) {
    int x = ex + (a & 1), y = ey + ((a >> 1) & 1), z = g.dim == 3 ? ez + ((a >> 2) & 1) : 1;
    bool ok = x >= 1 && y >= 1 && x <= g.nf[0] && y <= g.nf[1] && (g.dim == 2 || (z >= 1 && z <= g.nf[2]));
    fid[a] = ok ? (x - 1) + (int64_t)g.nf[0] * ((y - 1) + (int64_t)g.nf[1] * (z - 1)) : -1;
  }
  double s = 0.0;
  for (int rhs = 0; rhs < nrhs; ++rhs) {
    double ue[8], le[8];
    for (int a = 0; a < nn; ++a) {
      ue[a] = fid[a] >= 0 ? u[rhs * g.n_free + fid[a]] : 0.0;
      le[a] = fid[a] >= 0 ? lam[rhs * g.n_free + fid[a]] : 0.0;
    }
    for (int a = 0; a < nn; ++a) {
      double t = 0.0;
      for (int b = 0; b < nn; ++b) t += khat[(a | (g.dim == 2 ? 4 : 0)) * 8 + (b | (g.dim == 2 ? 4 : 0))] * ue[b];
      s += le[a] * t;
    }
  }
  out[e] = -rho[e] * s;
}

__device__ __forceinline__ int filter_count(const Geo& g, int ex, int ey, int ez) {
  int cx = (ex > 0) + 1 + (ex < g.ne[0] - 1);
  int cy = (ey > 0) + 1 + (ey < g.ne[1] - 1);
  int cz = g.dim == 3 ? (ez > 0) + 1 + (ez < g.ne[2] - 1) : 1;
  return cx * cy * cz;
}

// mode 0: out = F in (the 3^dim box mean over in-domain neighbours);
// mode 1: out = F^T in; mode 2: out = exp(F in), the coefficient of a
// log-coefficient field.
__global__ void k_box_filter(Geo g, const double* __restrict__ in, double* __restrict__ out, int mode) {
  const bool transpose = mode == 1;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= g.n_elem) return;
  const int ex = (int)(e % g.ne[0]);
  const int ey = (int)((e / g.ne[0]) % g.ne[1]);
  const int ez = (int)(e / ((int64_t)g.ne[0] * g.ne[1]));
  const int zr = g.dim == 3 ? 1 : 0;
  double s = 0.0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int x = ex + dx, y = ey + dy, z = ez + dz;
        if (x < 0 || y < 0 || z < 0 || x >= g.ne[0] || y >= g.ne[1] || z >= g.ne[2]) continue;
        int64_t e2 = x + (int64_t)g.ne[0] * (y + (int64_t)g.ne[1] * z);
        s += transpose ? in[e2] / (double)filter_count(g, x, y, z) : in[e2];
      }
  if (transpose) out[e] = s;
  else {
    const double m = s / (double)filter_count(g, ex, ey, ez);
    out[e] = mode == 2 ? exp(m) : m;
  }
}

}  // namespace

// ===========================================================================
// launchers

#define LAUNCH_CHECK() (void)hipGetLastError()

void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s, int max_blocks) {
  if (n <= 0) return;
  k_fill<double><<<hmin(cdiv(n, 256), (int64_t)max_blocks), 256, 0, s>>>(p, n, v);
}
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return;
  k_fill<float><<<hmin(cdiv(n, 256), 65536), 256, 0, s>>>(p, n, v);
}
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  k_fill<int32_t><<<hmin(cdiv(n, 256), 65536), 256, 0, s>>>(p, n, v);
}
void launch_kc_to_f64(const float* src, double* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_f32_to_f64<<<hmin(cdiv(n, 256), 65536), 256, 0, s>>>(src, dst, n);
}
// Largest LDS footprint (static + dynamic, bytes) of any kernel launched for
// a plan with these maxima and element size; LDS per workgroup is 160 KiB.
int front_fwd_chunks(int maxp) { return (int)cdiv(maxp, FK); }

// columns of Phi staged per workgroup of the local coarse matrices (<= 64 KB)
// The vertex stencils go to LDS too when they are small (up to 24 KB); with
// many vertices (every interface node primal) they are read from memory.
bool kc_stage_stencils(const PlanDev& P) { return (int64_t)P.max_nv * 27 * 12 <= 24576; }
int kc_cols(const PlanDev& P) {
  const int64_t stencils = kc_stage_stencils(P) ? (int64_t)P.max_nv * 27 * 12 : 0;
  return (int)hmax((int64_t)1, hmin((int64_t)8, (65536 - stencils) / ((int64_t)hmax(P.max_ns, 1) * 8)));
}
int64_t kc_lds_bytes(const PlanDev& P) {
  return (int64_t)kc_cols(P) * hmax(P.max_ns, 1) * 8 + (kc_stage_stencils(P) ? (int64_t)P.max_nv * 27 * 12 : 0);
}

int64_t max_lds_bytes(const PlanDev& P, int elt, int max_nrhs) {
  const int64_t mp = hmax(P.max_plane, 1);
  int64_t need = 0;
  need = hmax(need, mp * (SC_COLS + 1) * elt + 2048);                                  // schur couple
  need = hmax(need, mp * (CPL_COLS + 1) * elt);                                        // couple multi
  need = hmax(need, (int64_t)hmax(P.max_block, 1) * ((BS_WAVES_MAX + 9) * 8 + 2 * elt));  // block solve
  if (max_nrhs >= P.mr_min) need = hmax(need, (int64_t)hmax(P.max_block, 1) * (MR_COLS + 1) * elt);  // many-rhs block solve
  need = hmax(need, (int64_t)(P.max_na + P.max_nc + 1) * elt);                         // v2
  need = hmax(need, (int64_t)hmax(P.max_ng, 1) * elt);                                 // coarse rhs
  need = hmax(need, (int64_t)hmax(P.max_ns, 1) * elt + (int64_t)P.max_nar * 4);        // object means
  need = hmax(need, kc_lds_bytes(P));                                                  // local coarse matrices
  need = hmax(need, (int64_t)SWEEP_ROWS * (SWEEP_NB + 1) * elt + 2 * 32 * 33 * 8);   // sweep panel
  return need;
}

void launch_copy16(const void* a, void* b, int64_t n16, hipStream_t s) {
  if (n16 <= 0) return;
  k_copy16<<<hmin(cdiv(n16, 256), 65536), 256, 0, s>>>((const int4*)a, (int4*)b, n16);
}
void launch_sub(const double* a, const double* b, double* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_sub<<<hmin(cdiv(n, 256), 65536), 256, 0, s>>>(a, b, out, n);
}

void launch_q1_apply(const Geo& g, const double* khat, const double* rho, const double* x,
                     double* y, int nrhs, hipStream_t s) {
  if (g.dim == 3) {
    const int txn = (int)cdiv(g.nf[0], QX), tyn = (int)cdiv(g.nf[1], QY), tzn = (int)cdiv(g.nf[2], QZ);
    const int ntile = txn * tyn * tzn;
    const unsigned nblk = (unsigned)((ntile + 7) / 8 * 8);
    k_q1_apply3<<<dim3(nblk, nrhs), 256, 0, s>>>(g, khat, rho, x, y, txn, tyn, ntile);
    return;
  }
  k_q1_apply<<<dim3(cdiv(g.n_free, 256), nrhs), 256, 0, s>>>(g, khat, rho, x, y);
}

void launch_alpha(const PlanDev& P, int n_ss, const double* rho, int weighting, double* alpha,
                  hipStream_t s) {
  k_alpha<<<cdiv(n_ss, 256), 256, 0, s>>>(P, n_ss, rho, weighting, alpha);
}
void launch_delta(const PlanDev& P, const double* alpha, double* delta, hipStream_t s) {
  if (P.tot_g == 0) return;
  k_delta<<<cdiv(P.tot_g, 256), 256, 0, s>>>(P, alpha, delta);
}
void launch_coupling_coefs(const PlanDev& P, const Geo& g, const double* rho, double* coef, double* icoef,
                           hipStream_t s) {
  if (P.n_cpl == 0) return;
  k_coupling_coefs<<<cdiv(P.n_cpl, CPL_ROWS), CPL_ROWS, 0, s>>>(P, g, rho, coef, icoef);
}

template <typename T>
void Kern<T>::block_assemble(const PlanDev& P, const Geo& g, const double* rho, int setR, T* G, int max_nb,
                             hipStream_t s) {
  if (max_nb == 0 || P.max_block == 0) return;
  k_block_zero_lower<T><<<dim3(max_nb, P.n_sub), 256, 0, s>>>(P, setR, G);
  const int mx = setR ? P.max_nr : P.max_nI;
  k_block_assemble<T><<<dim3(cdiv(mx, 128), P.n_sub), 128, 0, s>>>(P, g, rho, setR, G);
}

template <typename T>
void Kern<T>::schur_couple(const PlanDev& P, int setR, int k, T* G, hipStream_t s) {
  const int mp = P.max_plane;
  if (P.n_sub <= 0 || mp <= 0) return;
  const size_t sm = (size_t)mp * (SC_COLS + 1) * sizeof(T);
  const int nch = (int)cdiv(mp, SC_COLS);
  const unsigned nblk = (unsigned)(((int64_t)nch * P.n_sub + 7) / 8 * 8);
  k_schur_couple<T><<<nblk, 256, sm, s>>>(P, setR, k, G, nch);
}

template <typename T>
void Kern<T>::sweep(SweepDesc* d_desc, const SweepDesc* h_desc, int nprob, int maxn, int maxp, T* pool,
                    T* scratch, int64_t scr_stride, int* status, int status_code, hipStream_t s,
                    Profiler* prof, const SweepAux* aux, int reg_max, int lookahead, int utile, int slab_w) {
  if (nprob == 0 || maxp == 0) return;
  if (maxn <= hmin(reg_max, 16 * RS_MAX_TILES)) {
    // register-resident: one workgroup per matrix, read once, written once
    double f = 0, by = 0;
    if (prof && h_desc)
      for (int q = 0; q < nprob; ++q) {
        const double n = h_desc[q].n, p = h_desc[q].p;
        f += n * n * p;
        by += sizeof(T) * (n * (n + 1) / 2 + n * n);
      }
    if (prof) prof->begin(5, s);
    // waves per workgroup: more waves for mid sizes, where the tiles per wave
    // and so the registers per lane stay low enough
    const int mt = (int)cdiv(maxn, 16);
    if (mt <= 4) k_sweep_reg<T, 4, 8><<<nprob, 8 * 64, 0, s>>>(d_desc, pool, status, status_code, -1);
    else if (mt <= 8) k_sweep_reg<T, 8, 8><<<nprob, 8 * 64, 0, s>>>(d_desc, pool, status, status_code, -1);
    else if (mt <= 11) k_sweep_reg<T, 11, 8><<<nprob, 8 * 64, 0, s>>>(d_desc, pool, status, status_code, -1);
    else if (mt <= 12) k_sweep_reg<T, 12, 12><<<nprob, 12 * 64, 0, s>>>(d_desc, pool, status, status_code, -1);
    else if (mt <= 17) k_sweep_reg<T, 17, 8><<<nprob, 8 * 64, 0, s>>>(d_desc, pool, status, status_code, -1);
    else k_sweep_reg<T, RS_MAX_TILES, 8><<<nprob, 8 * 64, 0, s>>>(d_desc, pool, status, status_code, -1);
    if (prof) prof->end(5, f, by, s);
    return;
  }
  if (scr_stride >= (int64_t)maxn * SLAB) {
    // slabs of sl pivots: register sweep of the diagonal block, CD, rank-sl update
    static_assert(SLAB <= 16 * 12, "slab diagonal blocks use the 12-tile register sweep");
    // Slab width: 192 pivots, or 96 for a few matrices whose first trailing
    // update is short (a chain where the one-workgroup pivot-block sweeps
    // dominate: a 96-pivot block sweeps in about a fifth of the time of a
    // 192-pivot one, for twice the slabs)
    int sl = SLAB;
    if (slab_w == 96) sl = 96;
    else if (slab_w == 0 && nprob <= 4 && h_desc) {
      double uf0 = 0;
      for (int q = 0; q < nprob; ++q) {
        const double m = h_desc[q].n - std::min<double>(SLAB, h_desc[q].p);
        uf0 += 2.0 * SLAB * m * (m + 1) / 2;
      }
      if (uf0 < kSlabInlineFlops) sl = 96;
    }
    const int64_t tiles = cdiv(maxn, TILE);
    const int64_t ntri = tiles * (tiles + 1) / 2;
    // with a second stream: the next slab's pivot block is updated first and
    // swept on s2 while the rest of the trailing update runs on s
    auto reg = [&](int j0, hipStream_t ss) {
      double df = 0, db = 0;
      if (prof && h_desc)
        for (int q = 0; q < nprob; ++q) {
          const double p = h_desc[q].p;
          if (j0 >= p) continue;
          const double sb = std::min<double>(sl, p - j0);
          df += sb * sb * sb;
          db += sizeof(T) * (sb * (sb + 1) / 2 + sb * sb);
        }
      // booked with the panel work (class 4): one workgroup per front sweeps
      // the slab's pivot block, a latency chain rather than a batch
      if (prof) prof->begin(4, ss);
      if (sl == 96) k_sweep_reg<T, 6, 8><<<nprob, 8 * 64, 0, ss>>>(d_desc, pool, status, status_code, j0, 96);
      else k_sweep_reg<T, SLAB / 16, 16><<<nprob, 16 * 64, 0, ss>>>(d_desc, pool, status, status_code, j0, SLAB);
      if (prof) prof->end(4, df, db, ss);
    };
    // Two orders for a slab with a look-ahead (u1: the next pivot block's
    // update, u2: the rest of the trailing update, wb: the writeback):
    //   s: cd u1 u2 wb | s2: reg(next)  when the rest is the longer branch;
    //   s: cd u1 reg(next) | s2: u2 wb  when the sweep is, so the chain of
    //   pivot-block sweeps and CD products runs on one stream without
    //   cross-stream hand-offs, and the sweep is dispatched before u2 fills
    //   the compute units.
    // The next slab's CD product waits for the branch on s2.
    reg(0, s);
    bool prev_inl = false;
    for (int j0 = 0; j0 < maxp; j0 += sl) {
      double cf = 0, cb = 0, uf = 0, ub = 0;
      for (int q = 0; h_desc && q < nprob; ++q) {
        const double n = h_desc[q].n, p = h_desc[q].p;
        if (j0 >= p) continue;
        const double sb = std::min<double>(sl, p - j0), m = n - sb;
        const double low = m * (m + 1) / 2;
        cf += 2.0 * m * sb * sb;
        cb += sizeof(T) * (2.0 * m * sb + sb * sb);
        uf += 2.0 * sb * low;
        ub += sizeof(T) * (2.0 * low + 2.0 * m * sb);
      }
      if (aux && j0 > 0) (void)hipStreamWaitEvent(s, prev_inl ? aux->c : aux->b, 0);
      if (prof) prof->begin(4, s);
      k_slab_cd<T><<<dim3(cdiv(maxn, TILE), cdiv(sl, TILE), nprob), 256, 0, s>>>(d_desc, pool, j0, scratch,
                                                                                scr_stride, sl);
      if (prof) prof->end(4, cf, cb, s);
      // trailing update by 64- or 128-row tiles of the lower triangle
      const int64_t utiles = cdiv(maxn, utile == 128 ? UT : TILE), untri = utiles * (utiles + 1) / 2;
      const unsigned ublk = (unsigned)((untri * nprob + 7) / 8 * 8);
      auto upd = [&](int region, hipStream_t ss) {
        if (utile == 128)
          k_slab_update128<T><<<ublk, 256, 0, ss>>>(d_desc, pool, j0, scratch, scr_stride, (int)untri, nprob, region,
                                                    sl);
        else
          k_slab_update<T><<<ublk, 256, 0, ss>>>(d_desc, pool, j0, scratch, scr_stride, (int)untri, nprob, region,
                                                 sl);
      };
      const unsigned wgrid = (unsigned)hmin(cdiv((int64_t)maxn * sl, 256), 2048);
      const bool next = j0 + sl < maxp;
      prev_inl = false;
      if (next && aux && lookahead != 1) {
        const bool inl = lookahead == 2 || (h_desc && uf < kSlabInlineFlops);
        if (prof) prof->begin(1, s);
        upd(1, s);
        if (prof) prof->end(1, 0.0, 0.0, s);
        (void)hipEventRecord(aux->a, s);
        (void)hipStreamWaitEvent(aux->s2, aux->a, 0);
        hipStream_t su = inl ? aux->s2 : s;
        if (inl) reg(j0 + sl, s);
        else {
          reg(j0 + sl, aux->s2);
          (void)hipEventRecord(aux->b, aux->s2);
        }
        if (prof) prof->begin(1, su);
        upd(2, su);
        if (prof) prof->end(1, uf, ub, su);
        k_slab_writeback<T><<<dim3(wgrid, nprob), 256, 0, su>>>(d_desc, pool, j0, scratch, scr_stride, sl);
        if (inl) (void)hipEventRecord(aux->c, aux->s2);
        prev_inl = inl;
      } else {
        if (prof) prof->begin(1, s);
        upd(0, s);
        if (prof) prof->end(1, uf, ub, s);
        k_slab_writeback<T><<<dim3(wgrid, nprob), 256, 0, s>>>(d_desc, pool, j0, scratch, scr_stride, sl);
        if (next) reg(j0 + sl, s);
      }
    }
    const int64_t st = cdiv(maxp, 32);
    k_symmetrize<T><<<dim3((unsigned)hmin(st * (st + 1) / 2, 4096), nprob), 256, 0, s>>>(d_desc, pool, 0);
    return;
  }
  const int64_t tiles = cdiv(maxn, TILE);
  const dim3 pgrid(cdiv(maxn, SWEEP_ROWS), nprob);
  const size_t psm = (size_t)hmin(maxn, SWEEP_ROWS) * (SWEEP_NB + 1) * sizeof(T);
  int prev = -1;
  for (int j0 = 0; j0 < maxp; j0 += SWEEP_NB) {
    double pf = 0, pby = 0, uf = 0, uby = 0;
    if (prof && h_desc)
      for (int q = 0; q < nprob; ++q) {
        const double n = h_desc[q].n, p = h_desc[q].p;
        if (j0 >= p) continue;
        const double jb = std::min<double>(SWEEP_NB, p - j0), m = n - jb;
        const double low = m * (m + 1) / 2;  // lower-triangle entries outside the panel
        pf += 2.0 * m * jb * jb;
        pby += sizeof(T) * (2.0 * m * jb + jb * jb);
        uf += 2.0 * jb * low;
        uby += sizeof(T) * (2.0 * low + 2.0 * n * jb);
      }
    if (prof) prof->begin(4, s);
    k_sweep_panel<T><<<pgrid, 256, psm, s>>>(d_desc, pool, j0, prev, scratch, scr_stride, status, status_code);
    if (prof) prof->end(4, pf, pby, s);
    if (prof) prof->begin(1, s);
    const int64_t ntri = tiles * (tiles + 1) / 2;
    k_sweep_update<T><<<(unsigned)((ntri * nprob + 7) / 8 * 8), 256, 0, s>>>(d_desc, pool, j0, scratch, scr_stride,
                                                                            (int)ntri, nprob);
    if (prof) prof->end(1, uf, uby, s);
    prev = j0;
  }
  k_sweep_panel<T><<<pgrid, 256, psm, s>>>(d_desc, pool, -1, prev, scratch, scr_stride, status, status_code);
  const int64_t st = cdiv(maxp, 32);
  k_symmetrize<T><<<dim3((unsigned)hmin(st * (st + 1) / 2, 4096), nprob), 256, 0, s>>>(d_desc, pool, 0);
}

template <typename T>
void Kern<T>::gemm(const GemmDesc* d_desc, const GemmDesc* h_desc, int nprob, int maxm, int maxn, const T* A,
                   int transA, const T* B, int transB, T* C, T alpha, T beta, hipStream_t s, Profiler* prof) {
  if (nprob == 0 || maxm == 0 || maxn == 0) return;
  int tm = (int)cdiv(maxm, TILE), tn = (int)cdiv(maxn, TILE);
  double f = 0, by = 0;
  if (prof && h_desc)
    for (int q = 0; q < nprob; ++q) {
      const double m = h_desc[q].m, n = h_desc[q].n, kk = h_desc[q].k;
      f += 2.0 * m * n * kk;
      by += sizeof(T) * (m * kk + kk * n + m * n * (beta == (T)0 ? 1.0 : 2.0));
    }
  const unsigned nb = (unsigned)(((int64_t)tm * tn * nprob + 7) / 8 * 8);
  if (prof) prof->begin(3, s);
  if (!transA && !transB && maxm <= GF_M) {
    if (maxn > GF_N && maxn <= GF_N3)
      k_gemm_full<T, GF_KC3, GF_N3><<<dim3(nprob, 1), 1024, 0, s>>>(d_desc, A, B, C, alpha, beta);
    else
      k_gemm_full<T, GF_KC, GF_N><<<dim3(nprob, cdiv(maxn, GF_N)), 1024, 0, s>>>(d_desc, A, B, C, alpha, beta);
    if (prof) prof->end(3, f, by, s);
    return;
  }
  if (!transA && !transB) k_gemm<T, 0, 0><<<nb, 256, 0, s>>>(d_desc, A, B, C, alpha, beta, tm, tn, nprob);
  else if (transA && !transB) k_gemm<T, 1, 0><<<nb, 256, 0, s>>>(d_desc, A, B, C, alpha, beta, tm, tn, nprob);
  else if (!transA && transB) k_gemm<T, 0, 1><<<nb, 256, 0, s>>>(d_desc, A, B, C, alpha, beta, tm, tn, nprob);
  else k_gemm<T, 1, 1><<<nb, 256, 0, s>>>(d_desc, A, B, C, alpha, beta, tm, tn, nprob);
  if (prof) prof->end(3, f, by, s);
}

template <typename T>
void Kern<T>::rhs_fill(const PlanDev& P, const Geo& g, const double* rho, T* Z, hipStream_t s) {
  if (P.max_zcols == 0) return;
  k_rhs_fill<T><<<dim3(cdiv(P.max_zcols, 64), P.n_sub), 64, 0, s>>>(P, g, rho, Z);
}

template <typename T>
void Kern<T>::couple_multi(const PlanDev& P, const Geo& g, const double* rho, int k, int fwd,
                           int ncols_max, T* Z, T* tmp, int64_t tmp_stride, hipStream_t s, int sub0, int nsub) {
  (void)g;
  (void)rho;
  if (ncols_max == 0 || nsub <= 0) return;
  const size_t sm = (size_t)hmax(P.max_plane, 1) * (CPL_COLS + 1) * sizeof(T);
  k_couple_multi<T><<<dim3(cdiv(ncols_max, CPL_COLS), nsub), 256, sm, s>>>(P, k, fwd, Z, tmp, tmp_stride, sub0);
}

template <typename T>
void Kern<T>::object_means(const PlanDev& P, const T* Z, T* XG, T* Sc, T* Tv, T* PhiG, T* YG, hipStream_t s) {
  if (P.n_sub == 0 || P.max_nc == 0) return;
  const int ld = hmax(P.max_ns, 1);
  const int64_t col = (int64_t)ld * sizeof(T), idx = (int64_t)P.max_nar * 4;
  const int ncol = P.max_na + P.max_nc;
  // at most 24 KB of LDS per workgroup: more resident workgroups (gathers
  // in flight) count for more than fewer re-reads of the index arrays
  if (8 * col + idx <= 24 * 1024)
    k_object_means<T, 8><<<dim3(cdiv(ncol, 8), P.n_sub), 256, 8 * col + idx, s>>>(P, Z, XG, Sc, Tv, PhiG, YG, ld);
  else if (4 * col + idx <= 24 * 1024)
    k_object_means<T, 4><<<dim3(cdiv(ncol, 4), P.n_sub), 256, 4 * col + idx, s>>>(P, Z, XG, Sc, Tv, PhiG, YG, ld);
  else if (2 * col + idx <= 24 * 1024)
    k_object_means<T, 2><<<dim3(cdiv(ncol, 2), P.n_sub), 256, 2 * col + idx, s>>>(P, Z, XG, Sc, Tv, PhiG, YG, ld);
  else
    k_object_means<T, 1><<<dim3(ncol, P.n_sub), 256, col + idx, s>>>(P, Z, XG, Sc, Tv, PhiG, YG, ld);
}

template <typename T>
void Kern<T>::lam_assemble(const PlanDev& P, const T* Sc, const T* LV, T* Lam, hipStream_t s) {
  const int64_t tot = (int64_t)P.max_na * P.max_nc;
  if (tot == 0) return;
  k_lam_assemble<T><<<dim3(cdiv(tot, 256), P.n_sub), 256, 0, s>>>(P, Sc, LV, Lam);
}

template <typename T>
void Kern<T>::kc_identity(const PlanDev& P, const Geo& g, const double* rho, const T* PhiR, const T* Lam, T* Kc,
                          double* vcoef, int32_t* vcode, int max_nv, hipStream_t s) {
  (void)g;
  (void)rho;
  if (P.max_nc == 0) return;
  const int cols = kc_cols(P);
  if (max_nv > 0)
    k_kc_identity<T><<<dim3(cdiv(max_nv, cols), P.n_sub), 256, (size_t)kc_lds_bytes(P), s>>>(
        P, PhiR, vcoef, vcode, Kc, cols, kc_stage_stencils(P) ? 1 : 0);
  const int nt = cdiv(P.max_nc, 32);
  k_kc_symmetrize<T><<<dim3(nt * (nt + 1) / 2, P.n_sub), 256, 0, s>>>(P, Lam, Kc);
}

void launch_vertex_stencil(const PlanDev& P, const Geo& g, const double* rho, double* vcoef, int32_t* vcode,
                           int max_nv, hipStream_t s) {
  if (max_nv > 0)
    k_vertex_stencil<<<dim3(cdiv((int64_t)max_nv * 27, 256), P.n_sub), 256, 0, s>>>(P, g, rho, nullptr, vcoef, vcode);
}

template <typename T>
void Kern<T>::kc_to_front(const PlanDev& P, const int32_t* subs_c, int ns, const T* Kc, double* fpool,
                          hipStream_t s) {
  if (ns == 0 || P.max_nc == 0) return;
  k_kc_to_front<T><<<dim3(cdiv((int64_t)P.max_nc * P.max_nc, 256), ns), 256, 0, s>>>(P, subs_c, Kc, fpool);
}

template <typename T>
void Kern<T>::front_gather(const PlanDev& P, const int32_t* fr, int nfr, int maxn, const T* Kc, double* fpool,
                           hipStream_t s) {
  if (nfr == 0 || maxn == 0) return;
  k_front_gather<T><<<dim3(cdiv(maxn, 4), nfr), 256, 0, s>>>(P, fr, Kc, fpool);
}

template <typename T>
void Kern<T>::gather_I(const PlanDev& P, const Geo& g, const double* r, T* vI, int nrhs, hipStream_t s) {
  if (P.max_nI == 0) return;
  k_gather_I<T><<<dim3(cdiv(P.max_nI, 256), P.n_sub, nrhs), 256, 0, s>>>(P, g, r, vI);
}

template <typename T>
void Kern<T>::block_solve(const PlanDev& P, const Geo& g, const double* rho, int setR, const T* G,
                          T* v, int nrhs, hipStream_t s, Profiler* prof, double g_entries, double vec_entries,
                          int set_max_block) {
  if (prof) prof->begin(2, s);
  if (nrhs >= P.mr_min) {
    const size_t smr = (size_t)hmax(P.max_block, 1) * (MR_COLS + 1) * sizeof(T);
    k_block_solve_mr<T><<<dim3(P.n_sub, cdiv(nrhs, MR_COLS)), MR_THREADS, smr, s>>>(P, setR, G, v, nrhs);
  } else {
    const int nt = (int)cdiv(set_max_block, 16), tiles = nt * (nt + 1) / 2;
    if (tiles <= 8 * 5) {
      const size_t sm = (size_t)hmax(P.max_block, 1) * ((8 + 9) * sizeof(double) + 2 * sizeof(T));
      k_block_solve<T, 512, 5, 3><<<dim3(P.n_sub, nrhs), 512, sm, s>>>(P, setR, G, v);
    } else {
      const size_t sm = (size_t)hmax(P.max_block, 1) * ((8 + 9) * sizeof(double) + 2 * sizeof(T));
      k_block_solve<T, 512, 9, 3><<<dim3(P.n_sub, nrhs), 512, sm, s>>>(P, setR, G, v);
    }
  }
  // the method must stream each lower-triangle G entry once per launch (4
  // flops per rhs off the diagonal) and read and write each vector once
  if (prof) prof->end(2, 4.0 * g_entries * nrhs, sizeof(T) * (g_entries + 2.0 * vec_entries * nrhs), s);
}

template <typename T>
void Kern<T>::gamma_kgi(const PlanDev& P, const Geo& g, const double* rho, const T* vI, T* q, int nrhs,
                        hipStream_t s) {
  if (P.max_ng == 0) return;
  (void)g;
  (void)rho;
  k_gamma_kgi<T><<<dim3(cdiv(P.max_ng, 128), P.n_sub, nrhs), 128, 0, s>>>(P, vI, q);
}

template <typename T>
void Kern<T>::gamma_t(const PlanDev& P, const Geo& g, const double* r, const T* q, const double* delta, T* gv,
                      int nrhs, hipStream_t s) {
  if (P.n_gam == 0) return;
  k_gamma_t<T><<<dim3(cdiv(P.n_gam, 256), nrhs), 256, 0, s>>>(P, g, r, q, delta, gv);
}

template <typename T>
void Kern<T>::neumann_rhs(const PlanDev& P, const T* gv, T* vR, int nrhs, hipStream_t s) {
  if (P.max_ng == 0) return;
  k_neumann_rhs<T><<<dim3(cdiv(P.max_ng, 128), P.n_sub, nrhs), 128, 0, s>>>(P, gv, vR);
}

template <typename T>
void Kern<T>::mu(const PlanDev& P, const T* vR, const T* Sc, T* mu_out, int nrhs, hipStream_t s) {
  if (P.max_na == 0) return;
  k_mu<T><<<dim3(P.n_sub, nrhs, cdiv(P.max_na, 64)), 256, ((size_t)P.max_na + 4 * 64) * sizeof(T), s>>>(P, vR, Sc,
                                                                                                    mu_out);
}

template <typename T>
void Kern<T>::coarse_rhs_local(const PlanDev& P, const T* XG, const T* PhiG, const T* Lam, const double* eps,
                               const T* gv, T* wv, T* bci, int nrhs, hipStream_t s) {
  if (P.max_nc == 0) return;
  // n_a + n_v = n_c: every local coarse dof is an average or a vertex
  if (nrhs >= P.mr_min)
    k_coarse_rhs_local_mr<T><<<dim3(cdiv(P.max_nc, 64), P.n_sub, cdiv(nrhs, MR_COLS)), 256, 0, s>>>(P, XG, PhiG, gv,
                                                                                                  wv, bci, nrhs);
  else
    k_coarse_rhs_local<T><<<dim3(cdiv(P.max_nc, CRL_COLS), P.n_sub, nrhs), 256, (size_t)hmax(P.max_ng, 1) * sizeof(T),
                            s>>>(P, XG, PhiG, gv, wv, bci);
  if (P.max_na > 0)
    k_coarse_rhs_avg<T><<<dim3(cdiv(P.max_na, CRA_COLS), P.n_sub, nrhs), 256, 0, s>>>(P, Lam, eps, gv, wv, bci);
}

template <typename T>
void Kern<T>::v2(const PlanDev& P, const T* vR, const T* XG, const T* mu_in, const T* lu, const T* YG,
                 const double* uc, T* v2_out, int nrhs, hipStream_t s) {
  if (P.max_ng == 0) return;
  if (nrhs >= P.mr_min) {
    k_v2_mr<T><<<dim3(cdiv(P.max_ng, 64), P.n_sub, cdiv(nrhs, MR_COLS)), 256, 0, s>>>(P, vR, XG, mu_in, lu, YG,
                                                                                     uc, v2_out, nrhs);
    return;
  }
  size_t sm = (size_t)(P.max_na + P.max_nv + 1 + 256) * sizeof(T);
  k_v2<T><<<dim3(cdiv(P.max_ng, 64), P.n_sub, nrhs), 256, sm, s>>>(P, vR, XG, mu_in, lu, YG, uc, v2_out);
}

template <typename T>
void Kern<T>::float_setup(const PlanDev& P, const T* Sc, T* Lam, double* eps, double* fdelta, hipStream_t s) {
  if (P.n_pinned == 0) return;
  k_float_setup<T><<<P.n_sub, 256, (size_t)hmax(P.max_na, 1) * sizeof(double), s>>>(P, Sc, Lam, eps, fdelta);
}
template <typename T>
void Kern<T>::float_mu(const PlanDev& P, const T* gv, T* mu_io, const double* eps, const double* fdelta,
                       double* fc, int nrhs, hipStream_t s) {
  if (P.n_pinned == 0) return;
  k_float_mu<T><<<dim3(P.n_sub, nrhs), 256, 0, s>>>(P, gv, mu_io, eps, fdelta, fc);
}
template <typename T>
void Kern<T>::float_v2(const PlanDev& P, const double* uc, const double* eps, const double* fc, T* v2,
                       int nrhs, hipStream_t s) {
  if (P.n_pinned == 0) return;
  k_float_v2<T><<<dim3(P.n_sub, nrhs), 256, 0, s>>>(P, uc, eps, fc, v2);
}

template <typename T>
void Kern<T>::lam_uc(const PlanDev& P, const T* Lam, const double* uc, T* lu, int nrhs, hipStream_t s) {
  if (P.max_na == 0) return;
  k_lam_uc<T><<<dim3(P.n_sub, nrhs, cdiv(P.max_na, 64)), 256, (size_t)(hmax(P.max_nc, 1) + 4 * 64) * sizeof(double),
                 s>>>(P, Lam, uc, lu);
}

template <typename T>
void Kern<T>::interior_rhs(const PlanDev& P, const Geo& g, const double* rho, const double* r, const double* w,
                           T* vI, int nrhs, hipStream_t s) {
  if (P.max_nI == 0) return;
  (void)rho;
  k_interior_rhs<T><<<dim3(cdiv(P.max_nI, 128), P.n_sub, nrhs), 128, 0, s>>>(P, g, r, w, vI);
}

template <typename T>
void Kern<T>::scatter_I(const PlanDev& P, const Geo& g, const T* vI, double* z, int nrhs, hipStream_t s) {
  if (P.max_nI == 0) return;
  k_scatter_I<T><<<dim3(cdiv(P.max_nI, 256), P.n_sub, nrhs), 256, 0, s>>>(P, g, vI, z);
}

void launch_gamma_w(const PlanDev& P, const Geo& g, const double* v2_d, const float* v2_f,
                    const double* delta, double* z, int nrhs, hipStream_t s) {
  if (P.n_gam == 0) return;
  dim3 grid(cdiv(P.n_gam, 256), nrhs);
  if (v2_d) k_gamma_w<double><<<grid, 256, 0, s>>>(P, g, v2_d, delta, z);
  else k_gamma_w<float><<<grid, 256, 0, s>>>(P, g, v2_f, delta, z);
}

void launch_front_zero_lower(const PlanDev& P, const int32_t* fronts, int nfr, int maxn, double* fpool,
                             hipStream_t s) {
  if (nfr == 0 || maxn == 0) return;
  k_front_zero_lower<<<dim3(cdiv(maxn, 32), nfr), 256, 0, s>>>(P, fronts, fpool);
}
void launch_kig_fill(const PlanDev& P, const Geo& g, const double* rho, hipStream_t s) {
  if (P.n_kig > 0) k_kig_fill<<<cdiv(P.n_kig, 256), 256, 0, s>>>(P, g, rho);
  if (P.n_kgi > 0) k_kgi_fill<<<cdiv(P.n_kgi, 256), 256, 0, s>>>(P, g, rho);
}
void launch_front_child_scatter(const PlanDev& P, const int32_t* children, int nchild, int maxn,
                                double* fpool, hipStream_t s) {
  if (nchild == 0 || maxn == 0) return;
  k_front_child_scatter<<<dim3(cdiv(maxn, 4), nchild), 256, 0, s>>>(P, children, fpool);
}
void launch_front_vec_init(const PlanDev& P, const int32_t* fr, int nfr, int maxn, const double* bci_d,
                           const float* bci_f, double* fvec, int64_t stride, int nrhs, hipStream_t s) {
  if (nfr == 0 || maxn == 0) return;
  const dim3 grid(cdiv(maxn, 256), nfr, nrhs);
  if (bci_d) k_front_vec_init<double><<<grid, 256, 0, s>>>(P, fr, bci_d, fvec, stride);
  else k_front_vec_init<float><<<grid, 256, 0, s>>>(P, fr, bci_f, fvec, stride);
}
void launch_front_vec_scatter(const PlanDev& P, const int32_t* children, int nchild, int maxn,
                              double* fvec, int64_t stride, int nrhs, hipStream_t s) {
  if (nchild == 0 || maxn == 0) return;
  k_front_vec_scatter<<<dim3(cdiv(maxn, 256), nchild, nrhs), 256, 0, s>>>(P, children, fvec, stride);
}
void launch_front_fwd(const PlanDev& P, const int32_t* fr, int nfr, int maxn, int maxp, const double* fpool,
                      double* fvec, double* xh, int64_t stride, int nrhs, hipStream_t s, double* part, bool pull) {
  if (nfr == 0 || maxp == 0) return;
  if (nrhs >= P.mr_min) {
    k_front_fwd_mr<<<dim3(cdiv(maxn, 64), nfr, cdiv(nrhs, MR_COLS)), 256, 0, s>>>(P, fr, fpool, fvec, xh, stride,
                                                                                  nrhs);
    return;
  }
  if (part) {
    const int pl = pull && P.front_pull ? 1 : 0;
    const int direct = maxp <= FK ? 1 : 0;  // one chunk: no separate sum of the chunks
    k_front_fwd_part<<<dim3(cdiv(maxn, 64), cdiv(maxp, FK), nfr * nrhs), 256, 0, s>>>(P, fr, fpool, fvec, stride,
                                                                                      nrhs, part, pl, direct, xh);
    if (!direct)
      k_front_fwd_fin<<<dim3(cdiv(maxn, 256), nfr, nrhs), 256, 0, s>>>(P, fr, fvec, xh, stride, nrhs, part, pl);
    return;
  }
  k_front_fwd<<<dim3(cdiv(maxn, 256), nfr, nrhs), 256, 0, s>>>(P, fr, fpool, fvec, xh, stride);
}
void launch_front_bwd(const PlanDev& P, const int32_t* fr, int nfr, int maxp, int maxb, const double* fpool,
                      const double* xh, int64_t stride, double* uc, int nrhs, hipStream_t s) {
  (void)maxb;
  if (nfr == 0 || maxp == 0) return;
  if (nrhs >= P.mr_min) {
    k_front_bwd_mr<<<dim3(cdiv(maxp, 64), nfr, cdiv(nrhs, MR_COLS)), 256, 0, s>>>(P, fr, fpool, xh, stride, uc, nrhs);
    return;
  }
  k_front_bwd<<<dim3(cdiv(maxp, 4), nfr, nrhs), 256, 0, s>>>(P, fr, fpool, xh, stride, uc);
}

void launch_dot(const double* a, const double* b, int64_t n, int nrhs, double* partial, int nblocks,
                double* out, hipStream_t s) {
  k_dot_partial<<<dim3(nblocks, nrhs), 256, 0, s>>>(a, b, n, partial);
  k_dot_final<<<nrhs, 256, 0, s>>>(partial, nblocks, out);
}
void launch_pcg_xr(double* x, double* r, const double* p, const double* q, const double* rz, const double* pq,
                   const int32_t* active, int64_t n, int nrhs, hipStream_t s) {
  k_pcg_xr<<<dim3(cdiv(n, 256), nrhs), 256, 0, s>>>(x, r, p, q, rz, pq, active, n);
}
void launch_pcg_p(double* p, const double* z, const double* num, const double* den, const int32_t* active,
                  int64_t n, int nrhs, hipStream_t s) {
  k_pcg_p<<<dim3(cdiv(n, 256), nrhs), 256, 0, s>>>(p, z, num, den, active, n);
}
void launch_pcg_p_flex(double* p, const double* z, const double* zdr, const double* rz_old,
                       const int32_t* active, int64_t n, int nrhs, hipStream_t s) {
  k_pcg_p<<<dim3(cdiv(n, 256), nrhs), 256, 0, s>>>(p, z, zdr, rz_old, active, n);
}

void launch_element_grad(const Geo& g, const double* khat, const double* rho, const double* u,
                         const double* lam, double* out, int nrhs, hipStream_t s) {
  k_element_grad<<<cdiv(g.n_elem, 256), 256, 0, s>>>(g, khat, rho, u, lam, out, nrhs);
}
void launch_box_filter(const Geo& g, const double* in, double* out, int mode, hipStream_t s) {
  k_box_filter<<<cdiv(g.n_elem, 256), 256, 0, s>>>(g, in, out, mode);
}

template struct Kern<double>;
template struct Kern<float>;

}  // namespace bddcso

namespace bddcso {
namespace {
// PCG bookkeeping on the device, one thread per right-hand side.
// After r is updated and rr = r.r: count the iteration, record alpha, test
// convergence (rr <= tol2), flag breakdown (p.q <= 0 or r.z <= 0).
__global__ void k_pcg_book1(int nrhs, int k, const int32_t* __restrict__ kd, const double* __restrict__ rz,
                            const double* __restrict__ pq, const double* __restrict__ rr,
                            const double* __restrict__ tol2, int32_t* __restrict__ active,
                            int32_t* __restrict__ iters, int32_t* __restrict__ flags,
                            double* __restrict__ hist_alpha, int32_t* __restrict__ nactive) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  // the iteration index: an argument, or (replayed launches) a device counter
  const int kk = kd ? *kd : k;
  const int j = threadIdx.x;
  if (j < nrhs) {
    if (active[j]) {
      iters[j] = kk + 1;
      const double a = rz[j] / pq[j];
      hist_alpha[kk * nrhs + j] = a;
      if (!(pq[j] > 0.0) || !(rz[j] > 0.0) || !isfinite(a)) {
        flags[j] |= 2;  // breakdown
        active[j] = 0;
      } else if (rr[j] <= tol2[j]) {
        flags[j] |= 1;  // converged
        active[j] = 0;
      }
    }
    if (active[j]) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *nactive = cnt;
}

// After p = z + beta p: record beta = num/rz and move rz <- rz_new; with a
// device counter, advance it to the next iteration.
__global__ void k_pcg_book2(int nrhs, int k, int32_t* __restrict__ kd, double* __restrict__ rz,
                            const double* __restrict__ num, const double* __restrict__ rz_new,
                            const int32_t* __restrict__ active, double* __restrict__ hist_beta) {
  const int j = threadIdx.x;
  const int kk = kd ? *kd : k;
  if (j < nrhs && active[j]) {
    hist_beta[kk * nrhs + j] = num[j] / rz[j];
    rz[j] = rz_new[j];
  }
  if (kd) {
    __syncthreads();
    if (threadIdx.x == 0) *kd = kk + 1;
  }
}

__global__ void k_copy_f64(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
}  // namespace

void launch_pcg_book1(int nrhs, int k, const int32_t* kd, const double* rz, const double* pq, const double* rr,
                      const double* tol2, int32_t* active, int32_t* iters, int32_t* flags, double* hist_alpha,
                      int32_t* nactive, hipStream_t s) {
  k_pcg_book1<<<1, 64, 0, s>>>(nrhs, k, kd, rz, pq, rr, tol2, active, iters, flags, hist_alpha, nactive);
}
void launch_pcg_book2(int nrhs, int k, int32_t* kd, double* rz, const double* num, const double* rz_new,
                      const int32_t* active, double* hist_beta, hipStream_t s) {
  k_pcg_book2<<<1, 64, 0, s>>>(nrhs, k, kd, rz, num, rz_new, active, hist_beta);
}
void launch_copy_f64(const double* a, double* b, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_copy_f64<<<hmin(cdiv(n, 256), 65536), 256, 0, s>>>(a, b, n);
}
}  // namespace bddcso
