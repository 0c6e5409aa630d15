// Plain structs shared by the host planner and the device kernels.
#pragma once
#include <cstdint>

namespace bddcso {

// In-plane offsets (x, y) of a node's stencil neighbours of rank at most its
// own within a block's plane (ranks run x fastest, then y): itself, x-1, and
// the three of row y-1.  In 2D (planes are lines in x) only the first two.
constexpr int kInPlaneLower[5][2] = {{0, 0}, {-1, 0}, {-1, -1}, {0, -1}, {1, -1}};

// One subdomain: an axis-aligned box of elements.  Local nodes are the free
// grid nodes of the closed box, numbered x fastest.  Sets: I (interior, not
// on Gamma), r (every local node except the primal vertices, Section 3's
// vertex elimination), Gamma entries (local nodes on the interface).
struct SubDev {
  int lo[3];      // global grid coordinates of local node (0,0,0)
  int m[3];       // local nodes per axis (m[2] = 1 in 2D)
  int elo[3];     // element box, inclusive lower corner
  int ehi[3];     // element box, exclusive upper corner
  int n_loc, n_I, n_r, n_g, n_v, n_a, n_c;
  int n_s;        // selected rows: the Gamma entries, then the r-set stencil
                  // neighbours of the primal vertices that are not on Gamma
  int nbI, nbR;   // diagonal blocks of the I and r factors
  int color;      // subdomains of one colour share no coarse dof
  int pin;        // floating subdomain without primal point constraints: the
                  // interior local node left out of the r-set (the constant
                  // of its kernel is carried separately), else -1
  int front;      // front the local coarse matrix is added to
  int64_t loc_off;   // offset of per-local-node tables
  int64_t I_off;     // offset of I-order tables / vectors
  int64_t r_off;     // offset of r-order tables / vectors
  int64_t g_off;     // offset of Gamma-entry tables / vectors
  int64_t v_off;     // offset of vertex tables
  int64_t a_off;     // offset into the average pointer table (n_a + 1 entries)
  int64_t am_off;    // offset of per-average vectors (sum of n_a before)
  int64_t c_off;     // offset of local coarse tables / vectors
  int64_t bI_off, bR_off;  // offsets into the block table
  int64_t Z_off;     // n_r x (n_a + n_v): [X | Y'] (column-major, ld n_r)
  int64_t sel_off;   // offset of the selected-row table
  int64_t XG_off;    // n_s x n_a (ld n_s): rows of X at the selected rows (0 at vertices)
  int64_t Sc_off;    // n_a x n_a: constraint Schur complement, swept
  int64_t T_off;     // n_a x n_c: C_r Y - [0 I] (then Lambda's vertex columns packed,
                     // n_a x n_v), and Lambda in a buffer of its own
  int64_t PhiG_off;  // n_s x n_v (ld n_s): Phi's vertex columns at the selected rows (the
                     // first n_g are the Gamma entries)
  int64_t YG_off;    // n_g x n_v (ld n_g): Y' at the Gamma entries (the unit entry of
                     // its coarse dof at a Gamma entry that is a primal vertex)
  int64_t Kc_off;    // n_c x n_c local coarse matrix
};

// One diagonal block of a block-tridiagonal local factor: the nodes of the
// set lying in planes [plane_lo, plane_hi) of the plane axis.
struct BlockDev {
  int start, size;          // first rank in set order, number of nodes
  int plane_lo, plane_hi;   // local plane range
  int first_n, last_n;      // nodes in the first / last plane of the block
  int ld;                   // leading dimension of its matrix: size rounded up to 16
  int64_t G_off;            // offset of its size x size matrix (ld x size storage, 16-aligned)
  int64_t cf_off;           // coupling rows of the first plane to block k-1 (-1: none)
  int64_t cb_off;           // coupling rows of the last plane to block k+1 (-1: none)
  int za;                   // r blocks: the columns 0..za-1 of [X | Y'] (in their stored
                            // order) whose right-hand sides reach this block or an earlier one
};

// One front of the multifrontal coarse factorization.  Positions 0..p-1 are
// its pivots (a separator of the nested dissection), p..n-1 the ancestors'
// dofs it couples to.
struct FrontDev {
  int64_t off;        // offset of the n x n matrix (column-major)
  int64_t voff;       // offset of its vector (n entries per rhs)
  int64_t idx_off;    // offset of its coarse ids (n entries)
  int64_t pmap_off;   // offset of the map of positions p..n-1 into the parent
  int n, p;
  int parent;         // -1 at a root
  int level;
  int nsrc;           // sources of the gather assembly (at most 2; -1: assembled by scatter)
  int src[2];         // a child front, or -(s + 1) for the local coarse matrix of subdomain s
  int64_t src_map[2]; // offset in front_imap: per position of this front, the source's index, -1 if none
};

// Batched dense sweep descriptor.
struct SweepDesc {
  int64_t off;   // offset of the n x n matrix in its pool
  int n, p;      // size and number of pivots to sweep
  int ld;
};

// Batched GEMM descriptor: C = beta C + alpha op(A) op(B).
struct GemmDesc {
  int64_t a, b, c;   // element offsets in their pools
  int m, n, k;
  int lda, ldb, ldc;
};

}  // namespace bddcso
