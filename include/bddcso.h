/*
 * bddcso.h -- C ABI of the MI355X (gfx950) BDDC-SO solver.
 *
 * Solves the Q1 finite-element discretisation of -div(rho grad u) = f on the
 * unit square / cube with zero Dirichlet data (the model problem of Section 2,
 * with the variable coefficient of Remark 4) by preconditioned conjugate
 * gradients, the preconditioner being BDDC-SO (Section 3): BDDC whose coarse
 * degrees of freedom are point values at, or averages over, subobjects --
 * the vertices, edges and faces of a finer partition (the subsubdomains)
 * that lie on the interface of the subdomain partition.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Mesh: structured, n_el[0] x n_el[1] (x n_el[2]) elements, spacing h[a]
 *    per axis.  For dim = 2, n_el[2] and h[2] are ignored.  Elements are
 *    numbered lexicographically with x fastest.
 *  - Unknowns: the free (non-boundary) grid nodes, numbered lexicographically
 *    with x fastest over 1..n_el[a]-1 per axis.  n_free is their count.
 *  - Vectors of several right-hand sides are stored [nrhs][n_free],
 *    contiguous, FP64.
 *  - Device pointers (suffix _dev) are HIP device memory owned by the caller;
 *    the library never frees them.  Host pointers are read during the call
 *    only, unless stated otherwise.
 *  - stream: a hipStream_t passed as void*; NULL means the default stream.
 *    Work is enqueued on that stream; calls return once it is enqueued,
 *    except where a call says it synchronises.
 *  - Every function returns a bddcso_status.  On error nothing is left
 *    half-built, and bddcso_last_error() returns a message for this thread.
 *  - Subdomains must be axis-aligned boxes of elements (every config of the
 *    paper's experiments is); subsubdomains may have any shape but each must
 *    lie inside one subdomain (Section 3).
 */
#ifndef BDDCSO_H
#define BDDCSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BDDCSO_OK = 0,
  BDDCSO_EINVAL = -1,     /* invalid argument or descriptor                  */
  BDDCSO_ENOMEM = -2,     /* device or host allocation failed                */
  BDDCSO_ESINGULAR = -3,  /* a local, constraint or coarse pivot was <= 0    */
  BDDCSO_EBREAKDOWN = -4, /* PCG breakdown: p^T A p <= 0 or r^T z <= 0       */
  BDDCSO_ENOCONV = -5,    /* maxit reached without meeting rtol              */
  BDDCSO_EHIP = -6        /* a HIP runtime call failed                       */
} bddcso_status;

typedef struct bddcso_problem bddcso_problem; /* host descriptors + classification */
typedef struct bddcso_precond bddcso_precond; /* device factors of one setup      */

/* Primal object kinds (Section 3; Remark 5 on acceptable paths).
 * BDDCSO_PRIMAL_HALF keeps only half of the codimension-one objects (faces
 * in 3D, edges in 2D) of the selected kinds: the "half of the face
 * constraints" of Section 5.1's vf-min, which does not say which half.  The
 * rule is a checkerboard over the fine partition: each subsubdomain gets,
 * per axis, the rank of its lowest element coordinate among all
 * subsubdomains' lowest coordinates; a face between subsubdomains j1 < j2
 * is kept when the sum of j1's ranks over the axes other than its normal
 * (the axis along which the two ranks differ most) is even.
 * BDDCSO_PRIMAL_VF_MIN = V | F | HALF. */
#define BDDCSO_PRIMAL_V 1
#define BDDCSO_PRIMAL_E 2
#define BDDCSO_PRIMAL_F 4
#define BDDCSO_PRIMAL_HALF 8
#define BDDCSO_PRIMAL_VF_MIN 13

typedef struct {
  int primal_mask;   /* OR of BDDCSO_PRIMAL_*; 7 = every subobject ("vef"),
                        13 = vertices and half of the faces ("vf-min")     */
  int weighting;     /* 0: eq. (W) counting weights; 1: Remark 4, weights by
                        the coefficient averaged over each subsubdomain       */
  int precision;     /* 0: FP64 throughout; 1: local factors, local solves
                        and Phi^T K Phi in FP32 (coarse problem, outer PCG
                        recurrences and dot products stay FP64)               */
  int coarse_solver; /* 0: nested-dissection multifrontal; 1: one dense front */
  int max_nrhs;      /* right-hand sides the workspace is sized for (>= 1)    */
  int maxit;         /* PCG iteration limit                                   */
  double rtol;       /* stop when ||r_k||_2 <= rtol ||b||_2 (x0 = 0)          */
  int fixed_iters;   /* > 0: run exactly this many iterations, no test        */
  int flexible;      /* 1: flexible CG, beta = z_{k+1}.(r_{k+1}-r_k)/rho_k;
                        used automatically when precision = 1               */
  int block_target;  /* target size of the dense diagonal blocks of the local
                        block-tridiagonal factors; 0 = default (192)          */
  int graph;         /* 1: the numeric setup and the two halves of a PCG
                        iteration are captured once (per right-hand-side
                        count) into HIP graphs and replayed on the caller's
                        stream; 0: ordinary launches.  bddcso_solve_noalloc
                        and profiled runs always launch directly.           */
  /* Launch shapes (results agree to rounding; chosen by bddcso_autotune).  */
  int sweep_reg_rows;/* largest matrix swept by the register-resident kernel
                        (<= 304; 0 = 304); larger ones take the slab path    */
  int slab_lookahead;/* slab sweeps: 0 = by the trailing update's size,
                        1 = none (each pivot block swept after the whole
                        update), 2 = always beside the rest of the update   */
  int mr_min_rhs;    /* right-hand sides from which the many-RHS kernels
                        are used (0 = 4)                                     */
  int update_tile;   /* tile rows of the slab sweeps' trailing update: 64 or
                        128 (0 = 64)                                         */
  int slab_width;    /* pivots per slab of the large sweeps: 96 or 192, or 0
                        (96 for a few matrices with short trailing updates,
                        else 192)                                            */
} bddcso_options;

/* Fills the defaults: vef, coefficient weights, FP64, multifrontal coarse,
 * 1 RHS, maxit 1000, rtol 1e-8, no fixed count, standard CG. */
void bddcso_default_options(bddcso_options* opts);

#define BDDCSO_MAX_RHS 64
typedef struct {
  int nrhs;
  int iters[BDDCSO_MAX_RHS];        /* operator applications in the loop     */
  int converged[BDDCSO_MAX_RHS];
  double relres[BDDCSO_MAX_RHS];    /* final ||r_k|| / ||b|| (recurrence)   */
  double lambda_min[BDDCSO_MAX_RHS];/* extreme Lanczos eigenvalues of BA     */
  double lambda_max[BDDCSO_MAX_RHS];
  double kappa[BDDCSO_MAX_RHS];     /* lambda_max / lambda_min               */
  int64_t n_coarse;
  double t_solve_ms;                /* host wall time of the solve call      */
} bddcso_stats;

/*
 * Creates the host descriptors and classifies the interface (Section 3):
 * Gamma = free nodes shared by two or more subdomains; each Gamma node is
 * keyed by the set of subsubdomains containing it (Remark 2 on
 * classification); connected sets of nodes with one key are the subobjects.
 * Host only (no device work).
 *   dim          2 or 3
 *   n_el[3]      elements per axis (n_el[a] >= 2)
 *   h[3]         mesh spacing per axis (> 0)
 *   elem_sub     [n_elements] subdomain id of each element, 0..n_sub-1
 *   elem_subsub  [n_elements] subsubdomain id, 0..n_subsub-1
 * Errors: EINVAL for ids out of range, a subdomain that is not a box, or a
 * subsubdomain that spans two subdomains.
 */
bddcso_status bddcso_problem_create(int dim, const int64_t n_el[3], const double h[3],
                                    const int32_t* elem_sub, const int32_t* elem_subsub,
                                    bddcso_problem** out);

/* Sizes after classification; any output pointer may be NULL.  n_coarse is
 * the number of subobjects selected by primal_mask (Table 1's "size of the
 * coarse problem"); counts[3] receives the selected vertices, edges, faces. */
bddcso_status bddcso_problem_info(const bddcso_problem* p, int primal_mask, int64_t* n_free,
                                  int64_t* n_gamma, int64_t* n_coarse, int* n_sub,
                                  int64_t counts[3]);

/*
 * Device workspace that bddcso_setup needs for these options: every factor,
 * basis, coarse front, plan table and per-application vector of one
 * preconditioner, each piece 256-byte aligned.  Host only (plans the
 * problem, no device work); the same sizes bddcso_setup lays out.
 * Errors: EINVAL (options or plan, e.g. a coarse front above 4 GiB).
 */
bddcso_status bddcso_setup_workspace_size(bddcso_problem* p, const bddcso_options* opts, size_t* bytes);

/*
 * Builds the preconditioner for coefficient rho (Remark 4), on the device:
 * local matrices, block factorizations of K_II and K_rr (primal vertices
 * eliminated), the constraint Schur complement, the coarse basis Phi_i, the
 * local coarse matrices Phi_i^T K_i Phi_i and the factorization of the
 * assembled coarse matrix (Section 3 with Definition 1).  Synchronises the
 * stream before returning.
 *   rho_dev       [n_elements] FP64 device array, > 0
 *   workspace_dev caller-owned device memory of at least ws_bytes =
 *                 bddcso_setup_workspace_size(...) bytes, 256-byte aligned;
 *                 it must outlive the preconditioner and is never freed by
 *                 the library.  NULL: the library allocates the same amount
 *                 itself (freed by bddcso_precond_destroy).
 * Errors: EINVAL (also: workspace too small or misaligned), ENOMEM,
 * ESINGULAR (a pivot <= 0, e.g. a floating subdomain left without enough
 * primal constraints), EHIP.
 */
bddcso_status bddcso_setup(bddcso_problem* p, const double* rho_dev, const bddcso_options* opts,
                           void* workspace_dev, size_t ws_bytes, void* stream, bddcso_precond** out);

/* Recomputes every numeric factor of an existing preconditioner for a new
 * coefficient field, reusing its plan and device memory: no allocation.
 * Enqueued on stream; pivot failures are reported by the next
 * bddcso_check_pivots or bddcso_solve.  Increments the generation. */
bddcso_status bddcso_refactor(bddcso_precond* pc, const double* rho_dev, void* stream);

/* Number of numeric setups (bddcso_setup's included) this preconditioner
 * has gone through: a caller that keeps results tied to one set of factors
 * (an adjoint solve after a forward solve) checks that it has not changed. */
bddcso_status bddcso_precond_generation(const bddcso_precond* pc, int64_t* generation);

/* Synchronises stream and returns ESINGULAR if the last setup/refactor met a
 * non-positive pivot. */
bddcso_status bddcso_check_pivots(bddcso_precond* pc, void* stream);

/* y = A x, the matrix-free Q1 operator with the preconditioner's rho
 * (Section 2, Remark 4).  x_dev, y_dev: [nrhs][n_free] FP64, distinct. */
bddcso_status bddcso_operator_apply(const bddcso_precond* pc, const double* x_dev, double* y_dev,
                                    int nrhs, void* stream);

/* z = B r, the BDDC-SO preconditioner (Definition 1 with V1 = U_I,
 * V2 = W~, Q1 = I, Q2 = (I - P) E; Section 3).  r_dev, z_dev:
 * [nrhs][n_free] FP64, distinct; nrhs <= max_nrhs. */
bddcso_status bddcso_apply(bddcso_precond* pc, const double* r_dev, double* z_dev, int nrhs,
                           void* stream);

/*
 * Solves A x = b by PCG preconditioned with BDDC-SO (Section 5's solver),
 * from x0 = 0, every right-hand side with its own recurrence, in lockstep;
 * converged columns are frozen.  Synchronises the stream once per iteration
 * for the convergence test (not in fixed_iters mode).
 *   b_dev, x_dev: [nrhs][n_free] FP64 device arrays; nrhs <= max_nrhs.
 *   stats: host struct filled on return (may be NULL).
 * Errors: EBREAKDOWN, ENOCONV (x holds the last iterate), ESINGULAR.
 */
bddcso_status bddcso_solve(bddcso_precond* pc, const double* b_dev, double* x_dev, int nrhs,
                           bddcso_stats* stats, void* stream);

/*
 * bddcso_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as bddcso_solve, but the solve state
 * (the six PCG vectors, dot partials, scalars, history and flags) lives in a
 * static 64 MiB device array of the library instead of the preconditioner's
 * memory; it needs about 48 * n_free * nrhs + 16 * (maxit + 1) * nrhs bytes,
 * i.e. n_free * nrhs up to about 1.39e6.  Larger solves return EINVAL and
 * run nothing.  The call allocates no device or pinned memory (the
 * preconditioner must already exist).  Every call on one device shares that
 * device's array, which keeps the last call's contents: calls that overlap
 * on one device (other streams or threads) race and must be serialised by
 * the caller.
 */
bddcso_status bddcso_solve_noalloc(bddcso_precond* pc, const double* b_dev, double* x_dev, int nrhs,
                                   bddcso_stats* stats, void* stream);

/* Element gradient of a loss through the solve:
 *   g_e = -rho_e * sum_k lam_k,e^T K^_e u_k,e
 * with K^_e the unit-coefficient Q1 element matrix and u_e, lam_e the
 * element's nodal values (zero at boundary nodes); the sum runs over the
 * nrhs columns.  u_dev, lam_dev: [nrhs][n_free]; g_dev: [n_elements]. */
bddcso_status bddcso_element_grad(const bddcso_precond* pc, const double* u_dev,
                                  const double* lam_dev, double* g_dev, int nrhs, void* stream);

/* 3^dim box mean of an element field over in-domain neighbours (normalised
 * by their count), or its transpose when transpose != 0.
 * in_dev, out_dev: [n_elements] FP64, distinct. */
bddcso_status bddcso_box_filter(const bddcso_problem* p, const double* in_dev, double* out_dev,
                                int transpose, void* stream);

/* The coefficient of a log-coefficient field: rho_e = exp((F theta)_e), with
 * F the 3^dim box mean of bddcso_box_filter (the smoothed log-coefficient of
 * the adjoint workload; not in the paper).  theta_dev, rho_dev:
 * [n_elements] FP64, distinct. */
bddcso_status bddcso_coef_from_log(const bddcso_problem* p, const double* theta_dev, double* rho_dev,
                                   void* stream);

/*
 * Autotuner: times one step (numeric setup and the PCG solve of b_dev) of
 * the problem for launch-shape variants of base and returns the fastest in
 * best.  The variants go knob by knob (coordinate descent): update_tile,
 * slab_lookahead, sweep_reg_rows, block_target, mr_min_rhs (nrhs > 1),
 * graph; each trial
 * builds a preconditioner in library-allocated memory, runs one untimed and
 * one timed step on the stream (HIP events) and frees it.  Every trial uses
 * base's method options (primal_mask, weighting, precision, coarse_solver,
 * rtol, maxit), so the variants compute the same preconditioner.
 *   rho_dev: [n_elements]; b_dev: [nrhs][n_free]; report may be NULL.
 */
#define BDDCSO_TUNE_MAX 32
typedef struct {
  int n_trials;
  int best;                              /* index into the arrays below      */
  bddcso_options tried[BDDCSO_TUNE_MAX];
  double step_ms[BDDCSO_TUNE_MAX];       /* setup + solve, HIP events        */
  int status[BDDCSO_TUNE_MAX];           /* bddcso_status of the trial       */
} bddcso_tune_report;

bddcso_status bddcso_autotune(bddcso_problem* p, const double* rho_dev, const bddcso_options* base,
                              const double* b_dev, int nrhs, void* stream, bddcso_options* best,
                              bddcso_tune_report* report);

/* Sizes and algorithmic work of the plan for these options (host only; no
 * device work).  Flop counts are those of the symmetric sweeps (n^2 p per
 * matrix of size n with p pivots, lower triangle). */
typedef struct {
  int64_t n_coarse;
  int64_t n_fronts;            /* fronts of the coarse factorization            */
  int64_t levels;              /* levels of the nested-dissection tree          */
  int64_t max_front;           /* largest front size                            */
  int64_t max_front_pivots;    /* largest pivot count of a front                */
  int64_t n_blocks;            /* diagonal blocks of all local factors          */
  int64_t max_block;           /* largest diagonal block                        */
  double coarse_factor_entries;/* sum over fronts of n * p                      */
  double coarse_sweep_flops;   /* sum over fronts of n^2 p                      */
  double local_sweep_flops;    /* sum over local blocks of size^3               */
  double device_bytes;         /* = bddcso_setup_workspace_size                 */
} bddcso_plan_stats;

bddcso_status bddcso_plan_info(bddcso_problem* p, const bddcso_options* opts, bddcso_plan_stats* out);

/* Timing of kernel classes with HIP events recorded around each of their
 * launches on the launching stream, from this call on.  class_mask: bit c
 * selects class c (0 switches it off and clears the record).  Classes: 1 the
 * trailing updates of the sweeps (rank-32 panels, rank-192 slabs; MFMA),
 * 2 the block-tridiagonal solves (HBM), 3 the batched GEMMs (MFMA), 4 the
 * pivot-block work of the large sweeps: 32-pivot panels, slab pivot blocks
 * (one workgroup each) and slab CD products, 5 the batched register-resident
 * sweeps of matrices up to 272 rows (MFMA), 6 the block Schur updates of the
 * local factor chains, 7 the plane-coupling products of the basis solves,
 * 8 the Q1 operator inside bddcso_solve (the last three HBM).
 * bddcso_profile_read waits for
 * the recorded events, then returns for one class the launches seen, their
 * summed duration and their summed algorithmic flops and bytes (the minimum
 * traffic: each operand read once, each output written once). */
bddcso_status bddcso_profile(bddcso_precond* pc, int class_mask);
bddcso_status bddcso_profile_read(bddcso_precond* pc, int kernel_class, int64_t* launches, double* total_ms,
                                  double* flops, double* bytes);

/* The same launches' work by the reference count of a banded
 * representation: local factors as lexicographic band Cholesky factors
 * (bandwidth m_x m_y + m_x + 1 in 3D, m_x + 1 in 2D; n b^2 flops to factor,
 * 2 nnz reads per triangular solve, 4 nnz flops per column of [X | Y']),
 * dense sweeps as Cholesky (p^3/3 + (n-p) p^2 + (n-p)^2 p for n rows and p
 * pivots); other classes as executed.  Host only; any pointer may be NULL. */
bddcso_status bddcso_profile_reference(const bddcso_precond* pc, int kernel_class, double* flops,
                                       double* bytes);

/* Plain device copy of `bytes` (a multiple of 16) from src_dev to dst_dev by
 * a streaming kernel: a known traffic against which hardware byte counters
 * are calibrated.  Not part of the solver. */
bddcso_status bddcso_copy_probe(const void* src_dev, void* dst_dev, int64_t bytes, void* stream);

/* Sizes of one preconditioner: coarse dofs, fronts of the coarse factor,
 * device bytes held.  Any pointer may be NULL. */
bddcso_status bddcso_precond_info(const bddcso_precond* pc, int64_t* n_coarse, int64_t* n_fronts,
                                  int64_t* device_bytes, int64_t* coarse_factor_entries);

/* Copies subdomain sub's local coarse matrix Phi_i^T K_i Phi_i (column-major,
 * n_c x n_c, FP64) and the global coarse ids of its rows to host buffers of
 * at least cap_nc entries (resp. cap_nc^2).  Synchronises the stream.
 * *nc receives n_c.  For checks of the setup one subdomain at a time. */
bddcso_status bddcso_local_coarse(const bddcso_precond* pc, int sub, double* kc_host,
                                  int64_t* ids_host, int64_t cap_nc, int64_t* nc, void* stream);

void bddcso_precond_destroy(bddcso_precond* pc);
void bddcso_problem_destroy(bddcso_problem* p);

/* Message of the last non-OK status returned on this thread ("" if none). */
const char* bddcso_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BDDCSO_H */
