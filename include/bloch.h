/*
 * bloch.h -- C ABI of the MI355X (gfx950) Bloch-Maxwell eigensolver.
 *
 * The library computes the smallest non-zero eigenvalues lambda and eigenvectors of the
 * two-dimensional Maxwell problem  curl (1/eps) curl u = lambda u  on the periodic unit
 * cell [0,a] x [0,b] with Bloch boundary conditions for the parameter k = (k1, k2)
 * (Boerm, Koehl, Talebi, "Computing Maxwell eigenmodes with Bloch boundary conditions",
 * arXiv 2304.00337: problem statement in Section 1, Bloch conditions in Section 1 and 2).
 * Discretisation: lowest-order Nedelec edge elements on an n x m grid with the Bloch-phase
 * modified basis of Section 3, giving the Hermitian pencil A e = lambda M e.  Method:
 * block preconditioned inverse iteration with null-space elimination and Ritz step
 * (Section 4), a geometric multigrid V-cycle for A + mu M as preconditioner and a nodal
 * multigrid for the null-space projection (Section 5), Rayleigh-quotient extrapolation of
 * starting blocks across k (Section 6) and throw-away vectors (Section 7).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Indices are 0-based.  Cell (c1,c2) is [c1 h1,(c1+1) h1] x [c2 h2,(c2+1) h2], h1 = a/n,
 * h2 = b/m, stored at c2*n + c1.  Edge degrees of freedom are line integrals along the
 * edges: x-edge (j1,j2) from node (j1,j2) to (j1+1,j2) at index j2*n + j1, y-edge (j1,j2)
 * from (j1,j2) to (j1,j2+1) at index n*m + j2*n + j1 (N_e = 2nm).  Node (j1,j2) sits at
 * (j1 h1, j2 h2), index j2*n + j1 (N_v = nm).  The Bloch phases are alpha = exp(i k1 a),
 * beta = exp(i k2 b); a Gamma point (k1 a and k2 b multiples of 2 pi within 1e-14) uses
 * alpha = beta = 1 exactly and the k = 0 treatment of the null space.
 *
 * Device block layout ("planar column blocks"): a block of `ncols` complex vectors of
 * length N is ncols consecutive columns; column j holds N real parts followed by N
 * imaginary parts: re(i,j) = base[j*2N + i], im(i,j) = base[j*2N + N + i].  FP64 blocks
 * are double, FP32 blocks float.  All device pointers are caller-owned device memory on
 * the device that was current at bl_create; they must not overlap unless stated.
 *
 * Host arrays are caller-owned and only read or written during the call.  The solver
 * handle owns all of its internal device memory and frees it in bl_destroy.  One handle
 * must not be used from two threads at once; work is issued on the stream given at
 * creation (NULL = the legacy default stream) and every call returns after that stream
 * has been synchronised, except where stated.
 *
 * Return codes: BL_OK (0) on success, a negative BL_E* code otherwise; bl_strerror gives
 * a message.  On BL_ENOCONV the outputs hold the current best approximations and their
 * residuals.
 */
#ifndef BLOCH_H_
#define BLOCH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BL_OK 0
#define BL_EINVAL (-1)   /* invalid argument (sizes, eps, k, options, null pointers) */
#define BL_ENOMEM (-2)   /* device or host allocation failed                          */
#define BL_EHIP (-3)     /* a HIP runtime call failed                                 */
#define BL_ENOCONV (-4)  /* max_iter reached before the wanted residuals met tol      */
#define BL_EAGAIN (-5)   /* result not ready (serving)                                */
#define BL_ESTATE (-6)   /* call not valid in the handle's current state              */

typedef struct bl_solver bl_solver;

/* The unit cell and its mesh (Section 3): n x m rectangles of the cell a x b. */
typedef struct bl_grid {
  int32_t n, m; /* cells per direction; >= 2, even on every smoothed multigrid level   */
  double a, b;  /* lattice periods, > 0                                                */
} bl_grid;

/* Options of the iteration.  bl_default_opts fills every field; zero-valued optional
 * fields select the defaults stated here. */
typedef struct bl_opts {
  int32_t nev;          /* wanted smallest non-zero eigenpairs (Section 4), >= 1           */
  int32_t nthrow;       /* additional throw-away vectors (Section 7), >= 0; p = nev+nthrow */
  int32_t max_iter;     /* iteration cap per Bloch parameter (default 200)                 */
  int32_t levels;       /* maximum multigrid levels, 0 = coarsen while possible            */
  int32_t coarsest_min; /* stop coarsening below this many cells per direction (8)         */
  int32_t nu_pre;       /* pre-smoothing sweeps of the edge and nodal V-cycles (1)         */
  int32_t nu_post;      /* post-smoothing sweeps (1)                                       */
  int32_t nodal_cycles; /* nodal V-cycles per null-space projection (Section 5) (2)        */
  int32_t variant;      /* 0 = gradient method [E_hat, E], 1 = LOBPCG (Section 4)          */
  int32_t precision;    /* 0 = FP64 throughout, 1 = mixed: V-cycle and nodal projection in
                           complex FP32, residuals, Gram, Ritz and extrapolation in FP64   */
  int32_t extrap_depth; /* previous Bloch parameters used for extrapolation, 1..3 (3)      */
  int32_t autotune;     /* 1 = time the candidate launch shapes of the smoothers and of the
                           Rayleigh-Ritz products when a handle is created and keep the
                           fastest (cached per shape; never changes results), 0 = fixed (1) */
  int32_t coarse_fuse;  /* 1 = run the coarse levels of every V-cycle (those whose vectors
                           fit one workgroup's LDS) in one launch per column; bit-identical
                           to the per-level launches, 0 = per-level launches (1)           */
  int32_t tiled_sweeps; /* 1 = each smoothing sweep of a level above the fused ones is one
                           launch over LDS tiles with halos (all four colours); 2 = as 1, and
                           the residual, restriction and prolongation of the nodal cycles
                           and of the FP32 edge cycles ride in the sweeps (the last pre-sweep
                           writes the restricted residual, the first post-sweep reads the
                           prolongated correction; a nodal solve's update rides in its last
                           sweep); all bit-identical to one launch per colour, 0 = one launch
                           per colour (2)                                                   */
  double tol;           /* stop when ||A e_i - lambda_i M e_i||_2 / (lambda_i ||M e_i||_2)
                           <= tol for the first nev vectors (1e-8)                         */
  double mu;            /* regularisation of the preconditioned A + mu M (Section 5);
                           <= 0 selects mu = max(lambda_p / 40, lambda_1 / 2) of the homogeneous
                           cell at k = 0, p = nev + nthrow                                 */
  double zero_rel;      /* extrapolation skips Ritz values below zero_rel times the
                           smallest eigenvalue of the previous parameter (1e-2)            */
  int32_t engine_streams; /* batches and servers: at most this many engines of one shape
                             exist at a time, each on a stream of its own (further problems
                             of the shape wait for a free slot); a shape of which one problem
                             fills the device is spread over them rather than packed into
                             one (1..16, default 3)                                        */
  int32_t tol_abs;      /* 1 = tol bounds the defects ||A e_i - lambda_i M e_i||_2 of the
                           M-normalised vectors (the stopping measure of the band-structure
                           experiment, Section 8), which relres then reports; 0 = relative
                           residuals (0)                                                   */
  int32_t tol_floor;    /* 1 = a pair also counts as converged once its relative residual
                           is below the FP64 rounding floor u ||A||_G / (|lambda_i| m_min),
                           u = 2^-53, ||A||_G = 8 kappa_max / (h1 h2) the stencil's Gershgorin
                           bound, m_min = min(h2/h1, h1/h2): the computed A e of a small
                           eigenvalue cancels to lambda M e and cannot resolve residuals below
                           it (acoustic band next to Gamma on fine meshes); 0 = off (0)    */
  int32_t nested_start; /* 1 = a problem's first Bloch parameter without a start block starts
                           from nested iteration (Section 6): the coarsest level's p smallest
                           non-zero eigenpairs by a dense solve, then prolongation and block
                           iteration to nested_tol on every level up to the finest, all in the
                           engine's device buffers; needs a coarsest level of at most 512
                           edges (checked at creation).  0 = the block in the slot (0)      */
  double nested_tol;    /* relative residual to which the levels below the finest are
                           iterated in the nested start; 0 selects 1e-2                    */
  double lock_rel;      /* soft locking of converged pairs (gradient variant): after a
                           round, the wanted pairs whose stopping measure is at most
                           lock_rel * tol get no preconditioned direction in the next basis
                           [E, C] (their vectors stay in it, so the Ritz step still refines
                           them, and a pair that drifts back above the bound is unlocked in
                           the next round); in a round of several slots, a slot with more
                           locked pairs than another keeps some of them unlocked, so that
                           all slots share one column count.  The stopping test over all nev
                           pairs is unchanged.  0 = off, at most 1 (0)                      */
  int32_t throw_precond; /* throw-away vectors (Section 7) that receive a preconditioned
                            direction in each round: the first throw_precond of them (next
                            to the wanted pairs); the others stay in the block E and are
                            refined by the Ritz step only (gradient variant).  0 = all (0)  */
  int32_t reserved_opts; /* must be 0                                                    */
} bl_opts;

/* Read-only facts about a solver handle. */
typedef struct bl_info {
  int32_t n, m, p, nev, levels, precision;
  int32_t level_n[16], level_m[16];
  double mu;
  size_t device_bytes;  /* device memory held by the handle */
  int64_t kernel_launches; /* launches issued since creation */
  int32_t edge_smooth_shape[3];  /* chosen launch shape of the edge smoother: threads per
                                    block, columns per thread, XCD-major order (0/1)   */
  int32_t nodal_smooth_shape[3]; /* same for the nodal smoother                        */
  int32_t rr_tile;      /* Rayleigh-Ritz output tile for the 2p-wide basis: 48 or 64   */
  int32_t fused_edge_level;   /* first level of the edge V-cycle run fused, -1 = none    */
  int32_t fused_nodal_level;  /* same for the nodal V-cycle (cycle precision)            */
  int32_t reserved;
  double autotune_ms;   /* time spent tuning at creation (0 when cached or off)        */
  int64_t locked_columns; /* columns left without a preconditioned direction (soft
                             locking, bl_opts.lock_rel, and the throw-away vectors past
                             bl_opts.throw_precond), summed over the iterations and slots
                             since creation                                             */
} bl_info;

/* Fill *opts with the defaults for `nev` wanted eigenpairs (nthrow = nev/2). */
void bl_default_opts(bl_opts* opts, int32_t nev);

/* Create a solver for the grid and permittivity (Section 1: eps periodic; Section 3:
 * piecewise constant per cell).  eps_cells: host array of n*m values > 0, finite, in cell
 * order; it is copied.  opts may be NULL (defaults for nev = 8).  stream: a hipStream_t
 * or NULL.  Sets up the multigrid hierarchy (bisection, Section 5) and the stabilised
 * node-patch factors (Section 5).  Errors: BL_EINVAL (sizes, eps, options), BL_ENOMEM,
 * BL_EHIP.  *out is NULL on error. */
int bl_create(const bl_grid* grid, const double* eps_cells, const bl_opts* opts,
              void* stream, bl_solver** out);

/* Free everything the handle owns.  NULL is allowed. */
void bl_destroy(bl_solver* s);

/* Device memory a solver for (grid, opts) will hold, in bytes (admission control). */
size_t bl_footprint_bytes(const bl_grid* grid, const bl_opts* opts);

int bl_get_info(const bl_solver* s, bl_info* out);

/* Solve for one Bloch parameter k (Section 4 iteration).
 * start_dev: device FP64 planar block of p = nev+nthrow columns of length N_e used as the
 *   starting block (it is null-space projected, M-orthonormalised and Ritz-rotated), or
 *   NULL to extrapolate from the eigenvector blocks of the previously solved parameters
 *   kept in the handle (Section 6); if NULL and no history exists: the nested start when
 *   opts.nested_start is set, else BL_ESTATE.
 * evals (host, nev), relres (host, nev): results; iters (host, 1): iterations used.
 * evecs_dev: NULL or device FP64 planar block of nev columns receiving M-orthonormal
 *   eigenvectors (each column's phase is arbitrary).
 * The solved block is pushed onto the handle's history (depth extrap_depth). */
int bl_solve_k(bl_solver* s, double k1, double k2, const void* start_dev, double* evals,
               double* relres, int32_t* iters, void* evecs_dev);

/* Band path: bl_solve_k for ks[2*t], ks[2*t+1], t = 0..nk-1, the first from start_dev
 * (or from the history when start_dev is NULL), every later one extrapolated from up to
 * extrap_depth predecessors (Section 6).  evals, relres: host nk*nev (row t = point t);
 * iters: host nk.  evecs_last_dev: NULL or device block of nev columns for the last
 * point.  Returns the first non-OK status, after finishing the path (BL_ENOCONV points
 * keep their best approximations). */
int bl_solve_path(bl_solver* s, const double* ks, int32_t nk, const void* start_dev,
                  double* evals, double* relres, int32_t* iters, void* evecs_last_dev);

/* ---- Bloch-parameter grid (Section 6) ----------------------------------------------------
 * The kappa x kappa grid k_ij = (pi/a (2 i/(kappa-1) - 1), pi/b (2 j/(kappa-1) - 1)),
 * i, j = 0..kappa-1, solved in raster order: row j = 0..kappa-1, in a row i = 0..kappa-1.
 * bl_raster_sources: the points whose eigenvector blocks give the start block of (i, j),
 *   oldest first, as (i', j') pairs in src (host, room for 3 pairs): none for (0, 0); in the
 *   first row the up to three points to the left; in columns 0..2 the up to three points
 *   below; elsewhere the three points to the left (the paper states this rule for rows
 *   j >= 3; rows 1 and 2 are read the same way).  Returns their number (0..3); BL_EINVAL for
 *   kappa < 2, src NULL or (i, j) outside the grid.  Host code only (no device work).
 * bl_solve_kgrid: solves every point, (0, 0) from start_dev (device FP64 planar block of p
 *   columns, required), every other one from the Rayleigh-quotient extrapolation over its
 *   sources (at most extrap_depth of them, the most recent first), each then iterated as in
 *   bl_solve_k.  evals, relres: host kappa*kappa*nev (row j*kappa + i); iters: host
 *   kappa*kappa.  Holds 15 more blocks of p columns on the device while it runs (BL_ENOMEM
 *   when they cannot be allocated); the handle's history afterwards holds the blocks of the
 *   last point's sources and the last point.  Returns BL_EINVAL (arguments), BL_EHIP, or
 *   after finishing the grid the first non-OK point status (BL_ENOCONV points keep their
 *   best approximations). */
int bl_raster_sources(int32_t kappa, int32_t i, int32_t j, int32_t* src);
int bl_solve_kgrid(bl_solver* s, int32_t kappa, const void* start_dev, double* evals,
                   double* relres, int32_t* iters);

/* Nested iteration for a first Bloch parameter (Section 6): the p smallest non-zero
 * eigenpairs of the coarsest level's pencil by a direct (dense) solve, then level by level
 * up the hierarchy: the block is prolongated to the next finer level and, below the finest
 * level, iterated there (that level taken as the finest of its own hierarchy, with the
 * handle's options and mu, to the relative residual tol_levels) before moving on, all in
 * the handle's own device buffers (the same path as the nested_start option).  out_dev
 * (device FP64 planar block of p columns of length N_e) receives the block prolongated to
 * the finest level: the start block of bl_solve_k / bl_solve_path / a batch problem.
 * level_iters: NULL or host array of `levels` entries receiving the iterations per level
 * (0 for the finest and the coarsest).  Errors: BL_EINVAL (arguments, or a coarsest level
 * of more than 512 edges), BL_ENOCONV (fewer than p non-zero coarse eigenvalues), BL_ENOMEM,
 * BL_EHIP.  Sets the handle's Bloch parameter for bl_apply to k. */
int bl_nested_start(bl_solver* s, double k1, double k2, double tol_levels, void* out_dev,
                    int32_t* level_iters);

/* Forget the extrapolation history. */
int bl_reset_history(bl_solver* s);

/* Per-iteration record of the last bl_solve_k: up to `cap` entries of nev relative
 * residuals each (host, row = iteration 0..), returns the number of rows written. */
int bl_last_residual_history(const bl_solver* s, double* relres, int32_t cap);

/* ---- Operator-level entry points (kernel tests and measurement) ------------------------
 * bl_set_k fixes the Bloch parameter for bl_apply (and assembles the coarse factors).
 * bl_apply runs one operator on `ncols` columns.  `prec` 0 = FP64 blocks, 1 = FP32.
 * `level` indexes the multigrid hierarchy (0 = finest).  Shapes per op:
 *   BL_OP_A, BL_OP_M, BL_OP_K    out = A x, M x, (A + mu M) x          edge -> edge
 *   BL_OP_LIFT                   out = L x (gradient of a nodal field) nodal -> edge
 *   BL_OP_LHM                    out = L^* M x                         edge -> nodal
 *   BL_OP_P                      out = L^* M L x (9-point, Section 5)  nodal -> nodal
 *   BL_OP_EDGE_SMOOTH            out (in/out, edge) <- one forward colour sweep 0..3 of
 *                                node-patch block Gauss-Seidel for K x = y (y = rhs)
 *   BL_OP_EDGE_SMOOTH_BACK       same with colours 3..0
 *   BL_OP_NODAL_SMOOTH           out (in/out, nodal) <- forward point GS sweep for P
 *   BL_OP_EDGE_VCYCLE            out = V-cycle(K, level) applied to x (zero start)
 *   BL_OP_NODAL_VCYCLE           out = V-cycle(P, level) applied to x (zero start)
 *   BL_OP_EDGE_PROLONG           out(level) = Pr x(level+1)            edge
 *   BL_OP_EDGE_RESTRICT          out(level+1) = Pr^* x(level)          edge
 *   BL_OP_NODAL_PROLONG          out(level) = Pn x(level+1)            nodal
 *   BL_OP_NODAL_RESTRICT         out(level+1) = Pn^* x(level)          nodal
 *   BL_OP_PROJECT                out = x - L Phi, Phi from nodal_cycles V-cycles for
 *                                P Phi = L^* M x (and the k = 0 deflation) (Section 4)
 *   BL_OP_COARSE_EDGE            out = K_c^{-1} x on the coarsest level
 *   BL_OP_COARSE_NODAL           out = P_c^{+} x on the coarsest level
 *   BL_OP_EIGRES                 out = A x_j - lambda_j M x_j (the iteration's residual,
 *                                Section 4), lambda = y: ncols FP64 values on the device
 *   BL_OP_EDGE_SWEEP             out <- one tiled sweep (colours 0..3, one launch) of the
 *                                node-patch Gauss-Seidel for K out = y, starting from x
 *                                (x and out must be different blocks)
 *   BL_OP_EDGE_SWEEP_BACK        same with colours 3..0
 *   BL_OP_NODAL_SWEEP            out <- one tiled point Gauss-Seidel sweep for P out = y
 *                                from x (colours 0..3); BL_OP_NODAL_SWEEP_BACK: 3..0
 * x, y, out: device blocks (y for the smoothers and sweeps).  Errors: BL_EINVAL, BL_ESTATE
 * (no k set), BL_EHIP. */
enum {
  BL_OP_A = 0, BL_OP_M = 1, BL_OP_K = 2, BL_OP_LIFT = 3, BL_OP_LHM = 4, BL_OP_P = 5,
  BL_OP_EDGE_SMOOTH = 6, BL_OP_EDGE_SMOOTH_BACK = 7, BL_OP_NODAL_SMOOTH = 8,
  BL_OP_EDGE_VCYCLE = 9, BL_OP_NODAL_VCYCLE = 10, BL_OP_EDGE_PROLONG = 11,
  BL_OP_EDGE_RESTRICT = 12, BL_OP_NODAL_PROLONG = 13, BL_OP_NODAL_RESTRICT = 14,
  BL_OP_PROJECT = 15, BL_OP_COARSE_EDGE = 16, BL_OP_COARSE_NODAL = 17, BL_OP_EIGRES = 18,
  BL_OP_EDGE_SWEEP = 19, BL_OP_EDGE_SWEEP_BACK = 20, BL_OP_NODAL_SWEEP = 21,
  BL_OP_NODAL_SWEEP_BACK = 22
};
int bl_set_k(bl_solver* s, double k1, double k2);
int bl_apply(bl_solver* s, int32_t op, int32_t level, int32_t prec, int32_t ncols,
             const void* x, const void* y, void* out);

/* Measurement: with timing enabled, every launch of the finest-level edge smoother (a tiled
 * sweep of all four colours, or one colour pass with tiled_sweeps = 0: the V-cycle's
 * dominant kernel) is bracketed by HIP events on the handle's stream; bl_get_timing returns
 * the summed duration in ms, the number of timed launches, the summed column count of those
 * launches and their summed algorithmic HBM bytes (per column: a sweep reads the right-hand
 * side and, unless it starts from zero, the iterate, and writes the iterate; a colour pass
 * reads the iterate and half the right-hand side and writes half the iterate; per slot the
 * cell coefficients and the patch inverses once) since timing was (re)enabled.  Enabling
 * allocates 4096 events (BL_EHIP on failure); at most 2048 launches are timed between two
 * residual evaluations. */
int bl_set_timing(bl_solver* s, int32_t enable);
int bl_get_timing(const bl_solver* s, double* total_ms, int64_t* launches, int64_t* columns, double* alg_bytes);

/* Dense FP64 helpers of the Ritz step (Section 4), exposed for tests.
 * bl_gram: out (host q x r, row-major complex interleaved re,im) = X^* W for device
 *   planar FP64 blocks X (q columns) and W (r columns) of length len.
 * bl_ritz_small: generalized Hermitian eigenproblem H y = theta G y for host q x q
 *   row-major interleaved complex G (Hermitian positive semi-definite) and H (Hermitian):
 *   G is orthonormalised by pivoted Cholesky of its unit-diagonal scaling; directions whose
 *   squared distance from the kept ones is below 1e-10 (relative) are dropped; the `want` smallest
 *   Ritz values above zero_thr are returned in theta (host) and their G-orthonormal
 *   coefficient vectors in Y (host q x want, row-major interleaved).  Runs on the GPU;
 *   1 <= q <= 512, 1 <= want <= q (else BL_EINVAL).
 *   Returns the number of values found (>= 0) or an error. */
int bl_gram(bl_solver* s, const void* X, int32_t q, const void* W, int32_t r, int64_t len,
            double* out);
int bl_ritz_small(bl_solver* s, const double* G, const double* H, int32_t q, int32_t want,
                  double zero_thr, double* theta, double* Y);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): bl_gram with no allocation.  out_dev
 * (device, q x r, row-major complex interleaved re,im, caller-owned) = X^* W for the device
 * planar FP64 blocks X (q columns) and W (r columns) of length len, queued on the handle's
 * stream (valid once the stream has been synchronised; no host copy, no synchronisation).
 * The row-block partial sums use a fixed per-GPU device array of 2^21 doubles (16 MiB,
 * held until the process ends) instead of a per-call allocation: BL_EINVAL when
 * row blocks (ceil(len / 1024), at most 256) x q x r x 2 exceeds it, or when the current
 * device is not the handle's.  Every call on one GPU shares that array: calls that overlap
 * on one GPU (other streams or handles) race.  Same kernels and summation order as bl_gram,
 * so the results are bit-identical to it. */
int bl_gram_noalloc(bl_solver* s, const void* X, int32_t q, const void* W, int32_t r, int64_t len,
                    void* out_dev);
/* bl_rr_products: the Ritz step's products G = S^* M S and H = S^* A S (host q x q each,
 *   row-major interleaved complex) for a device planar FP64 block S of q <= 3p columns of
 *   length N_e, with the handle's permittivity and the Bloch parameter of bl_set_k; they
 *   are formed straight from S (M S and A S are not stored).  Errors: BL_EINVAL, BL_ESTATE
 *   (no k set), BL_EHIP. */
int bl_rr_products(bl_solver* s, const void* S, int32_t q, double* G, double* H);

/* ---- Batched solves (many problems in the same launches) --------------------------------
 * Problems of equal shape (n, m, a, b and block width p = nev + nthrow) share one engine:
 * every kernel launch of an iteration round covers all of its problem slots, each with its
 * own permittivity, mu, Bloch parameter, coarse solvers and eigenvector history.  Shapes
 * run on separate streams.  A problem's results do not depend on the other problems of the
 * batch (each slot's arithmetic and reduction order is the same as when it is solved alone). */
typedef struct bl_problem {
  bl_grid grid;
  const double* eps;      /* host, n*m cell values > 0 (read during the call)               */
  int32_t nev, nthrow;    /* wanted pairs and throw-away vectors; p = nev + nthrow <= 80     */
  int32_t nk;             /* Bloch parameters on the path, >= 1                              */
  int32_t reserved0;
  const double* ks;       /* host, 2*nk: k1, k2 per point, solved in order with extrapolation */
  const void* start_dev;  /* device FP64 planar block of p columns of length N_e; NULL only
                             with opts.nested_start (then the nested start)                 */
  double* evals;          /* host out, nk*nev (row t = point t)                              */
  double* relres;         /* host out, nk*nev                                                */
  int32_t* iters;         /* host out, nk                                                    */
  double* point_ms;       /* NULL or host out, nk: wall time from the start of each point to
                             the round in which it converged, ms                             */
  void* evecs_dev;        /* NULL or device FP64 planar block of nev columns, last point     */
  int32_t status;         /* out: BL_OK, BL_ENOCONV, BL_EINVAL, BL_ENOMEM                    */
  int32_t reserved1;
} bl_problem;

/* Solve `count` problems with the common options `opts` (nev and nthrow are taken from each
 * problem; NULL = defaults).  max_slots: most slots per shape engine (0 = as many as the
 * problems of that shape, within 90% of the free device memory).  stream: synchronised
 * before the start blocks are read; the work runs on streams of the library's own.
 * Returns BL_OK when every problem succeeded, else the first failing status (per-problem
 * statuses in bl_problem.status; results of BL_ENOCONV problems hold the best values). */
int bl_batch_solve(const bl_opts* opts, bl_problem* probs, int32_t count, int32_t max_slots,
                   void* stream);

/* A batch context keeps its shape engines (device memory, coarse set-up buffers) between
 * runs, so that repeated batches of the same shapes allocate nothing.  bl_batch_run has the
 * semantics of bl_batch_solve with the context's options; hbm_budget 0 = 90% of the free
 * device memory at creation. */
typedef struct bl_batch bl_batch;
int bl_batch_create(const bl_opts* opts, int32_t max_slots, size_t hbm_budget, bl_batch** out);
int bl_batch_run(bl_batch* b, bl_problem* probs, int32_t count, void* stream);
void bl_batch_destroy(bl_batch* b);
/* Facts about the context's live engines (one per shape and slot group): fills *out for
 * engine `index` when it exists and returns the number of live engines (>= 0). */
int bl_batch_engine_info(const bl_batch* b, int32_t index, bl_info* out);
/* Finest-level smoother timing (as bl_set_timing / bl_get_timing) summed over every engine
 * of the context, including engines released since timing was enabled. */
int bl_batch_set_timing(bl_batch* b, int32_t enable);
int bl_batch_get_timing(const bl_batch* b, double* total_ms, int64_t* launches, int64_t* columns,
                        double* alg_bytes);

/* ---- Serving: asynchronous requests with continuous batching -----------------------------
 * A server owns a worker thread that admits requests by device-memory footprint (engines of
 * the request's shape with a free slot, or a new engine within hbm_budget bytes; idle
 * engines of other shapes are released to make room), runs iteration rounds over every busy
 * engine, and lets requests that arrive while others run join at the next round. */
typedef struct bl_server bl_server;

typedef struct bl_request {
  bl_grid grid;
  const double* eps;      /* host, n*m (copied by bl_server_submit)                          */
  int32_t nev, nthrow, nk, reserved0;
  const double* ks;       /* host, 2*nk (copied)                                             */
  const void* start_dev;  /* device FP64 planar block of p columns, written completely
                             before the call (the server reads it on a stream of its own);
                             must stay valid and unchanged until the result is polled; NULL
                             only with opts.nested_start (then the nested start)           */
} bl_request;

typedef struct bl_request_info {
  int32_t status;         /* the request's status (as returned by bl_server_poll)            */
  int32_t total_iters;    /* iterations summed over the path                                 */
  double queue_s;         /* submit -> admitted to a slot, seconds                           */
  double run_s;           /* admitted -> results complete                                    */
  double latency_s;       /* submit -> results complete                                      */
} bl_request_info;

typedef struct bl_server_counters {
  int64_t rounds;          /* iteration rounds run                                           */
  int64_t kernel_launches; /* launches issued by all engines                                 */
  size_t device_bytes;     /* device memory held by the live engines                          */
  int32_t engines;         /* live engines                                                   */
  int32_t queued;          /* requests waiting for admission                                  */
  int32_t pending;         /* requests submitted and not yet polled                           */
  int32_t reserved;
} bl_server_counters;

/* opts: common options (nev, nthrow from each request; NULL = defaults).  hbm_budget: device
 * bytes the engines may hold (0 = 90% of the free memory).  max_slots: most slots per
 * engine (0 = 256).  The server works on the device current at creation. */
int bl_server_create(const bl_opts* opts, size_t hbm_budget, int32_t max_slots, bl_server** out);
/* Queue a request; *ticket identifies it.  Validation errors are returned here. */
int bl_server_submit(bl_server* s, const bl_request* req, uint64_t* ticket);
/* BL_EAGAIN while the request runs; otherwise copies the results (evals, relres nk*nev,
 * iters nk, each may be NULL), fills *info (may be NULL), forgets the ticket and returns
 * the request's status.  BL_EINVAL for an unknown ticket. */
int bl_server_poll(bl_server* s, uint64_t ticket, double* evals, double* relres,
                   int32_t* iters, bl_request_info* info);
/* Counters; returns the worker's error (BL_OK while it runs). */
int bl_server_stats(bl_server* s, bl_server_counters* out);
/* Stop the worker and free every engine; results not polled are lost. */
void bl_server_destroy(bl_server* s);

const char* bl_strerror(int code);
/* Message of the most recent error on the calling thread (static storage). */
const char* bl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BLOCH_H_ */
