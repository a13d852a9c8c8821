/*
 * pn.h -- C ABI of the MI355X (gfx950) staggered-grid real P_N solver.
 *
 * Method: Koerner, Portsmouth & Jakob, "P_N-Method for Multiple Scattering in
 * Participating Media" (EGSR 2018).  The radiative transfer equation is
 * projected onto real spherical harmonics up to order N ((N+1)^2 coefficients
 * L^{l,m}, section "Real-valued P_N-Equations"), discretised by central
 * differences on a staggered voxel grid (section "Precomputation") and the
 * resulting sparse system A u = Q (section "Discretized Radiative Transfer
 * Equation", A = T + C - S) is solved iteratively on the normal equations
 * A^T A u = A^T Q (section "Runtime").
 *
 * Conventions common to every entry point
 *  - All array pointers are DEVICE pointers (HIP device memory of the current
 *    device) unless stated otherwise.  The caller owns them; the library never
 *    frees them.  The library owns its context and workspace (pn_destroy).
 *  - Cell-centred fields are nz*ny*nx arrays, x fastest, z slowest.
 *  - Solution / right-hand-side vectors use the "staggered SoA" layout reported
 *    by pn_layout_query: coefficient k = l*l + l + m occupies the contiguous
 *    range [offset[k], offset[k+1]) and is itself an (ez, ey, ex) array (x
 *    fastest) over the lattice of its staggering class (cls[k] = (px,py,pz)).
 *    A class with p_d = 1 sits on the cell faces normal to axis d; under the
 *    vacuum boundary its extent along d is n_d + 1 (both boundary faces), under
 *    the periodic boundary it is n_d.  Classes follow the reflection parities
 *    of Y_R^{l,m}: px = m mod 2 (m >= 0) or (|m|+1) mod 2 (m < 0),
 *    py = [m < 0], pz = (l + |m|) mod 2.
 *  - Errors are reported by status code, never by exception or abort.
 *    pn_last_error(ctx) returns a message for the last failing call on ctx.
 *  - A context is bound to one HIP stream (given at setup).  pn_apply and
 *    pn_apply64 are asynchronous on that stream; pn_solve and pn_residual64
 *    return after the result is complete (they synchronise with the host).
 *  - Calls on one context must not overlap (contexts are not thread-safe).
 */
#ifndef PN_H
#define PN_H

#ifdef __cplusplus
extern "C" {
#endif

#define PN_ABI_VERSION 1
#define PN_MAX_ORDER 7
#define PN_MAX_COEFF 64

typedef struct pn_ctx pn_ctx;

typedef enum {
  PN_OK = 0,
  PN_ERR_ARG = 1,            /* invalid argument (null pointer, order, size)  */
  PN_ERR_ALLOC = 2,          /* device or host allocation failed              */
  PN_ERR_HIP = 3,            /* a HIP runtime call failed                     */
  PN_ERR_NONFINITE = 4,      /* NaN/Inf in the medium or the right-hand side  */
  PN_ERR_NOT_CONVERGED = 5,  /* tolerance not reached within the limits       */
  PN_ERR_BREAKDOWN = 6       /* Krylov breakdown (zero curvature)             */
} pn_status;

typedef enum { PN_BC_VACUUM = 0, PN_BC_PERIODIC = 1, PN_BC_NEUMANN = 2, PN_BC_PER_AXIS = 3 } pn_bc;
typedef enum { PN_FP32_IR = 0, PN_FP64 = 1 } pn_precision;

/* Grid of nx*ny*nz cells of edge h (h <= 0 selects h = 1/nx, i.e. the unit
 * cube for cubic grids).  bc, the same on every axis: PN_BC_VACUUM =
 * homogeneous Dirichlet on every coefficient (the paper's Dirichlet mode:
 * entries referencing a location outside the domain are dropped, section
 * "Runtime"), PN_BC_PERIODIC = wrap-around, PN_BC_NEUMANN = the paper's
 * Neumann mode (such an entry moves to the coefficient at the closest
 * location inside the domain, section "Runtime"); PN_BC_PER_AXIS: the type
 * of axis d is bc_axis[d] (one of the three; e.g. a 2D problem as one
 * periodic cell in z).  Face-centred classes have n_d + 1 points along a
 * vacuum or Neumann axis, n_d along a periodic one. */
typedef struct {
  int nx, ny, nz;
  double h;
  int bc;
  int bc_axis[3];     /* used when bc == PN_BC_PER_AXIS */
} pn_grid;

/* RTE parameters at the cell centres (section "Runtime": "RTE parameter
 * fields").  sigma_t: extinction; albedo: sigma_s / sigma_t; g: the
 * Henyey-Greenstein mean cosine, uniform over the medium (the phase-function
 * moments enter as lambda_l p^{l,0} = g^l, appendix "Scattering term");
 * sigma_t_min: every cell with sigma_t < sigma_t_min is raised to it (the
 * paper's extinction threshold; vacuum makes A singular).  sigma_s is
 * albedo * thresholded sigma_t.  Both arrays are device FP32, nz*ny*nx.  The
 * library copies what it needs at setup; the caller may free them after. */
typedef struct {
  const float* sigma_t;
  const float* albedo;
  float g;
  float sigma_t_min;
} pn_medium;

typedef struct {
  int order, ncoeff;
  int nx, ny, nz, bc;
  int bc_axis[3];                    /* boundary type of each axis           */
  long long n_unknowns;
  int cls[PN_MAX_COEFF][3];
  int ext[PN_MAX_COEFF][3];          /* (ex, ey, ez) per coefficient          */
  long long offset[PN_MAX_COEFF + 1];
} pn_layout;

typedef struct {
  int precision;      /* PN_FP32_IR (FP32 Krylov + FP64 refinement) or PN_FP64 */
  int max_iter;       /* total Krylov iterations over all refinement steps    */
  int max_refine;     /* refinement steps (PN_FP32_IR)                         */
  double inner_tol;   /* relative reduction of the inner FP32 residual         */
  int use_guess;      /* 0: start from x = 0; 1: start from the x passed in    */
  int graph_iters;    /* Krylov iterations per captured HIP graph launch (the
                         host reads the stop flag after each launch)           */
  int variant;        /* PN_VARIANT_AUTO, _CGLS, _CG, _CG_EQ, _SCHUR, _SCHUR_MG */
  int learned;        /* PN_LEARNED_* (needs a network, pn_attach_net in pn_nn.h) */
} pn_solve_opts;

/* Learned start and correction (PN_FP32_IR only; ignored without a network):
 * OFF: plain solve.  GUESS: the initial iterate is s * u, u the network's
 * prediction for the medium and Q, s the scalar minimising ||Q - s A u||_2,
 * kept only if it cuts the residual below 0.9 ||Q|| (use_guess = 0 only;
 * info->learned_ratio reports the ratio either way).
 * GUESS_CORRECT: also, before every inner solve whose preceding step was not
 * itself a correction, x += s * u with u the prediction for the current
 * residual and s chosen the same way, kept only if it cuts the residual
 * norm below 0.9 of its value (a flexible, residual-minimising preconditioner
 * step of the refinement). */
#define PN_LEARNED_OFF 0
#define PN_LEARNED_GUESS 1
#define PN_LEARNED_GUESS_CORRECT 2

/* Krylov variant of the FP32 inner solve.  SCHUR: the even-parity form.  The
 * transport couples only bands l and l +- 1, and the band parity of a
 * coefficient is the parity of its staggering class, so with u = (u_e, u_o)
 * (even / odd l) A = [[D_e, T_eo], [T_oe, D_o]] with D_e, D_o diagonal and,
 * when no axis is Neumann, T_oe = -T_eo^T (the transport part is skew,
 * section "Discretized Radiative Transfer Equation").  The inner solve then
 * runs conjugate gradients with a Jacobi preconditioner on the symmetric
 * positive definite Schur complement S = D_e - T_eo D_o^-1 T_oe for u_e
 * (right-hand side r_e - T_eo D_o^-1 r_o) and recovers u_o = D_o^-1 (r_o -
 * T_oe u_e); its residual equals that of the whole system, and the inner stop
 * tests it against inner_tol times the refinement residual.  One iteration
 * applies A once (odd rows from the even part, then even rows), where CG on
 * the normal equations applies A and A^T.  PN_ERR_ARG with a Neumann axis, with
 * zero extinction in some cell (D_o singular: raise sigma_t_min) or PN_FP64.
 * SCHUR_MG: the same PCG with a multigrid preconditioner in place of the
 * Jacobi one.  S couples every even coefficient to itself only at the six
 * lattice neighbours (a weighted diffusion operator per coefficient, the
 * band-l form of the diffusion equation that P1 collapses to, section
 * "Results"), so B r = 0.6 M r + P V(P^T r): M the Jacobi inverse diagonal,
 * P the piecewise-constant prolongation over 2 x 2 x 2 aggregates of each
 * coefficient's lattice and V one V-cycle on the Galerkin coarse operators
 * (damped Jacobi smoothing, coarsening down to at most 5 points per axis).
 * B is symmetric positive definite and formed per solve from the medium;
 * the solution is the same, only the iteration count changes.  A periodic
 * axis is cut at its seam in the preconditioner only (the solve stays
 * periodic).  PN_ERR_ARG where SCHUR is refused.
 * CGLS: the residual-based CGLS
 * form (r <- r - alpha q fused into s = A^T r).  CG: CG on the normal
 * equations A^T A u = A^T Q with the recursive normal residual
 * (s <- s - alpha A^T q, ||r||^2 <- ||r||^2 - alpha gamma; 10 vector passes
 * per iteration, and the A^T pass streams one vector instead of two), on
 * whichever stencil is in use.  CG_EQ: the same on the row-equilibrated
 * system W A u = W Q, W = diag(1 / ||row of A||_2) (the row norm taken with
 * every transport neighbour present, formed from the medium inside the
 * kernels: no extra memory traffic); the inner stop then tests the W-weighted
 * residual.  Needs the register-window stencil (PN_ERR_ARG with pn_set_tiles
 * or PN_FP64).  AUTO: on the register-window stencil SCHUR_MG for odd orders
 * with at least 2^17 even-band unknowns, SCHUR otherwise (CG_EQ when an axis
 * is Neumann or some cell has zero extinction); CG on the LDS-tiled one; the
 * batched solve treats AUTO as CG_EQ.  The FP64 refinement checks the true, unweighted residual
 * ||Q - A x|| in every case. */
#define PN_VARIANT_AUTO 0
#define PN_VARIANT_CGLS 1
#define PN_VARIANT_CG 2
#define PN_VARIANT_CG_EQ 3
#define PN_VARIANT_SCHUR 4
#define PN_VARIANT_SCHUR_MG 5

#define PN_MAX_HISTORY 64
/* Phases of a solve timed in pn_solve_info.t_ms (wall milliseconds, host
 * clock at the points where the solve synchronises with the device):
 * SETUP: argument checks, the non-finite check of Q, packing Q and x0;
 * RESIDUAL: the FP64 residual evaluations of the refinement; KRYLOV: the FP32
 * (or FP64) inner Krylov solves; LEARNED: network predictions and their
 * residual-minimising scaling; FINISH: unpacking x. */
#define PN_PHASES 5
#define PN_PHASE_SETUP 0
#define PN_PHASE_RESIDUAL 1
#define PN_PHASE_KRYLOV 2
#define PN_PHASE_LEARNED 3
#define PN_PHASE_FINISH 4
typedef struct {
  int status;
  int outer_iters;          /* FP64 residual evaluations                       */
  int inner_iters;          /* Krylov iterations (each = one A and one A^T)    */
  double rel_residual;      /* ||Q - A x||_2 / ||Q||_2 in FP64 at exit         */
  double bnorm;             /* ||Q||_2                                         */
  double seconds;           /* wall time of the solve                          */
  int nhistory;
  double history[PN_MAX_HISTORY]; /* FP64 relative residual per refinement step */
  int learned_steps;        /* learned guesses / corrections applied           */
  double learned_ratio;     /* residual ratio the learned initial guess offers  */
  double t_ms[PN_PHASES];   /* wall milliseconds per phase (PN_PHASE_*); zero in
                               the per-system infos of pn_batch_solve           */
  double bytes;             /* algorithmic memory traffic of the solve's kernels:
                               vector elements each kernel must read and write
                               (per unknown) and the medium (8 bytes per cell
                               per stencil pass) -- not a counter reading       */
  double achieved_gbs;      /* bytes / (RESIDUAL + KRYLOV time), GB/s; zero in
                               the per-system infos of pn_batch_solve           */
} pn_solve_info;

int pn_abi_version(void);
const char* pn_status_string(int status);

/* Default options: FP32_IR, max_iter 200000, max_refine 40, inner_tol 1e-2,
 * use_guess 0, graph_iters 8, variant AUTO, learned OFF. */
void pn_default_opts(pn_solve_opts* opts);

/* Builds a solver context for truncation order 1 <= order <= 7 on `grid`
 * with `medium` (section "Runtime": the system is built from the RTE
 * parameter fields, the resolution and the boundary type).  The
 * transport couplings int omega_d Y^k Y^k' are the closed forms of the
 * appendix ("Final equation", real-valued derivation).  Thresholds sigma_t,
 * checks the medium for NaN/Inf (PN_ERR_NONFINITE) and allocates the Krylov
 * workspace (5 FP32 vectors).  `stream` is a hipStream_t (NULL = the null
 * stream).  On failure *out is NULL. */
pn_status pn_setup(int order, const pn_grid* grid, const pn_medium* medium,
                   void* stream, pn_ctx** out);

/* Fills *layout (host struct) with the staggered SoA layout of ctx. */
pn_status pn_layout_query(const pn_ctx* ctx, pn_layout* layout);

/* y = A x (transpose == 0) or y = A^T x (transpose != 0) in FP32, where A is
 * the discretised operator of section "Discretized Radiative Transfer
 * Equation": per row of coefficient k (band l) at lattice point x_i,
 *   sum_d sum_k' A_d[k,k'] (x_k'(x_i + h/2 e_d) - x_k'(x_i - h/2 e_d)) / h
 *   + (sigma_t(x_i) - g^l sigma_s(x_i)) x_k(x_i)
 * with sigma_t, sigma_s averaged from the adjacent cell centres.  A^T flips
 * the sign of the transport part (it is skew-symmetric).  x and y are device
 * FP32 vectors of n_unknowns entries and must not overlap.  Asynchronous. */
pn_status pn_apply(pn_ctx* ctx, const float* x, float* y, int transpose);

/* The operator of the even-parity solve (PN_VARIANT_SCHUR) in FP32, with
 * A = [[D_e, T_eo], [T_oe, D_o]] split by band parity (even / odd l):
 *   y_o = -D_o^-1 T_oe x_e,   y_e = D_e x_e + T_eo y_o = S x_e,
 * S = D_e - T_eo D_o^-1 T_oe the Schur complement of the even bands.  Reads
 * only the even-band entries of x (packed layout, n_unknowns entries) and
 * writes every entry of y.  These are the two stencil passes of one PCG
 * iteration.  PN_ERR_ARG with a Neumann axis (there T_oe != -T_eo^T and the
 * solve does not use S).  Asynchronous on the context stream. */
pn_status pn_apply_schur(pn_ctx* ctx, const float* x, float* y);

/* The preconditioner of the even-parity solve applied to r: z_e = B r_e on
 * the even-band entries, z_o = 0.  variant PN_VARIANT_SCHUR: B = M, the
 * Jacobi inverse diagonal of S (bfloat16); PN_VARIANT_SCHUR_MG: B = 0.6 M +
 * P V P^T, the multigrid form (see the variants below).  B is symmetric positive definite and depends on the medium
 * only; it is formed at the first call (or solve) and kept.  r, z: device
 * FP32 packed vectors (n_unknowns), not overlapping.  Overwrites the Krylov
 * workspace (a following pn_solve re-initialises it).  PN_ERR_ARG for another
 * variant, a Neumann axis or zero extinction.
 * Asynchronous on the context stream. */
pn_status pn_apply_precond(pn_ctx* ctx, int variant, const float* r, float* z);

/* Single-scattered light of a point light folded into the emission term
 * (section "Rendering"): writes rhs (DEVICE FP32, packed layout, n_unknowns
 * entries) with, at the location y of every unknown (coefficient k = (l, m)),
 *   Q^{l,m}(y) = sigma_s(y) power exp(-tau) / (4 pi r^2) g^l Y_R^{l,m}(w),
 * the in-scattered uncollided light: r = |y - light| (at least h / 2), w =
 * (y - light) / r, tau = the optical depth of the segment light -> y through
 * the thresholded extinction of the cells (constant per cell, zero outside
 * the grid), sigma_s the mean of the cells adjacent to y, and g^l Y_R^{l,m}(w)
 * the projection of the Henyey-Greenstein phase function.  light: HOST array
 * of 3 physical coordinates (the grid spans [0, n_d h] along axis d; the light
 * may lie outside).  Solving with this right-hand side gives the
 * multiple-scattered light.  PN_ERR_ARG on a periodic axis or non-finite
 * arguments.  Asynchronous on the context stream. */
pn_status pn_single_scatter(pn_ctx* ctx, const double* light, double power, float* rhs);

/* Un-staggering (section "Rendering"): every coefficient of the solution x
 * (DEVICE FP64, packed layout) interpolated to the voxel centres -- its own
 * lattice point along an axis where its class is centred, the mean of the
 * cell's two faces where it sits on faces (face n is face 0 on a periodic
 * axis); the extra boundary coefficients are dropped.  out: DEVICE FP32
 * [ncoeff][nz][ny][nx].  Asynchronous on the context stream. */
pn_status pn_unstagger(pn_ctx* ctx, const double* x, float* out);

/* Row weights of the equilibrated CG variant (PN_VARIANT_CG_EQ): w[i] =
 * 1 / (d_i^2 + sum of the squared transport entries of row i with every
 * neighbour present), d_i the diagonal -- 1 / ||row i of A||_2^2 away from
 * the boundary, smaller next to a vacuum boundary, where the row loses
 * entries.  w: DEVICE FP32, packed layout, n_unknowns entries.  Async on the
 * context stream. */
pn_status pn_row_weights(pn_ctx* ctx, float* w);

/* Same operator evaluated in FP64 (couplings, interpolation and products in
 * double) on FP64 vectors.  Asynchronous. */
pn_status pn_apply64(pn_ctx* ctx, const double* x, double* y, int transpose);

/* r = Q - A x in FP64 (x FP64, Q FP32, r FP64 output, may be NULL) and the
 * relative residual ||r||_2 / ||Q||_2 written to *rel (host).  Synchronous. */
pn_status pn_residual64(pn_ctx* ctx, const float* rhs, const double* x,
                        double* r, double* rel);

/* Solves A x = Q (rhs = Q, device FP32; x device FP64, in/out) to
 * ||Q - A x||_2 <= tol ||Q||_2 with the residual evaluated in FP64.
 * PN_FP32_IR: iterative refinement around conjugate gradients on the normal
 * equations without forming A^T A (section "Runtime" / "Results"; the
 * row-equilibrated CG by default, plain CG or CGLS on request) run in FP32
 * with FP64 dot products and scalars.  PN_FP64: CGLS in FP64 throughout.  Returns PN_ERR_NOT_CONVERGED (x = last iterate, finite) when
 * the limits are hit, PN_ERR_NONFINITE for a non-finite rhs.  rhs == 0
 * returns x = 0 immediately.  opts NULL = defaults; info may be NULL. */
pn_status pn_solve(pn_ctx* ctx, const float* rhs, double* x, double tol,
                   const pn_solve_opts* opts, pn_solve_info* info);

/* Times `iters` back-to-back FP32 applies (transpose selects A^T) on the
 * library's internal padded workspace -- the apply of the Krylov loop --
 * with HIP events on the context stream; writes the mean milliseconds per
 * apply to *ms_per_apply (host).  Synchronous.  For benchmarking. */
pn_status pn_bench_apply(pn_ctx* ctx, int iters, int transpose, double* ms_per_apply);

/* Times one kernel of the FP32 Krylov loop in its in-loop form on the
 * library's padded workspace, with HIP events on the context stream; writes
 * the mean milliseconds per launch.  The plain applies run `iters` times back
 * to back; the in-loop kernels run inside `iters` iterations of the loop's
 * own kernel sequence (q = W A p, s -= alpha A^T q, x/p update: the cache
 * state of a solve), timed by events around the requested one.  kernel:
 *   PN_KERNEL_APPLY      y = A x (no reduction; as pn_bench_apply)
 *   PN_KERNEL_APPLY_T    y = A^T x
 *   PN_KERNEL_APPLY_EQ   q = W A p with the FP64 partials of <A p, W A p>
 *   PN_KERNEL_SUPD       s -= alpha A^T q with the FP64 partials of ||s||^2
 *   PN_KERNEL_UPDATE     x += alpha p, p = s + beta p
 * Resets the device scalars (the next pn_solve re-initialises them) and
 * overwrites the workspace.  PN_ERR_ARG for an unknown kernel, or for the
 * in-loop kernels while the LDS-tiled stencil is selected.  Synchronous.
 * For benchmarking. */
#define PN_KERNEL_APPLY 0
#define PN_KERNEL_APPLY_T 1
#define PN_KERNEL_APPLY_EQ 2
#define PN_KERNEL_SUPD 3
#define PN_KERNEL_UPDATE 4
/* The kernels of the even-parity loop (PN_VARIANT_SCHUR), timed inside its
 * own kernel sequence:
 *   PN_KERNEL_ODD_W      w_o = -D_o^-1 T_oe p_e (odd rows) with the FP64
 *                        partials of <p, S p> = <p_e, D_e p_e> + <w_o, D_o w_o>
 *   PN_KERNEL_EVEN_R     r_e -= alpha (D_e p_e + T_eo w_o) (even rows) with
 *                        <r, M r>, <r, r>
 *   PN_KERNEL_PCG_XP     x += alpha p, p = M r + beta p
 * and of its multigrid form (PN_VARIANT_SCHUR_MG; PN_ERR_ARG where it does
 * not apply), inside odd rows | even rows | V-cycle | x/p:
 *   PN_KERNEL_MG_VCYCLE  the whole V-cycle on P^T r (restriction, down and up
 *                        passes of every level, coarsest solve), timed as one
 *   PN_KERNEL_PCG_XP_MG  x += alpha p, p = omega_f M r + P z_1 + beta p */
#define PN_KERNEL_ODD_W 5
#define PN_KERNEL_EVEN_R 6
#define PN_KERNEL_PCG_XP 7
#define PN_KERNEL_MG_VCYCLE 8
#define PN_KERNEL_PCG_XP_MG 9
pn_status pn_bench_kernel(pn_ctx* ctx, int kernel, int iters, double* ms);

/* Launch tuning: planes of z handled per thread block in the stencil apply
 * (0 = automatic).  Results do not depend on it (bitwise). */
pn_status pn_set_zchunk(pn_ctx* ctx, int zchunk);
int pn_get_zchunk(const pn_ctx* ctx);

/* Opt-in LDS-tiled FP32 stencil (vacuum boundary): a block owns a tx x ty
 * tile of (x, y) columns and zchunk planes (0 = automatic); pn_apply and the
 * CG variant then use it.  tx = ty = 0 switches back to the register-window
 * stencil (the default).  Fails with PN_ERR_ARG for shapes that do not fit
 * (at most 256 threads, the tile's one-point border no larger than the
 * block, LDS within the device limit).  pn_get_tiles reports the current
 * shape (tx = ty = 0 when the tiled stencil is not in use). */
pn_status pn_set_tiles(pn_ctx* ctx, int tx, int ty, int zchunk);
pn_status pn_get_tiles(const pn_ctx* ctx, int* tx, int* ty, int* zchunk);

/* Coupling table compiled into the library for `order`: writes up to `cap`
 * entries (row k, axis d, column k', value int omega_d Y^k Y^k') into the
 * host arrays and returns the total count (-1 on bad arguments). */
int pn_coupling_table(int order, int* k, int* d, int* kp, double* v, int cap);

/* Launch autotuner: times the FP32 stencil apply of ctx for each candidate
 * z-chunk (planes of z one thread block marches; the launch width against
 * the window re-read at chunk borders) with `iters` timed launches each,
 * keeps the fastest for ctx and records it in the process-wide tune cache
 * under (order, nx, ny, nz, bc).  pn_setup and pn_batch_setup take the launch
 * shape from that cache when it has an entry.  Writes the chosen z-chunk and
 * its mean milliseconds per apply (either pointer may be NULL).  Results do
 * not depend on the launch shape (bitwise).  Synchronous. */
pn_status pn_autotune(pn_ctx* ctx, int iters, int* zchunk, double* ms_per_apply);

/* The tune cache as a text file, one entry per line:
 * "order nx ny nz bc zchunk ms" ('#' starts a comment line), bc = the
 * boundary types of the axes as bc_x + 3 bc_y + 9 bc_z (0..26).  Load merges the
 * file into the cache (PN_ERR_ARG on a missing file or a malformed line; the
 * lines before it are kept). */
pn_status pn_tune_cache_save(const char* path);
pn_status pn_tune_cache_load(const char* path);
int pn_tune_cache_size(void);
void pn_tune_cache_clear(void);

/* ------------------------------------------------------------------------
 * Batched solve: many media of uneven grid size and order, each with nrhs
 * right-hand sides (emission fields), solved together.  A system is one
 * (problem p, right-hand side r) pair, index p * nrhs + r.  Each Krylov stage
 * is one launch over all systems of an order (stencil) or over all systems
 * (scalars, vectors), the iterations are captured in one HIP graph, and every
 * system carries its own device-side scalars and convergence flags, so it
 * stops on its own.  The right-hand sides of one problem share its A; their
 * thread blocks for one tile run next to each other so the medium is fetched
 * from memory once per tile.  Per system the arithmetic is that of pn_solve
 * (the FP32 Krylov variant of opts, FP64 dot products and iterative
 * refinement) with the same launch shape, so results match pn_solve on the
 * same system bitwise.
 * ---------------------------------------------------------------------- */
typedef struct pn_batch pn_batch;

typedef struct {
  int order;          /* 1..7 */
  pn_grid grid;
  pn_medium medium;   /* copied at setup, as for pn_setup */
} pn_problem;

/* Builds the batch: per problem the medium and padded geometry, per system
 * the Krylov workspace (7 FP32 vectors and one FP64 vector of the padded
 * length, about 36 bytes per unknown).  tune != 0 runs the autotuner for every
 * (order, grid, bc) not yet in the tune cache first.  On failure *out is NULL
 * and pn_batch_last_error(NULL) tells why. */
pn_status pn_batch_setup(int nprob, const pn_problem* probs, int nrhs, int tune, void* stream,
                         pn_batch** out);

/* Layout of problem `prob` (as pn_layout_query). */
pn_status pn_batch_layout(const pn_batch* batch, int prob, pn_layout* layout);
/* Context of problem `prob` (geometry and medium, no Krylov workspace):
 * valid for pn_layout_query, pn_net_features and pn_net_targets only; owned
 * by the batch.  Every entry point that needs the Krylov workspace (pn_apply,
 * pn_apply64, pn_row_weights, pn_residual64, pn_solve, the bench and tuning
 * calls, pn_set_zchunk, pn_set_tiles, pn_attach_net) returns PN_ERR_ARG on it
 * without touching the device.  NULL on bad arguments. */
pn_ctx* pn_batch_problem(const pn_batch* batch, int prob);
/* Launch z-chunk used for problem `prob` (-1 on bad arguments). */
int pn_batch_zchunk(const pn_batch* batch, int prob);
/* Total unknowns over all systems. */
long long pn_batch_unknowns(const pn_batch* batch);

/* Solves every system to ||Q - A x||_2 <= tol ||Q||_2.  rhs and x are HOST
 * arrays of nprob * nrhs DEVICE pointers (packed layout of the system's
 * problem; rhs FP32, x FP64 in/out as for pn_solve).  opts as for pn_solve;
 * precision must be PN_FP32_IR.  variant: AUTO (= CG_EQ), CG_EQ, CG or CGLS
 * run every system of an order in shared launches (one captured graph over
 * all systems); SCHUR_MG solves the systems one after another by the
 * single-system multigrid even-parity path (bitwise the result of pn_solve
 * with the same z-chunk), each problem using its first system's scratch
 * vectors as the Krylov workspace and keeping its preconditioner and graph
 * (PN_ERR_ARG when some problem has a Neumann axis or zero extinction); up
 * to four problems run at once, each on its own stream, from host threads;
 * SCHUR is refused.  info: NULL or a host array of
 * nprob * nrhs entries, one per system (seconds = wall time of the whole
 * batch, or of the system's own solve with SCHUR_MG).  Returns
 * PN_OK when every system converged, else the status of the first system that
 * did not (the others are still solved; see info).  Synchronous. */
pn_status pn_batch_solve(pn_batch* batch, const float* const* rhs, double* const* x, double tol,
                         const pn_solve_opts* opts, pn_solve_info* info);

/* Times `iters` batched FP32 applies over every system (each system's
 * direction vector into its product vector, as in the Krylov loop) with HIP
 * events; writes the mean milliseconds per batched apply.  Synchronous. */
pn_status pn_batch_bench_apply(pn_batch* batch, int iters, int transpose, double* ms_per_apply);

void pn_batch_destroy(pn_batch* batch);
const char* pn_batch_last_error(const pn_batch* batch);

/* Frees the context and its workspace.  NULL is ignored. */
void pn_destroy(pn_ctx* ctx);

/* Message of the last failing call on ctx (or of the last failing pn_setup
 * when ctx is NULL).  The string is owned by the library. */
const char* pn_last_error(const pn_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PN_H */
