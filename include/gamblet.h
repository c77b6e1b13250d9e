/*
 * gamblet.h -- C ABI of the MI355X (gfx950) gamblet hierarchy and solve.
 *
 * Problem (Section 1, discrete form of Section 5.1): find the Q1 finite
 * element function u on the unit square meshed by n x n square cells,
 * n = 2^q, h = 1/n, such that <phi_j, u>_a = int phi_j g for every interior
 * node j, with u equal to given Dirichlet values on the boundary.  The
 * coefficient a is one positive value per cell; the source g is one value
 * per cell.
 *
 * Method (Section 4 and Algorithm 2 of Section 5): the fine-to-coarse
 * hierarchy of localized gamblets is built once per coefficient field
 * (gbl_build): for k = q..2, the subband operator B^(k) = W^(k) A^(k) W^(k)T
 * (eq. defining B, Section 4.7), one small SPD patch system per coarse
 * cell (Definition 5.3) giving the restriction R^(k-1,k) = pibar + D W
 * (theorem expressing R through pibar and D), and the Galerkin coarse
 * operator A^(k-1) = R A^(k) R^T (Theorem 4.8).  A solve (gbl_solve)
 * restricts the right-hand side through the levels (eq. g^(k-1) = R g^(k)),
 * solves the independent subband systems B^(k) w^(k) = W^(k) g^(k) and the
 * coarse system A^(1) U^(1) = g^(1) (Section 4.7), and sums the subbands
 * (Theorem 4.15).  Because the hierarchy is localized, that sum is an
 * approximate inverse; gbl_solve wraps it in flexible conjugate gradients on
 * the FP64 fine residual until the requested accuracy is reached (inexact
 * inner solves are allowed, Theorem 5.6).
 *
 * Memory and ownership
 *  - All array arguments named *_dev are device pointers (HIP global memory)
 *    on the current device; the caller owns them and keeps them alive until
 *    the call's stream work has completed.
 *  - The hierarchy lives in one caller-owned device workspace whose size is
 *    given by gbl_workspace_bytes; the library never allocates device memory
 *    itself.  The library owns only the small host-side context returned by
 *    gbl_build, released by gbl_destroy.
 *  - Every call enqueues its kernels on the given stream (0 = null stream)
 *    and, where it must read a device status word, synchronises that stream.
 *
 * Layouts (C order, float64 unless stated)
 *  - cell arrays  [n][n]      : index ex*n + ey, cell [ex h,(ex+1)h) x [ey h,(ey+1)h)
 *  - nodal arrays [n+1][n+1]  : index i*(n+1) + j, node (i h, j h)
 *  - batched arrays carry a leading [nrhs] dimension.
 *
 * Errors: every function returns an int status; nothing throws across the
 * ABI.  gbl_last_error() gives a message for the last failing call on a
 * context (or the last failing context-less call when ctx is NULL).
 */
#ifndef GAMBLET_H
#define GAMBLET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GBL_VERSION 10000 /* 1.0.0 */

enum gbl_status {
  GBL_OK = 0,
  GBL_EINVAL = -1,   /* bad argument: q out of range, null pointer, a <= 0 or non-finite, nrhs too large */
  GBL_ENOTSPD = -2,  /* FP64: a patch or coarse matrix had a non-positive pivot (MIXED: see gbl_build_flags) */
  GBL_ENOCONV = -3,  /* the solve did not reach rtol within max_outer iterations, or diverged (then
                        gbl_solve_info reports NaN); u holds the last iterate */
  GBL_ENOMEM = -4,   /* the workspace is smaller than gbl_workspace_bytes reports */
  GBL_EHIP = -5      /* a HIP runtime call failed */
};

enum gbl_precision {
  GBL_FP64 = 0,   /* hierarchy, patch solves and subband CG in FP64 */
  GBL_MIXED = 1,  /* hierarchy and subband CG in FP32; fine residual, outer iteration and A^(1) in FP64 */
  GBL_MIXED_FP64_BUILD = 2  /* hierarchy built in FP64 (patch solves, Galerkin products, A^(1)), then copied to
                               FP32 for the subband iterations; fine residual and outer iteration in FP64.  For
                               coefficients whose contrast exceeds FP32's resolution (about 1e7), where FP32
                               Galerkin products lose positive definiteness.  The workspace holds both copies */
};

enum gbl_inner {
  GBL_INNER_CHEBYSHEV = 0,  /* Chebyshev iteration: a fixed polynomial preconditioner, no inner products */
  GBL_INNER_CG = 1,         /* conjugate gradients */
  GBL_INNER_CHEB_CG = 2     /* Chebyshev on the finest subband system, conjugate gradients on the coarser ones */
};

typedef struct gbl_opts {
  int rho;            /* patch radius in coarse cells (box |dx|,|dy| <= rho, Definition 5.3) of the finest
                         transition (and of all levels when rho_coarse = 0); 1..4, or 5 with rho_coarse set.
                         The paper sizes the radius of level k like ln(1/H_k), larger on finer levels; with
                         inclusions of very high coefficient about as wide as the finest patches, the finest
                         transition is the one whose radius decides the outer iteration count */
  int precision;      /* enum gbl_precision */
  double rtol;        /* target relative l2 error of u; the solve stops when the larger of ||S r|| and the
                         last correction, over the last two iterations, is below rtol / f of ||u||, with
                         f = max(3, 1 / (1 - c)) and c the per-iteration contraction of these estimates
                         (the larger of the geometric means over the last 16 iterations
                         and over the whole solve, capped at 0.995) */
  int max_outer;      /* maximum outer (flexible CG) iterations */
  int inner_iters;    /* iterations on the finest subband system per outer iteration (Chebyshev: <= 32) */
  int max_rhs;        /* right-hand sides solved together: a solve or adjoint call takes any number of right-
                         hand sides and runs them in blocks of min(max_rhs, 64), every kernel of an iteration
                         launched once for the whole block (each right-hand side with its own copy of the
                         solve vectors, so the workspace grows with it); 1..4096 */
  int inner_iters_coarse; /* iterations on each coarser subband system (k < q) (Chebyshev: <= 32) */
  int inner_kind;     /* enum gbl_inner: the iteration used on the subband systems B^(k) w = W g
                         (Section 4.7), block-Jacobi (3 x 3 parent blocks) preconditioned */
  double kappa;       /* Chebyshev: the interval is [G / kappa, G] on the finest level, G the block-
                         Gershgorin bound of lambda_max computed at build time; > 1 */
  double kappa_coarse;/* the same on the coarser levels */
  int level_q_mass;   /* level-q gamblets: 0 = the nodal basis (psi^(q)_i = phi_i, the default); 1..4 = the
                         localized mass inverse of Algorithm 2 and Definition 5.2 with this patch radius in
                         node steps (psi^(q)_i = sum_j Minv_ji phi_j; see gbl_mass_inverse), with
                         A^(q) = Minv^T A Minv; needs Chebyshev inner iterations and q >= 3 + (level_q_mass
                         > 3); the gamblet transform calls reject such a hierarchy */
  int rho_coarse;     /* patch radius of the transitions below the finest (levels k < q, Algorithm 2 allows
                         one radius per level); 0 = rho; 1..4 */
  double window_tol;  /* window corrections of the subband preconditioner on the levels k < q (0 = off, the
                         default; needs conjugate gradients there: inner_kind GBL_INNER_CG or
                         GBL_INNER_CHEB_CG).  Section 4.8 bounds the condition number of B^(k) by a constant
                         that grows with the contrast of a; with inclusions of very high coefficient the
                         block-Jacobi preconditioned B^(k) keeps a few localized modes of tiny Rayleigh quotient
                         (an inclusion spanning several parents moving almost rigidly).  For every 3 x 3 group
                         of parents (27 subband unknowns) the build factorizes the principal submatrix B_w in
                         FP64 and keeps B_w^-1 when tr(D_w B_w^-1) > window_tol, D_w the block diagonal of B_w
                         (the trace lies between 1 / lambda_min and 27 / lambda_min of the pencil (B_w, D_w));
                         the preconditioner becomes D^-1 + sum over kept windows of P_w^T B_w^-1 P_w (additive
                         Schwarz, symmetric positive definite).  1000 keeps the windows whose pencil has an
                         eigenvalue below 0.027 and always those below 0.001.  Costs 27^2 words per window of
                         workspace on every level k in [3, q - 1] */
  int exact;          /* 1: the exact (unlocalized) hierarchy of Algorithm 1 -- gamblets over the whole level,
                         dense FP64 level matrices A^(k), B^(k), R^(k-1,k), every subband system solved by a dense
                         Cholesky factorization; the solve is the subband sum of Theorem 4.15 with two FP64
                         refinement steps.  Needs precision GBL_FP64 and 2 <= q <= 7 (the memory grows like 4^2q);
                         gbl_adjoint and the batched calls reject it.  0: the localized hierarchy (default) */
  int geometry;       /* 0: 2^q x 2^q cells, (2^q - 1)^2 interior nodes (the default).  1 (exact only): the mesh of
                         Example 5.1 (Section 5.1), (2^q + 1)^2 cells of side 1 / (2^q + 1), 2^q x 2^q interior nodes,
                         node (i, j) in level-(q-1) cell ((i-1)/2, (j-1)/2): a_dev is [2^q + 1][2^q + 1] */
  int source;         /* 0: g_dev holds one value per cell (b_i = (h^2/4) sum of the four cells); 1 (exact only):
                         g_dev holds the values at the interior nodes, [m][m] with m nodes per side, and b = M g
                         with the Q1 mass matrix (Example 5.1's source) */
  int w_kind;         /* rows of W^(k) over a parent's m children: 0 (default) the normalised Helmert rows of
                         Construction 4.13; 1 (exact only) the differences e_t - e_{t+1} of Construction 4.11.
                         A^(k), R and the solve do not depend on it; B^(k) and the transform coefficients do
                         (the transform then applies (W W^T)^-1 per parent) */
  int dim;            /* space dimension: 2 (default) or 3 (exact only, 2 <= q <= 4: the problem on the unit cube
                         with trilinear elements, 2^q (geometry 0) or 2^q + 1 (geometry 1) cells per side, eight
                         children per parent and seven subband rows).  In 3-D every array gains a third index
                         of the same extent: a_dev [n][n][n], g_dev [nrhs][n][n][n] (nodal: [n-1]^3), u_dev
                         [nrhs][n+1]^3, node (i, j, l) -> ((i-1) m + (j-1)) m + (l-1) on level q, 8^q
                         transform coefficients */
  int autotune;       /* 1: pick each level's build kernels by timing (dense patch solves on the vector units or
                         the matrix cores; band patch solves of the finest level in LDS or in registers; Galerkin
                         product per coarse row or on strips): the first build of a level shape times every
                         applicable candidate (one warm-up and two timed launches each) and keeps the fastest per
                         (device, precision, shape); later builds reuse it.  The build's result is the chosen
                         kernel's, so two devices may pick differently and round differently.  0: the built-in
                         rule (default) */
  const char* autotune_path; /* autotune: file that keeps the choices across processes (read when first used,
                         appended to; one line per choice with both candidates' times), or NULL for this
                         process only.  The string must stay valid for the duration of gbl_build */
  int tensor;         /* 1 (exact only, dim 2): the coefficient is a symmetric matrix per cell (the matrix-valued
                         a(x) of Section 1): a_dev is [n][n][3] = (a11, a12, a22), each positive definite (else
                         EINVAL).  0: a scalar per cell (default) */
} gbl_opts;

typedef struct gbl_solve_info {
  int outer_iters;        /* outer iterations taken (max over right-hand sides) */
  int status;             /* same value as the return code */
  double rel_update;      /* last error estimate (see rtol), relative to ||u|| (max over rhs) */
  double rel_residual;    /* ||b - A u|| / ||b|| at exit (max over rhs) */
} gbl_solve_info;

typedef struct gbl_level_desc {
  /* Device views into the workspace for level k (for inspection and tests).
   * Level k has side nk = 2^k: cells for k < q, node slots for k = q (slot
   * (x, y) is node (x, y); slots with x = 0 or y = 0 hold no unknown).
   * Arrays are offset-major (the grid position is the fastest index) so that
   * neighbouring threads read neighbouring words.  elem_bytes is 8 (FP64) or
   * 4 (MIXED). */
  int k;
  int nk;
  int s;              /* A^(k) stencil half-width; A[ox][oy][x][y] = A_{(x,y),(x+ox-s,y+oy-s)} */
  int t;              /* B^(k) parent-stencil half-width (k >= 2).  Entry (ox, oy, i, j) of parent
                         p = px*(nk/2)+py couples subband row (p, i) to (parent (px+ox-t, py+oy-t), j);
                         stored block-interleaved: B[p/64][ox][oy][i][j][p%64] (groups of 64 parents) */
  int rw;             /* R^(k-1,k) block width (k >= 2); R[bx][by][cx][cy] = R_{(cx,cy),(2(cx-rho)+bx, 2(cy-rho)+by)} */
  int rho;            /* effective patch radius at this level */
  int elem_bytes;
  const void* A;      /* A^(k) */
  const void* B;      /* B^(k), NULL for k = 1 */
  const void* R;      /* R^(k-1,k), NULL for k = 1 */
  int nwin;           /* kept windows of the preconditioner (window_tol > 0, 3 <= k < q), else 0 */
  const int* wlist;   /* [nwin] window origins x0 * (nk/2) + y0 (parents x0..x0+2, y0..y0+2), any order */
  const void* winv;   /* [nwin][27][27] B_w^-1, unknown (3 dx + dy) * 3 + t of parent (x0 + dx, y0 + dy) */
  int dense;          /* 1 for the exact hierarchy: A is [n][n], B [nsub][nsub] (subband row t * (n_{k-1}) + parent,
                         identity rows where a parent has fewer children), R [n_{k-1}][n], row-major FP64; level-q
                         unknowns are the interior nodes (i - 1) m + (j - 1), level-k < q unknowns the cells
                         x 2^k + y.  0 for the localized hierarchy (the stencil layouts above) */
  int n;              /* unknowns of level k (dense only) */
  int nsub;           /* subband rows of level k, 2^dim - 1 per parent (dense only) */
  int patch_kernel;   /* autotune: the variant that built level k's patch solves (dense: 0 vector units, 1 matrix
                         cores; finest-level band: 0 LDS, 1 registers), else -1 (the built-in rule) */
  int galerkin_kernel;/* autotune: the variant of A^(k-1) = R A^(k) R^T (0 per coarse row, 1 strips), else -1 */
} gbl_level_desc;

typedef struct gbl_ctx gbl_ctx;

/* Library version (GBL_VERSION). */
int gbl_version(void);

/* Fill *opts with defaults: rho 3, MIXED, rtol 1e-8, max_outer 100,
 * Chebyshev inner iterations, inner_iters 16, inner_iters_coarse 2,
 * kappa 200, kappa_coarse 10, max_rhs 1, window_tol 0, exact 0, geometry 0,
 * source 0, w_kind 0, dim 2, autotune 0, autotune_path NULL, tensor 0. */
int gbl_default_opts(gbl_opts* opts);

/* Device workspace needed for a hierarchy of depth q (2 <= q <= 12) with
 * these options, including min(opts->max_rhs, 64) copies of the solve buffers.
 * Pure host computation.  EINVAL on a bad q or options. */
int gbl_workspace_bytes(int q, const gbl_opts* opts, size_t* bytes);

/* Build the localized hierarchy for the cell coefficient a_dev [n][n] (n = 2^q;
 * n = 2^q + 1 for the exact hierarchy with geometry 1), or with opts->exact
 * the exact hierarchy of Algorithm 1 (dense FP64 level matrices, Cholesky
 * factors of every B^(k) and of A^(1)).
 * The hierarchy is stored in ws_dev (ws_bytes >= gbl_workspace_bytes); the
 * caller must keep ws_dev alive and untouched until gbl_destroy.  On success
 * *out receives a new context.  EINVAL if any a <= 0 or non-finite (checked on
 * the device), ENOTSPD on a non-positive pivot, ENOMEM if ws_bytes is short.
 * Synchronises the stream once at the end to read the status word. */
int gbl_build(gbl_ctx** out, int q, const double* a_dev, const gbl_opts* opts,
              void* ws_dev, size_t ws_bytes, void* stream);

/* Solve for nrhs >= 1 right-hand sides (in blocks of min(opts->max_rhs, 64); a block
 * iterates until all its right-hand sides meet rtol).
 * g_dev : [nrhs][n][n] cell source ([nrhs][n-1][n-1] interior nodal values when
 *         opts->source = 1).
 * u_dev : [nrhs][n+1][n+1] nodal; on entry its boundary entries hold the
 *         Dirichlet data (interior entries are ignored), on exit the interior
 *         holds the solution.
 * info  : optional (may be NULL).
 * ENOCONV if rtol was not reached within max_outer iterations (u holds the
 * last iterate).  The exact hierarchy applies the subband solve of Theorem
 * 4.15 (every subband system solved by its Cholesky factor) and two FP64
 * refinement steps with A^(q); its info reports no iterations.
 * Synchronises the stream. */
int gbl_solve(gbl_ctx* ctx, int nrhs, const double* g_dev, double* u_dev,
              gbl_solve_info* info, void* stream);

/* Adjoint gradient of a scalar J(u) (not in the paper; differentiates the
 * discrete problem of Section 5.1).  With u the solution returned by gbl_solve
 * for coefficient a and source g, and dJdu_dev [nrhs][n+1][n+1] the gradient
 * of J with respect to the nodal values (boundary entries ignored), solves
 * the symmetric adjoint system A lambda = dJ/du with the same hierarchy and
 * writes
 *   dJdloga_dev [nrhs][n][n] : -a_e lambda_e^T K_e u_e per cell
 *   dJdg_dev    [nrhs][n][n] : (h^2/4) sum of lambda over the cell's corners (may be NULL)
 *   lambda_dev  [nrhs][n+1][n+1] : the adjoint state, zero on the boundary (may be NULL)
 * where K_e is the unit bilinear element stiffness.  u_dev is read only.
 * Same status codes as gbl_solve. */
int gbl_adjoint(gbl_ctx* ctx, int nrhs, const double* u_dev, const double* dJdu_dev,
                double* dJdloga_dev, double* dJdg_dev, double* lambda_dev,
                gbl_solve_info* info, void* stream);

/* Batched build of independent problems of uneven depth (the workload of
 * many small problems, each too small to fill the GPU alone).  Problem i has
 * depth q[i] (2..12), coefficient a_dev[i] ([2^q_i][2^q_i]) and its own
 * workspace ws_dev[i] of ws_bytes[i] >= gbl_workspace_bytes(q[i], opts)
 * bytes; all problems share opts.  The problems are built concurrently by a
 * pool of host threads (GBL_BATCH_WORKERS, default 8), each with its own HIP
 * stream, largest first; the work starts after what is already enqueued on
 * `stream`, and `stream` waits for all of it.  Returns when every build has
 * finished.  ctx_out[i] receives the context of problem i (NULL if its build
 * failed; release each with gbl_destroy) and status[i] its gbl_build status.
 * Return value: GBL_OK if every problem built, else the first failing status
 * in problem order (gbl_last_error(NULL) names the problem).  EINVAL on a
 * null array or nprob < 1. */
int gbl_build_batched(int nprob, const int* q, const double* const* a_dev, const gbl_opts* opts,
                      void* const* ws_dev, const size_t* ws_bytes, gbl_ctx** ctx_out, int* status,
                      void* stream);

/* Batched solve: problem i solves nrhs[i] right-hand sides (blocks as in gbl_solve),
 * g_dev[i] [nrhs_i][n_i][n_i] into u_dev[i] [nrhs_i][n_i+1][n_i+1] (boundary
 * values in, solution out) with context ctx[i], concurrently as in
 * gbl_build_batched.  info (optional) is an array of nprob records; status[i]
 * is problem i's gbl_solve status.  Return value as for gbl_build_batched.
 * Two entries of ctx must not be the same context. */
int gbl_solve_batched(int nprob, gbl_ctx* const* ctx, const int* nrhs, const double* const* g_dev,
                      double* const* u_dev, gbl_solve_info* info, int* status, void* stream);

/* Build flags (bit set).  GBL_FLAG_PIVOTS_REGULARIZED: in MIXED precision,
 * one or more pivots of a patch factorisation (scaled to a unit diagonal) or
 * of the coarse A^(1) factor fell below 1e-6 in FP32 -- a patch straddling a
 * coefficient jump beyond single-precision resolution -- and were raised to
 * that floor.  The hierarchy is still symmetric positive definite (any patch
 * solution D gives a full-rank R = pibar + D W, Section 4.7), so solves stay
 * correct, but may need more outer iterations; GBL_FP64 avoids it.  In FP64
 * a non-positive pivot is the ENOTSPD error instead. */
#define GBL_FLAG_PIVOTS_REGULARIZED 1u
int gbl_build_flags(const gbl_ctx* ctx, unsigned* flags);

/* Describe level k (1 <= k <= q) of a built hierarchy.  EINVAL on a bad k. */
int gbl_level_layout(const gbl_ctx* ctx, int k, gbl_level_desc* desc);

/* ---- Gamblet transform and compression ------------------------------------
 * The representation of a level-q vector u in the basis of normalized
 * gamblets psi^(1)_i / ||psi^(1)_i||_a and chi^(k)_j / ||chi^(k)_j||_a,
 * k = 2..q, of the built (localized) hierarchy (discussion of Example 5.1 and
 * Figures 10-11; chi^(k) = W^(k) psi^(k), psi^(k-1) = R^(k-1,k) psi^(k)).
 * Level-(k-1) measurements are child sums of level-k ones (R pi^T = I for
 * R = pibar + D W, Section 4.7), so U^(k-1) = pi U^(k) and
 * w^(k) = W^(k) (U^(k) - R^T U^(k-1)); the coefficients are U^(1)_i
 * sqrt(A^(1)_ii) and w^(k)_j sqrt(B^(k)_jj).  The inverse is the
 * reconstruction of Theorem 4.15.  All arithmetic is FP64 (the operators are
 * read in the hierarchy's precision).
 *
 * Coefficient layout (device, FP64, 4^q values, owned by the caller): level 1
 * at offset 0 (4 values, slot x * 2 + y); level k >= 2 at offset 4^(k-1)
 * (3 * 4^(k-1) values, entry t * 4^(k-1) + parent, parent = px * 2^(k-1) + py,
 * t = 0..2 the subband index of the parent; entries of padding rows -- parents
 * on the low edges of level q with fewer than four children -- are zero).
 * u is nodal, [(2^q + 1)^2] FP64 on the device; boundary entries are ignored on
 * input and written as zero on output.  Calls on one context must not overlap
 * (they use its workspace). */

/* Number of coefficients, 4^q.  EINVAL on NULL arguments. */
int gbl_transform_size(const gbl_ctx* ctx, size_t* count);

/* coef = normalized gamblet coefficients of u.  Asynchronous on stream.
 * EINVAL on NULL arguments or a hierarchy built with level_q_mass > 0 (its
 * level-q measurements are not nodal values), EHIP on a launch failure. */
int gbl_transform(gbl_ctx* ctx, const double* u_dev, double* coef_dev, void* stream);

/* u = sum of the coefficients times the normalized gamblets (the inverse of
 * gbl_transform up to rounding).  Asynchronous on stream.  Errors as above. */
int gbl_inverse_transform(gbl_ctx* ctx, const double* coef_dev, double* u_dev, void* stream);

/* Compression by thresholding (Figure 11): keep the keep largest |coef| over
 * all levels and set the others to zero, in place; coefficients equal to the
 * smallest kept magnitude are kept too, NaN entries are zeroed.  keep <= 0
 * zeroes all, keep >= 4^q changes nothing.  threshold (host, may be NULL)
 * receives the smallest kept magnitude (+inf for keep <= 0, 0 for keep >= 4^q);
 * when it is given the call waits for the stream.  EINVAL on NULL ctx / coef. */
int gbl_compress(gbl_ctx* ctx, double* coef_dev, long keep, double* threshold, void* stream);

/* Allocation-free compression, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops).  The same
 * selection as gbl_compress on any FP64 device vector of `count` entries, no
 * hierarchy needed: keep the `keep` largest |coef| in place, zero the others
 * (ties at the smallest kept magnitude kept, NaN zeroed; keep <= 0 zeroes all,
 * keep >= count changes nothing); threshold (host, may be NULL) as for
 * gbl_compress, and when given the call waits for the stream.  Its selection
 * state (about 8.4 KB) lives in a fixed array of the library's device memory,
 * one per GPU, held until the process ends; the call allocates nothing.
 * Calls that overlap on one GPU (concurrent streams or host threads) share
 * that array and race; serialise them.  Limit: count <= 4294967295 (the
 * histogram counters are 32-bit), else GBL_EINVAL; GBL_EINVAL on a NULL coef,
 * GBL_EHIP on a launch or copy failure (message via gbl_last_error(NULL)). */
int gbl_compress_noalloc(double* coef_dev, long count, long keep, double* threshold, void* stream);

/* Energy norm sqrt(u^T A u) of a nodal u (boundary entries ignored) with the
 * FP64 fine stiffness matrix of the hierarchy's coefficient.  Waits for the
 * stream; *norm is a host double.  EINVAL on NULL arguments. */
int gbl_energy_norm(gbl_ctx* ctx, const double* u_dev, double* norm, void* stream);

/* ------------------------------------------------------------------------
 * Level-q gamblets from the localized inverse of the mass matrix (Algorithm
 * 2: the mass matrix, the localized mass inverse, the level-q gamblets, their
 * load and their stiffness matrix; Definition 5.2).  For every interior node
 * i the patch is the box of interior nodes within rho_q node steps of i;
 * y^(i) solves M^(i,rho_q) y = e_i on it (M_ij = int phi_i phi_j, Q1 on the
 * 2^q x 2^q cell grid of the unit square), psi^(q)_i = sum_j y^(i)_j phi_j,
 * g^(q)_i = int psi^(q)_i g = sum_j y^(i)_j b_j and A^(q) = Minv^T A Minv.
 * On this grid y^(i) is the outer product of two one-dimensional factors.
 *
 * Common to all calls: q in [2, 12], rho_q in [1, 4], n = 2^q, m = n - 1;
 * interior vectors are FP64 [m][m], node (ix, iy) at ix * m + iy, node
 * coordinates 1 + ix, 1 + iy on the (n+1) x (n+1) grid.  All pointers are
 * device memory owned by the caller; no call allocates.  Every call is
 * asynchronous on stream and returns GBL_EINVAL for a bad q, rho_q or a NULL
 * pointer (message via gbl_last_error(NULL)), GBL_EHIP if a launch fails.
 * ------------------------------------------------------------------------ */

/* The table of one-dimensional factors (Definition 5.2):
 * table[x][d + rho_q], x in [0, m), d in [-rho_q, rho_q], is the entry at
 * x + d of the inverse of the 1-D mass matrix h tridiag(1, 4, 1)/6 on the
 * interval of interior coordinates within rho_q of x, applied to e_x (zero
 * outside the interval).  Output table_dev: [m][2 rho_q + 1]. */
int gbl_mass_inverse(int q, int rho_q, double* table_dev, void* stream);

/* psi^(q)_i in the nodal basis: psi_dev[i][(dx + rho_q)(2 rho_q + 1) + dy +
 * rho_q] = table[ix][dx + rho_q] * table[iy][dy + rho_q], the weight of
 * phi at node i + (dx, dy).  Output: [m^2][(2 rho_q + 1)^2]. */
int gbl_level_q_gamblets(int q, int rho_q, const double* table_dev, double* psi_dev, void* stream);

/* g^(q) = Minv^T b for a nodal load b_j = int phi_j g (interior vectors).
 * b and gq must not overlap (GBL_EINVAL if they are the same pointer). */
int gbl_level_q_load(int q, int rho_q, const double* table_dev, const double* b_dev, double* gq_dev, void* stream);

/* A^(q)_ij = int grad psi_i . a grad psi_j for the cell coefficient a_dev
 * ([n][n] FP64, a[ex][ey] on cell ex*n + ey, positive; not checked here).
 * Output aq_dev: [m^2][(2S + 1)^2], S = 2 rho_q + 1, entry (dx + S)(2S + 1)
 * + dy + S of row i couples node i with i + (dx, dy); zero where that node
 * is not interior.  The operator is symmetric positive definite. */
int gbl_level_q_operator(int q, int rho_q, const double* a_dev, const double* table_dev, double* aq_dev,
                         void* stream);

/* Nodal values u = Minv U of the level-q combination sum_i U_i psi^(q)_i.
 * U and u must not overlap. */
int gbl_level_q_to_nodal(int q, int rho_q, const double* table_dev, const double* U_dev, double* u_dev,
                         void* stream);

/* Kernel classes for the optional timing of gbl_profile_*. */
enum gbl_prof_kernel {
  GBL_PROF_ASSEMBLE = 0,          /* fine stiffness A^(q) */
  GBL_PROF_SUBBAND_OPERATOR = 1,  /* B^(k) = W A^(k) W^T and block-Jacobi factors */
  GBL_PROF_PATCH_SOLVE = 2,       /* patch Cholesky solves and R^(k-1,k), levels k < q */
  GBL_PROF_GALERKIN = 3,          /* A^(k-1) = R A^(k) R^T */
  GBL_PROF_RESTRICT = 4,          /* g^(k-1) = R g^(k) */
  GBL_PROF_CG_INIT = 5,           /* subband CG start, coarser levels */
  GBL_PROF_CG_SPMV = 6,           /* subband CG operator application, coarser levels */
  GBL_PROF_CG_UPDATE = 7,         /* subband CG vector update, coarser levels */
  GBL_PROF_PROLONG = 8,           /* v^(k) = R^T v^(k-1) + W^T w^(k) */
  GBL_PROF_FINE_APPLY = 9,        /* FP64 fine operator in the outer iteration */
  GBL_PROF_GRADIENT = 10,         /* adjoint cell gradient */
  GBL_PROF_FINE_CG = 11,          /* finest-level subband iteration (CG or Chebyshev, fused) */
  GBL_PROF_PATCH_BAND = 12,       /* band patch solves and R^(q-1,q) at the finest transition */
  GBL_PROF_NUM_KERNELS = 13
};

/* Process-wide kernel timing: every launch of a class whose bit (1 << class)
 * is set in mask is bracketed by HIP events recorded on its stream (mask 0
 * switches timing off; it is off by default).  gbl_profile_read waits for
 * the recorded events and returns the summed elapsed time (ms) and the number
 * of timed launches since the last reset.  Not for concurrent use from
 * several host threads. */
int gbl_profile_enable(unsigned mask);
int gbl_profile_reset(void);
int gbl_profile_read(int kernel, double* total_ms, long* launches);

/* Release the host context (the workspace stays owned by the caller). */
int gbl_destroy(gbl_ctx* ctx);

/* Message of the last error on ctx, or of the last context-less failure when
 * ctx is NULL.  Never NULL. */
const char* gbl_last_error(const gbl_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* GAMBLET_H */
