/*
 * phmg.h -- C ABI of the MI355X (gfx950) Vanka-star / phMG / FGMRES library.
 *
 * The library solves the discrete Stokes saddle-point system K x = b
 * (Section 2, eq. "eq:saddle": K = [A B^T; B 0]) with restarted flexible
 * GMRES (Section 4, solver paragraph: FGMRES(30)) right-preconditioned by a
 * monolithic multigrid cycle: hMG (Section 3.1, eq. "eq:TG-operator") or
 * phMG defect correction (Section 3.2, eq. "eq:DC-TG-operator"), whose
 * smoother is additive Schwarz over Vanka-star patches (Section 3.4,
 * eq. "eq:ASM", figure "fig:patches"), each patch system solved exactly.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Level 0 is the finest level; level nlevels-1 is the coarsest and is
 *    solved by a dense direct solve.
 *  - Descriptor arrays (phmg_csr, phmg_patches, coarse_null) are HOST
 *    pointers.  phmg_hierarchy_create validates them on the host, copies them
 *    to device memory owned by the library and never reads them again.
 *  - Vector arguments b and x of relax_apply / vcycle / fgmres_solve are
 *    DEVICE pointers to float64 arrays of the level's length, owned by the
 *    caller.  b is read only; x is read and written.  b and x must not alias.
 *  - All work is enqueued on the stream given at creation (a hipStream_t
 *    passed as void*; NULL = the default stream).  relax_setup and
 *    fgmres_solve synchronise that stream before returning; relax_apply and
 *    vcycle are asynchronous.
 *  - Every call returns a phmg_status.  No exception crosses the ABI.  On an
 *    error, phmg_last_error() returns a thread-local message naming the level
 *    and, where relevant, the patch.
 *  - Calls on one context are not thread safe; use one context per thread.
 */
#ifndef PHMG_H
#define PHMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct phmg_ctx_s* phmg_ctx;

typedef enum {
    PHMG_OK = 0,
    PHMG_EINVAL = -1,     /* malformed or inconsistent input; nothing was launched      */
    PHMG_ENOMEM = -2,     /* device allocation failed                                    */
    PHMG_ESINGULAR = -3,  /* a patch (or the coarse matrix) has a pivot <= 1e-14 ||.||_inf */
    PHMG_ENOCONV = -4,    /* fgmres_solve hit maxit; x holds the last iterate            */
    PHMG_EHIP = -5,       /* a HIP runtime call failed                                   */
    PHMG_ESTATE = -6      /* call order violated (e.g. apply before setup)               */
} phmg_status;

/* Compressed sparse row matrix.  rowptr[0] = 0, rowptr[nrows] = nnz, column
 * indices strictly ascending inside each row, all values finite.  Sizes
 * must satisfy nnz < 2^31. */
typedef struct {
    int32_t nrows, ncols;
    int64_t nnz;
    const int32_t* rowptr;   /* nrows + 1 */
    const int32_t* col;      /* nnz       */
    const double* val;       /* nnz       */
} phmg_csr;

/* Vanka-star patches of one level (Section 3.4): patch i owns the DoFs
 * dofs[ptr[i] .. ptr[i+1]), strictly ascending, 1 <= m_i <= PHMG_MAX_PATCH.
 * weight (optional, same length as dofs) holds the diagonal of the
 * partition-of-unity operator W_i of eq. "eq:ASM"; NULL means W_i = I. */
typedef struct {
    int32_t npatch;
    const int64_t* ptr;      /* npatch + 1 */
    const int32_t* dofs;     /* ptr[npatch] */
    const double* weight;    /* ptr[npatch] or NULL */
} phmg_patches;

#define PHMG_MAX_PATCH 1024
/* The coarsest level is solved with a dense inverse of its (bordered) matrix. */
#define PHMG_MAX_COARSE 8192

/* Cycle parameters (Section 3.1-3.2; V^{(n_V, nu_p, nu_h)} of Section 4):
 * levels 0 .. n_plevels-1 are p-levels relaxed with nu_p sweeps and coarsened
 * by defect correction; the hMG part starting at level n_plevels is applied
 * n_v times (stationary iterations from zero); h-levels use nu_h sweeps.
 * Pre- and post-smoothing use the same count.
 * smoother = PHMG_SMOOTHER_RICHARDSON: each sweep is x += omega M^{-1}(b - K x).
 * smoother = PHMG_SMOOTHER_CHEBYSHEV (the paper's experiments, Section 4):
 * nu steps of Chebyshev acceleration of M^{-1} over [cheb_lo, cheb_hi] *
 * lambda, where lambda estimates the largest eigenvalue of M^{-1} K by
 * the largest real Ritz value of eig_iters Arnoldi steps (classical
 * Gram-Schmidt twice) run at set-up from v_j = 1 + sin(j)/2. */
typedef struct {
    int32_t nu_p, nu_h, n_v, n_plevels;
    double omega;
    int32_t smoother, eig_iters;
    double cheb_lo, cheb_hi;
} phmg_cycle_opts;

#define PHMG_SMOOTHER_RICHARDSON 0
#define PHMG_SMOOTHER_CHEBYSHEV 1

/* Patch-factor storage precision of a level (the apply accumulates in the
 * precision of the factors, the residual and the scatter stay float64). */
typedef enum { PHMG_PREC_F64 = 0, PHMG_PREC_F32 = 1, PHMG_PREC_BF16 = 2 } phmg_precision;

typedef struct {
    int32_t nlevels;                 /* >= 2 */
    const phmg_csr* K;               /* nlevels matrices, square, free DoFs only          */
    const phmg_csr* P;               /* nlevels-1 prolongations: P[l] is n_l x n_{l+1}    */
    const phmg_patches* patches;     /* nlevels-1 (none on the coarsest level)            */
    const double* coarse_null;       /* kernel vector z of K_{nlevels-1}, or NULL when
                                        the coarsest matrix is nonsingular                 */
} phmg_hierarchy_desc;

/* Validate and upload a hierarchy: the level matrices K_l (Section 2, the
 * saddle-point system of eq. "eq:saddle" on each level of Section 3.1-3.2), the
 * Vanka-star patches (Section 3.4, figure "fig:patches") and the prolongations
 * P_l (Section 3.1: interpolation between nested spaces; Section 3.2: between
 * orders on one mesh).  R_l = P_l^T is formed explicitly on the host and
 * uploaded; the DoF -> patch-slot map used by the deterministic scatter is built
 * here.  Errors: PHMG_EINVAL for any malformed array (message names the level,
 * patch or row), nothing uploaded; PHMG_ENOMEM.  On success *out owns all device
 * memory it uses; the descriptor's host arrays may be freed on return. */
phmg_status phmg_hierarchy_create(const phmg_hierarchy_desc* desc, const phmg_cycle_opts* opts,
                                  void* stream, phmg_ctx* out);

/* Set-up of the relaxation on one level (level < 0: every level), Section 3.4:
 * patch extraction K_i = I_i K I_i^T (the patch submatrix of eq. "eq:ASM") and
 * factorisation of every patch, and on the coarsest level the factorisation of
 * the (bordered) coarse matrix (Section 4: direct solve on the coarsest grid).
 * Patch systems are inverted by Gauss-Jordan elimination with partial pivoting
 * (the same pivots as LU with partial pivoting, the paper's exact patch solves)
 * and the explicit inverse is stored in the level's precision; with the
 * Chebyshev smoother the eigenvalue estimate of M^{-1} K is formed here too.
 * Returns PHMG_ESINGULAR naming the first singular patch (|pivot| <= 1e-14
 * ||K_i||_inf) or the coarse matrix.  Synchronises the stream. */
phmg_status phmg_relax_setup(phmg_ctx ctx, int level);

/* Choose the storage precision of the patch inverses of one level (before
 * relax_setup of that level, or followed by a new relax_setup). */
phmg_status phmg_set_precision(phmg_ctx ctx, int level, phmg_precision prec);

/* Layout of the stored patch inverses of one level (before relax_setup of
 * that level, or followed by a new relax_setup).
 * PHMG_STORAGE_AUTO (the default): when K_l is symmetric to rounding
 * (structurally symmetric and |K_ij - K_ji| <= 1e-12 max(max_k |K_ik|,
 * max_k |K_jk|) for every entry), each patch inverse is stored as its
 * symmetric part S_i = (K_i^{-1} + K_i^{-T}) / 2, lower triangle only (row
 * strips of 16: the strictly lower part and the diagonal 16 x 16 block), which
 * roughly halves the bytes a sweep streams; S_i^T = S_i also serves the
 * adjoint sweep.  Otherwise the general layout is used.
 * PHMG_STORAGE_GENERAL: always B_i = (P_i K_i)^{-1} in full (P_i the pivoting
 * permutation), with K_i^{-T} = P_i^T B_i^T for the adjoint sweep. */
typedef enum { PHMG_STORAGE_AUTO = 0, PHMG_STORAGE_GENERAL = 1 } phmg_storage;
phmg_status phmg_set_patch_storage(phmg_ctx ctx, int level, phmg_storage storage);

/* nu sweeps of x <- x + omega * sum_i R_i^T W_i K_i^{-1} R_i (b - K_l x) on
 * level `level` (eq. "eq:ASM").  level must not be the coarsest. */
phmg_status phmg_relax_apply(phmg_ctx ctx, int level, const double* b, double* x, int nu);

/* x <- B b: one preconditioner application on level 0 -- the hMG V-cycle of
 * Section 3.1 (eq. "eq:TG-operator" applied recursively) or, with n_plevels > 0,
 * the phMG defect-correction cycle of Section 3.2 (eq. "eq:DC-TG-operator"),
 * started from x = 0.  The content of x on entry is ignored.  PHMG_ESTATE
 * before relax_setup of every level.  Asynchronous. */
phmg_status phmg_vcycle(phmg_ctx ctx, const double* b, double* x);

/* Replay the preconditioner as a HIP graph (default on): the first
 * phmg_vcycle / FGMRES iteration after a set-up captures one V-cycle on a
 * private stream into a graph with fixed input and output buffers; later
 * applications copy in, launch the graph on the context stream and copy out.
 * Results are bitwise identical to the eager launches.  Graphs are bypassed
 * while per-kernel profiling is enabled. */
phmg_status phmg_set_graphs(phmg_ctx ctx, int on);

/* Restarted flexible GMRES (Section 4, solver paragraph: FGMRES with restart
 * `restart`, the paper's 30) on level 0, right-preconditioned by phmg_vcycle,
 * from the initial guess in x.  A cycle ends when the Givens residual estimate
 * drops to rtol * ||b - K x_0||_2, on an exact breakdown, or after maxit inner
 * iterations; the solve has converged when the true residual satisfies the same
 * bound, else it restarts (PHMG_ENOCONV after maxit, with x = the last iterate).
 * On return *iters is the number of inner iterations and *relres the true
 * residual ||b - K x||_2 / ||b - K x_0||_2.  PHMG_EINVAL, with x unchanged, when
 * b or x holds a NaN or Inf (found by the device norm of b - K x_0 before any
 * iteration).  Synchronises the stream. */
phmg_status phmg_fgmres_solve(phmg_ctx ctx, const double* b, double* x, double rtol, int restart, int maxit,
                              int* iters, double* relres);

/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the sweeps of phmg_relax_apply, bit for bit, with the three work buffers of a
 * sweep -- residual (n doubles), Chebyshev direction (n) and staged patch
 * results (sum of the level's patch sizes) -- taken from one device array of
 * PHMG_NOALLOC_MAX_DOUBLES doubles (32 MiB) that the library reserves at load
 * time on every GPU it runs on, instead of from the context.  The call makes no
 * device allocation and no timing event (per-kernel profiling does not see it).
 * b and x are the caller's DEVICE pointers as in phmg_relax_apply; the call is
 * asynchronous on the context stream.  Errors: PHMG_EINVAL when the level needs
 * 2 n + sum m (each rounded up to 32 doubles) > PHMG_NOALLOC_MAX_DOUBLES, before
 * any launch; PHMG_ESTATE before relax_setup of the level.  Every call on one
 * GPU shares that GPU's array (no buffer needs to start at zero): calls that
 * overlap in time on one GPU -- two streams, two threads, two contexts -- race
 * and must be serialised by the caller. */
#define PHMG_NOALLOC_MAX_DOUBLES (4 << 20)
phmg_status phmg_relax_apply_noalloc(phmg_ctx ctx, int level, const double* b, double* x, int nu);

/* Adjoint (transposed) operators, for gradients through a solve.  They reuse
 * the factors of relax_setup: with the stored B_i = (P_i K_i)^{-1},
 * K_i^{-T} = P_i^T B_i^T, so the transposed sweep gathers W_i r[S_i] in DoF
 * order, streams B_i^T and scatters through the pivot permutation (gather and
 * scatter swap roles).  K^T is K itself when K is exactly symmetric (checked at
 * create), else an explicit transposed copy made there.
 *   relax_apply_transposed: nu sweeps x <- x + omega M^T (b - K_l^T x) with
 *     M^T = sum_i R_i^T K_i^{-T} W_i R_i (Chebyshev: the forward interval);
 *   vcycle_transposed:  x <- B^T b, B the preconditioner of phmg_vcycle (the
 *     same cycle with K^T, the adjoint sweeps and the transposed coarse solve;
 *     pre- and post-smoothing use equal counts, so this is exactly B^T);
 *   fgmres_solve_transposed: FGMRES on K^T x = b right-preconditioned by B^T,
 *     with the stopping rule and outputs of phmg_fgmres_solve.
 * Same argument conventions, synchronisation and errors as the forward calls. */
phmg_status phmg_relax_apply_transposed(phmg_ctx ctx, int level, const double* b, double* x, int nu);
phmg_status phmg_vcycle_transposed(phmg_ctx ctx, const double* b, double* x);
phmg_status phmg_fgmres_solve_transposed(phmg_ctx ctx, const double* b, double* x, double rtol, int restart,
                                         int maxit, int* iters, double* relres);

/* Gradients through the solve (adjoint method).  For J(x_1..x_B) with
 * K(theta) x_c = G f_c, the gradients are dJ/dtheta = -sum_c lam_c^T (dK/dtheta) x_c
 * and dJ/df_c = G^T lam_c, where K^T lam_c = dJ/dx_c (phmg_fgmres_solve_transposed).
 *   S (HOST csr, n_theta x nnz(K_0)): S[v, e] = d K_e / d theta_v, e indexing the
 *     nonzeros of K_0 in its CSR order;
 *   G (HOST csr, n_0 x n_f): the map from forcing parameters to the right-hand side.
 * set_sensitivities copies both (and forms G^T) into device memory; it may be
 * called again after K changes.  forcing_rhs: B_c = G F_c.  gradients:
 * grad_theta (n_theta) = -S w with w_e = sum_c Lam_c[i_e] X_c[j_e], and, when
 * grad_f is not NULL, grad_f_c = G^T Lam_c.  X, Lam (nrhs x n_0), F and grad_f
 * (nrhs x n_f) and grad_theta are DEVICE float64 arrays, systems one after
 * another.  Asynchronous; PHMG_ESTATE before set_sensitivities. */
phmg_status phmg_set_sensitivities(phmg_ctx ctx, const phmg_csr* S, const phmg_csr* G);
phmg_status phmg_forcing_rhs(phmg_ctx ctx, int nrhs, const double* F, double* B);
phmg_status phmg_gradients(phmg_ctx ctx, int nrhs, const double* X, const double* Lam, double* grad_theta,
                           double* grad_f);

/* Full-block-factorisation preconditioner (Section 3.3, eq. "eq:fbf"):
 *   P^{-1} = [I  -A~^{-1} B^T; 0  I] [A~^{-1}  0; 0  S~^{-1}] [I  0; -B A~^{-1}  I]
 * applied to r = [r_u; r_p] as y_u = A~^{-1} r_u, z_p = S~^{-1}(r_p - B y_u),
 * z_u = y_u - A~^{-1} B^T z_p.  A~^{-1} is one cycle (phmg_vcycle) of
 * `velocity`, a hierarchy created on the velocity block A of K (its own
 * levels, patches -- the paper uses vertex-star velocity patches -- and
 * transfers; set up before use); S~^{-1} is any n_p x n_p matrix, in the paper
 * the inverse block-diagonal pressure mass matrix (Scott-Vogelius), with the
 * sign of the Schur complement -B A^{-1} B^T.  K (n x n, velocity DoFs first),
 * B (n_p x n_u) and S_inv are HOST csr arrays copied at create.
 * fbf_fgmres_solve: FGMRES on K right-preconditioned by P^{-1}, with the
 * stopping rule and outputs of phmg_fgmres_solve.  Work runs on the velocity
 * context's stream; destroy the FBF object before its velocity context. */
typedef struct phmg_fbf_s* phmg_fbf;
phmg_status phmg_fbf_create(phmg_ctx velocity, const phmg_csr* K, const phmg_csr* B, const phmg_csr* S_inv,
                            phmg_fbf* out);
phmg_status phmg_fbf_apply(phmg_fbf fbf, const double* r, double* z);
phmg_status phmg_fbf_fgmres_solve(phmg_fbf fbf, const double* b, double* x, double rtol, int restart, int maxit,
                                  int* iters, double* relres);
phmg_status phmg_fbf_destroy(phmg_fbf fbf);

/* Several right-hand sides at once (1 <= nrhs <= PHMG_MAX_RHS).  B and X are
 * DEVICE float64 arrays of nrhs * n_l entries holding the systems one after
 * another (X[c * n_l + i] is DoF i of system c, i.e. a (nrhs, n) row-major
 * tensor); B is read only, X is read and written, they must not alias.
 * Column c of every result is what the single-system call computes for
 * (b_c, x_c), up to rounding: the sweeps are shared so that each patch
 * inverse and each matrix entry is read once per sweep for all systems, and
 * the patch solves run as dense products on MFMA (float64 16x16x4 for F64
 * factors; float32 16x16x4 with float32 accumulation for F32 and BF16
 * factors).  The first batched call after a set-up autotunes the block
 * kernel shapes (synchronising the stream); relax_apply_batched and
 * vcycle_batched are otherwise asynchronous. */
#define PHMG_MAX_RHS 16
phmg_status phmg_relax_apply_batched(phmg_ctx ctx, int level, int nrhs, const double* B, double* X, int nu);
phmg_status phmg_vcycle_batched(phmg_ctx ctx, int nrhs, const double* B, double* X);
/* FGMRES for every system, in lockstep: each column keeps its own
 * Hessenberg matrix, Givens rotations and stopping test (the single-system
 * rule of phmg_fgmres_solve, so iters[c] equals what phmg_fgmres_solve
 * reports for system c); a column that has stopped idles while the others
 * finish their cycle.  iters and relres are HOST arrays of nrhs entries.
 * restart <= 31.  Returns PHMG_ENOCONV if any system hit maxit.
 * Synchronises the stream. */
phmg_status phmg_fgmres_solve_batched(phmg_ctx ctx, int nrhs, const double* B, double* X, double rtol, int restart,
                                      int maxit, int32_t* iters, double* relres);

/* The adjoint counterparts for up to PHMG_MAX_RHS systems K^T x_c = b_c (the
 * per-system rules of phmg_vcycle_transposed / phmg_fgmres_solve_transposed).
 * They need every relaxed level symmetric to rounding and set up in the
 * default (symmetric) layout, where the adjoint patch solve K_i^{-T} W_i is
 * applied as K_i^{-1} W_i with the block kernels; otherwise PHMG_EINVAL (use
 * the single-system adjoint).  Same layout and limits as the forward calls. */
phmg_status phmg_vcycle_batched_transposed(phmg_ctx ctx, int nrhs, const double* B, double* X);
phmg_status phmg_fgmres_solve_batched_transposed(phmg_ctx ctx, int nrhs, const double* B, double* X, double rtol,
                                                 int restart, int maxit, int32_t* iters, double* relres);

/* Residual r = b - K_l x on a level (device pointers, asynchronous). */

/* The pressure kernel (Section 2: with Dirichlet data on the whole boundary the
 * pressure is determined up to a constant, p in L^2_0; K z = 0 for the constant
 * pressure z = [0; 1_p]).  set_kernel_vector copies z (HOST, n_0 values, finite,
 * not all zero; NULL removes it).  project_kernel maps every system x_c of X
 * (DEVICE, nrhs x n_0 float64, systems one after another, 1 <= nrhs <= 16) to
 * x_c - (z . x_c / z . z) z, the l2-orthogonal projection off span{z}: for
 * z = [0; 1_p], the removal of the pressure mean.  Asynchronous; no device
 * allocation.  PHMG_ESTATE without a kernel vector. */
phmg_status phmg_set_kernel_vector(phmg_ctx ctx, const double* z);
phmg_status phmg_project_kernel(phmg_ctx ctx, int nrhs, double* X);
phmg_status phmg_residual(phmg_ctx ctx, int level, const double* b, const double* x, double* r);

/* Per-level sizes: n, nnz(K), npatch, sum m, sum m^2, max m, the Chebyshev
 * eigenvalue estimate (0 before set-up or for Richardson), the patch-solve
 * kernel shape chosen by the set-up autotuner, the number of shapes
 * compiled for the level's precision and layout, whether the stored inverses
 * use the symmetric layout (after set-up), the SpMV kernel variant of K_l
 * (see phmg_set_spmv_variant), the stored element count, and the kernel shape
 * of the multi-right-hand-side patch solve with the number of such shapes for
 * the level's precision (block_variant is -1 until the first batched call
 * after a precision or layout change has tuned it). */
typedef struct {
    int32_t n, npatch, max_m, precision;
    int64_t nnz, sum_m, sum_m2;
    double lambda_max;
    int32_t apply_variant, apply_variants;
    int32_t symmetric_storage, spmv_variant;
    int64_t stored_elements;
    int32_t block_variant, block_variants;
} phmg_level_info;
phmg_status phmg_get_level_info(phmg_ctx ctx, int level, phmg_level_info* info);

/* Override the autotuner's patch-solve kernel shape of one level (0 <=
 * variant < apply_variants of phmg_level_info, for the level's current
 * precision and layout; kept until either changes).  Every shape computes the
 * same result bit for bit; this exists for tests and tuning studies. */
phmg_status phmg_set_apply_variant(phmg_ctx ctx, int level, int variant);

/* Override the autotuner's kernel shape of the multi-right-hand-side patch
 * solve (the batched relaxation, V-cycle and FGMRES) of one level: 0 <=
 * variant < block_variants of phmg_level_info.  Call it after the set-up that
 * fixes the level's layout; kept until the level's precision or layout
 * changes.  Shapes differ in how rows and columns are dealt to lanes, not in
 * the order of any sum: results are bit-identical.  For tests and tuning
 * studies. */
phmg_status phmg_set_block_variant(phmg_ctx ctx, int level, int variant);

/* Override the autotuner's SpMV kernel of one matrix (matrix 0: K_level, 1:
 * P_level, 2: R_level = P_level^T; the coarsest level has only K), or (matrix
 * 3) the form of the cycle's restricted residual: variant 0 computes r = b - K
 * x and then R r, variants 1-6 compute R b - (R K) x in one pass with 2, 4,
 * ..., 64 lanes per coarse row (R K is formed at create when it has no more
 * nonzeros than K; otherwise only variant 0 exists).  Variants
 * 0-5: CSR with 2, 4, ..., 64 lanes per row; 6-11: the same with the rows of
 * each XCD contiguous; 12: row blocks (at most 32 rows and 1024 nonzeros per
 * workgroup, products staged in LDS, 8 lanes per row), available when no row
 * has more than 1024 nonzeros; 13-16: CSR with 4, 8, 16, 32 lanes per row and
 * 8 (instead of 4) entries in flight per lane; 17-19: CSR with 4, 8, 16 lanes
 * per row and 4 consecutive entries per lane (16-byte index and value loads).
 * Variants differ only in summation order.  Kept
 * until the next override; for tests and tuning studies.  The adjoint cycle
 * always uses the two-step form with K^T. */
phmg_status phmg_set_spmv_variant(phmg_ctx ctx, int level, int matrix, int variant);

/* Override the autotuner's kernel shape of one block SpMM (the residuals and
 * transfers of the multi-right-hand-side path; matrix 0: K_level, 1: P_level,
 * 2: R_level; the coarsest level has only K).  Variants 0-2: 16 lanes per row
 * (one per system) with 1, 2 or 4 groups of 16 lanes per row; 3-5: the same
 * with the rows of each XCD contiguous; 6 / 7: 4 / 2 lanes per row with 4 / 8
 * systems per lane; 8 / 9: the same with XCD-contiguous rows.  Variants 0, 3
 * and 6-9 add every row's entries in row order for each system and give the
 * same bits; 1, 2, 4, 5 differ from them in rounding.  Kept until the next
 * override; for tests and tuning studies. */
phmg_status phmg_set_spmm_variant(phmg_ctx ctx, int level, int matrix, int variant);

/* Optional per-kernel, per-level timing with HIP events recorded on the
 * context stream around every launch of the selected kernels (off by
 * default).  kernel_mask has bit k set for kernel id k (0 = off).  Each timed
 * launch is bracketed by two events; results are unchanged.
 * phmg_profile_read synchronises the stream and returns the summed elapsed
 * milliseconds and the number of launches of one kernel on one level
 * (level = -1: all levels) since the last phmg_profile_reset. */
typedef enum {
    PHMG_K_PATCH_APPLY = 0,   /* batched patch solve y_i = K_i^{-1} r[S_i]           */
    PHMG_K_SCATTER = 1,       /* weighted scatter-add x += omega sum R_i^T W_i y_i   */
    PHMG_K_SPMV = 2,          /* residual and transfer SpMVs                          */
    PHMG_K_EXTRACT = 3,       /* patch extraction                                     */
    PHMG_K_FACTOR = 4,        /* patch Gauss-Jordan inversion                         */
    PHMG_K_COUNT = 5
} phmg_kernel_id;
#define PHMG_MAX_LEVELS 16
phmg_status phmg_profile_enable(phmg_ctx ctx, unsigned kernel_mask);
phmg_status phmg_profile_read(phmg_ctx ctx, int kernel, int level, double* total_ms, int64_t* launches);
phmg_status phmg_profile_reset(phmg_ctx ctx);

phmg_status phmg_hierarchy_destroy(phmg_ctx ctx);

/* Largest real part of the eigenvalues of the leading k x k block of a real
 * upper-Hessenberg matrix H (host, column-major, leading dimension ldh >= k):
 * the Chebyshev bound that relax_setup derives from its Arnoldi steps
 * (complex shifted QR).  Pure host computation. */
phmg_status phmg_ritz_max_real(const double* H, int ldh, int k, double* out);

/* Thread-local description of the last error ("" when none). */
const char* phmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PHMG_H */
