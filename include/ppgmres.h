/*
 * ppgmres.h - C ABI of the MI355X (gfx950) polynomial-preconditioned GMRES
 * library (Loe & Morgan, "Toward Efficient Polynomial Preconditioning for
 * GMRES", arXiv 1911.07065).
 *
 * Conventions for every entry point:
 *  - Plain C types only. "device" pointers are HIP device memory owned by the
 *    caller; "host" pointers are ordinary CPU memory owned by the caller.
 *    The library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are ordered on that stream; results written to device memory are
 *    valid after the stream is synchronised. Entry points that return host
 *    results (info structs, roots) synchronise the stream themselves.
 *  - Indices are int32, values are IEEE binary64 unless stated otherwise.
 *  - Negative status = error: outputs are left unspecified, pp_last_error()
 *    returns a message (thread-local). Positive status = warning with valid
 *    outputs. No C++ exception crosses the boundary.
 *  - Handles (pp_matrix, pp_poly) are library-owned; a pp_poly is immutable
 *    after creation and may be shared between streams; a pp_matrix holds
 *    scratch memory and must not be used by two streams at once.
 */
#ifndef PPGMRES_H
#define PPGMRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PP_OK = 0,
    PP_NOCONV = 1,     /* tolerance not reached (max cycles or stall); best x returned */
    PP_BREAKDOWN = 2,  /* setup Krylov space invariant at k < d: degree lowered to k */
    PP_UNSTABLE = 3,   /* stability check above its threshold */
    PP_EINVAL = -1,    /* bad argument */
    PP_ENOMEM = -2,    /* device or host allocation failed */
    PP_EDEVICE = -3,   /* HIP runtime error */
    PP_ESINGULAR = -4  /* H_dd singular or a zero harmonic Ritz value */
} pp_status;

/* Arithmetic of a chain / Krylov vectors. */
typedef enum {
    PP_F64 = 0,   /* binary64 storage and arithmetic */
    PP_F32 = 1,   /* binary32 storage and arithmetic */
    PP_BF16S = 2  /* bfloat16 vector storage, binary32 arithmetic, binary32 matrix values */
} pp_prec;

/* Which polynomial pp_apply evaluates. */
typedef enum {
    PP_APPLY_P = 0,   /* y = p(A) v      (Algorithm 3; eq. 3.1) */
    PP_APPLY_PHI = 1, /* y = phi(A) v = v - pi(A) v  (Algorithm 1) */
    PP_APPLY_PI = 2   /* y = pi(A) v     (eqs. 2.1, 2.2) */
} pp_apply_kind;

typedef struct pp_matrix_s *pp_matrix;
typedef struct pp_poly_s *pp_poly;

/* Result of pp_gmres_setup. */
typedef struct {
    int d;           /* degree reached (number of harmonic Ritz values) */
    int d_eff;       /* roots after Algorithm 2 (d + n_added) */
    int n_added;     /* roots added for stability */
    int breakdown;   /* 1 if the setup Krylov space became invariant */
    int64_t mvps;    /* sparse products used by the setup cycle */
    int64_t dots;    /* inner products and norms used by the setup cycle */
    double t_setup_s;
} pp_setup_info;

/* Options of pp_solve. */
typedef struct {
    int m;            /* GMRES restart length (Krylov dimension per cycle) */
    int max_cycles;   /* cycle limit */
    double tol;       /* stop when ||b - A x|| <= tol ||b|| */
    pp_prec inner;    /* precision of the phi/p chains and the Krylov basis */
    int stall_cycles; /* NOCONV if this many cycles cut ||r|| by < 1% (0: off) */
    double inner_eta; /* a reduced-precision cycle stops once its shortcut residual is
                         <= max(tol ||b||, inner_eta ||r||); 0 = default (1e-5 FP32,
                         1e-2 BF16); ignored for FP64 cycles */
    double *history;  /* optional host array: true relative residual before each cycle
                         and at the end (history_cap entries at most) */
    int history_cap;
    int new_poly_degree; /* > 0: the variant of section 5.2 (ChPoly): every cycle first builds
                            a new polynomial of this degree from one GMRES(d) cycle started at
                            the current residual, and uses it for that cycle's phi and p; the
                            polynomial argument of pp_solve may then be NULL. 0: off */
    int new_poly_add;    /* ChPoly: add roots for stability (Algorithm 2) */
    int graphs;          /* pp_batch_solve: 1 = capture the device work of a restart cycle (the
                            Arnoldi steps with their chains, Gram-Schmidt and the Givens updates
                            of every pair, then the correction and the true residual), per
                            segment of graph_steps steps and per precision, into HIP graphs and
                            replay them in later cycles; 0 = launch the same work eagerly. Same
                            results either way. Ignored by pp_solve. */
    int graph_steps;     /* pp_batch_solve: the cycle runs in segments of this many Arnoldi steps
                            (each a graph with opts->graphs); between segments the host reads one
                            flag and skips the rest of the cycle once every pair has stopped.
                            0 = the whole cycle as one segment. Ignored by pp_solve. */
    int lookahead;       /* pp_solve: 1 = after queueing an Arnoldi step, also queue phi(A) of the
                            next basis vector before the host waits for the step's Hessenberg
                            column (the GPU keeps working while the host runs the Givens
                            update), unless the shortcut residuals so far say the step may end
                            the cycle: the last residual times the last step's reduction factor
                            must exceed the target by more than the ratio of one phi(A)
                            application's time (tuned launch time x launches) to a host round
                            trip (15 us), at least 2; never on a cycle's first step. A wrong
                            guess costs one phi(A) application,
                            whose result is discarded; the iterates are the same either way.
                            0 = wait for the column first. Ignored by pp_batch_solve. */
} pp_solve_opts;

/* Result of pp_solve. */
typedef struct {
    int status;            /* pp_status of the solve */
    int cycles;            /* restarts + 1 */
    int iters;             /* outer Arnoldi steps in total */
    int fp64_cycles;       /* cycles run with FP64 inner arithmetic */
    int64_t mvps;          /* sparse products (solve only) */
    int64_t vops;          /* length-n vector operations */
    int64_t dots;          /* inner products and norms */
    double relres;         /* true ||b - A x|| / ||b|| in FP64 */
    double relres_shortcut;/* last cycle's ||beta e1 - Hbar z|| / ||b|| */
    double t_solve_s;
    int lookahead_discarded; /* phi(A) applications queued ahead (pp_solve_opts.lookahead) that the
                                cycle did not need; not counted in mvps */
} pp_info;

/* ------------------------------------------------------------------ */
/* Matrix handle                                                        */
/* ------------------------------------------------------------------ */

/* Wrap a square CSR matrix that lives in device memory (section 1: A is
 * large, sparse, real and nonsymmetric).
 *   n, nnz   : size and number of stored entries (nnz < 2^31).
 *   rowptr   : device int32[n+1], rowptr[0] = 0, non-decreasing.
 *   colind   : device int32[nnz], column indices in [0, n).
 *   val      : device double[nnz].
 * The arrays are borrowed, not copied: they must stay valid and unchanged
 * (except through pp_matrix_set_values) while the handle lives. The library
 * allocates a float32 copy of the values and a row-tile plan.
 * Errors: PP_EINVAL on bad sizes or a malformed rowptr, PP_ENOMEM, PP_EDEVICE. */
pp_status pp_matrix_create(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *colind,
                           const double *val, void *stream, pp_matrix *out);

/* Point the handle at new values (same pattern), e.g. after a parameter
 * update; refreshes the float32 copy. val: device double[nnz]. */
pp_status pp_matrix_set_values(pp_matrix A, const double *val, void *stream);

/* Release the handle and its scratch memory (not the caller's arrays). */
void pp_matrix_destroy(pp_matrix A);

/* Autotune the chain-step kernel for this matrix and precision: every
 * variant (row tiles with LDS row sums, or LPR lanes per row with U rows in
 * flight, each with and without the XCD-aware workgroup order) is timed on
 * one sparse product and the fastest is kept in the handle. Runs by itself
 * before a precision's first chain; variant/remap/us_per_launch (host, may
 * be NULL) receive the choice and its time per launch in microseconds. */
pp_status pp_matrix_tune(pp_matrix A, int prec, void *stream, int *variant, int *remap,
                         double *us_per_launch);

/* Force a chain-step variant (0 <= variant < 34, remap 0/1; 15 = persistent) for a precision
 * instead of tuning, e.g. to test every variant. Variant 31 (box) applies to a
 * constant-coefficient 5- or 7-point box stencil (see pp_matrix_march's
 * `constant`) whose grid lines hold a multiple of 4 points: it reads no
 * per-row matrix data, only the interior row's coefficients, and sums each
 * row's terms as the pattern-coded variants do; PP_EINVAL elsewhere.
 * Variants 32 and 33 (csort4, csort2) read the column-sorted copy that
 * pp_matrix_create builds for matrices of at least 4096 rows without a
 * diagonal-format copy: rows in blocks of 8192, columns in 16 to 128 bands,
 * each (block, band) tile's entries sorted by column so that a wave's
 * gathers share cache lines; a second launch adds, per row, the diagonal
 * product and the 4 (csort4) or 2 (csort2) partial sums in band order, then
 * finishes the step. PP_EINVAL when the copy is absent. */
pp_status pp_matrix_set_variant(pp_matrix A, int prec, int variant, int remap);

/* The chain-step variant in use for a precision, without tuning: variant
 * (host) receives -1 if the precision has not been tuned or set yet, 15 when
 * the persistent kernel is in use; remap and us_per_launch (host, may be
 * NULL) receive the XCD remap flag and the tuned time per launch in
 * microseconds (0 if the variant was forced). */
pp_status pp_matrix_variant(pp_matrix A, int prec, int *variant, int *remap, double *us_per_launch);

/* Two chain steps per launch (Algorithms 1 and 3: two consecutive real
 * roots, or the two sparse products of one conjugate pair). On a matrix whose rows are the
 * points of a gx x gy x gz box with entries only on the diagonals 0, +-1,
 * +-gx (and +-gx gy), none joining the end of a grid line to the start of
 * the next (5- and 7-point stencils; detected at pp_matrix_create), one
 * launch applies both factors: a workgroup stages its tile of the input and
 * two grid points around it, forms the first factor's result on the tile
 * and one point around it, and the second factor on the tile. The results
 * equal two single launches up to the order of rounding. pp_matrix_tune
 * turns it on for a precision when one launch beats two single steps;
 * pp_matrix_set_variant turns it off.
 *   pp_matrix_set_pair_steps: mode 1 on, 0 off, for a tuned (or set)
 *     precision; PP_EINVAL for mode 1 on a matrix without the box geometry or
 *     its pattern-coded copy, or for bfloat16 vectors.
 *   pp_matrix_pair_steps: *mode (host) 1 if in use; box (host int[3], may be
 *     NULL) the geometry, zeros if none; us_pair (host, may be NULL) the tuned
 *     time of one two-step launch in microseconds (0 if not timed). */
pp_status pp_matrix_set_pair_steps(pp_matrix A, int prec, int mode);
pp_status pp_matrix_pair_steps(pp_matrix A, int prec, int *mode, int *box, double *us_pair);

/* Several chain steps per launch, marching along the grid (Algorithms 1 and
 * 3): on a box-stencil matrix (as for pp_matrix_set_pair_steps) up to
 * `steps` consecutive steps that each apply one sparse product without the
 * accumulator of p (the real-root steps and conjugate-pair steps of a phi or
 * pi chain) run as one launch. A workgroup owns an x-y tile (an x range in
 * 2-D) and a chunk of cz planes along z (y in 2-D); it keeps the last three
 * planes of every intermediate result, on the tile and the points around it
 * that the later steps read, in LDS, so a launch reads its input and the
 * pattern bytes and writes its last result once. The results equal single
 * launches up to the order of rounding. pp_matrix_tune times 2, 3 and 4
 * steps per launch (and a few chunk sizes) and keeps the count with the
 * lowest time per step when it beats a single step.
 *   pp_matrix_set_march: steps 0 (off) or 2..4 (every group of at least two
 *     fusable steps marches), cz planes per chunk (0: a default that gives
 *     at least 1024 workgroups), depth 1..3 planes of loads a workgroup keeps
 *     in flight (0: 1; more than 1 only on constant-coefficient stencils,
 *     see below); PP_EINVAL for a matrix without the box
 *     geometry or its pattern-coded copy, bfloat16 vectors, or a precision
 *     not tuned or set yet. pp_matrix_set_variant turns it off.
 *   pp_matrix_march: *steps (host) the count in use (0: none), cz and us
 *     (host, may be NULL) its chunk size and tuned time per launch;
 *     constant (host, may be NULL) 1 when every row is one interior row's
 *     stencil truncated at the box (a constant-coefficient stencil): the
 *     kernel then takes that row's coefficients for every point and reads
 *     no pattern bytes. */
pp_status pp_matrix_set_march(pp_matrix A, int prec, int steps, int cz, int depth);
pp_status pp_matrix_march(pp_matrix A, int prec, int *steps, int *cz, double *us, int *constant);

/* Two chain steps per launch on whole grid lines (the fusion rules of
 * pp_matrix_set_march with two steps): on a constant-coefficient 7-point box
 * stencil whose grid lines hold 64, 128 or 256 points, a workgroup owns a
 * block of whole x-lines (a few in y by a few in z), stages the input on
 * them and two lines around them in y and z in LDS, forms the first step on
 * its lines and one line around them, then the second step, which it
 * stores. There is no halo along the lines and no per-point index
 * arithmetic, which suits grids too small for marching to fill the GPU.
 * The results equal single launches up to the order of rounding.
 * pp_matrix_tune times it beside the marching kernel's two-step launches
 * and keeps the faster.
 *   pp_matrix_set_march_shape: shape 1 turns it on (every group of two
 *     fusable steps runs one such launch; pp_matrix_march then reports
 *     steps 2), 0 returns two-step groups to the marching kernel; PP_EINVAL
 *     where it does not apply, for bfloat16 vectors, or for a precision not
 *     tuned or set yet. pp_matrix_set_variant and pp_matrix_set_march turn it
 *     off.
 *   pp_matrix_march_shape: *shape (host) 1 while two-step launches use it. */
pp_status pp_matrix_set_march_shape(pp_matrix A, int prec, int shape);
pp_status pp_matrix_march_shape(pp_matrix A, int prec, int *shape);

/* Composition with a diagonal right preconditioner M^{-1} = diag(s)
 * (eqs. (1.3)-(1.4), section 1): from now on the handle's operator is
 * A diag(s). Its chains, pp_gmres_setup (the polynomial is built for
 * A M^{-1}, section 3.1) and pp_apply use the scaled values, and pp_solve
 * solves phi(A M^{-1}) y = b and returns x = diag(s) p(A M^{-1}) y (the
 * solution of A x = b; residuals are those of A x = b).
 *   s : device double[n] (copied), or NULL for Jacobi, s_i = 1 / a_ii of the
 *       current values (recomputed by every pp_matrix_set_values).
 * The handle then owns a scaled copy of the values; the caller's values
 * stay borrowed and unchanged. Returns PP_ESINGULAR (Jacobi) if a row has no
 * stored diagonal or a zero one; on any error the handle reverts to the
 * unscaled matrix. */
pp_status pp_matrix_right_scale(pp_matrix A, const double *s, void *stream);

/* Copy the right scaling s of a scaled handle into s (device double[n]);
 * PP_EINVAL if the handle has none. */
pp_status pp_matrix_scale(pp_matrix A, double *s, void *stream);

/* Composition with block-Jacobi (eqs. (1.3)-(1.4), section 1, and
 * section 3.1: the polynomial is built for A M^{-1}): M is the block
 * diagonal of A in blocks of bs consecutive rows (1 <= bs <= 64; the last
 * block holds the remaining rows). B = A M^{-1} is a new sparse matrix
 * (row i of B gathers a_ij times row j of M^{-1}, so B holds whole blocks of
 * columns), built on the host from A's current values:
 *   pp_block_jacobi_nnz writes B's number of stored entries (host *nnz_b);
 *   pp_block_jacobi fills caller-allocated device arrays with B's CSR
 *     (rowptr_b int32[n+1], colind_b int32[nnz_b] ascending in each row,
 *     val_b double[nnz_b]) and M^{-1}'s blocks (minv double[ceil(n/bs) bs bs],
 *     block k row-major at minv + k bs bs, entry (r, c) of the block is
 *     (M^{-1})_{k bs + r, k bs + c});
 *   pp_matrix_right_blocks attaches minv (copied) to a handle B made from
 *     those arrays: pp_solve on B then solves phi(B) y = b and returns
 *     x = M^{-1} p(B) y, the solution of A x = b (after a right scaling of
 *     B, if any, is undone); pp_gmres_setup and pp_apply work on B.
 * PP_ESINGULAR if a diagonal block is singular (a zero pivot after partial
 * pivoting, in double); PP_ENOMEM if the host copies of B or M^{-1} cannot
 * be allocated. PP_EINVAL if A already has a right scaling or
 * right blocks (its solution would then need both undone). A handle with
 * right blocks has no transpose (pp_matrix_transpose returns PP_EINVAL). */
pp_status pp_block_jacobi_nnz(pp_matrix A, int bs, void *stream, int64_t *nnz_b);
pp_status pp_block_jacobi(pp_matrix A, int bs, int32_t *rowptr_b, int32_t *colind_b, double *val_b, double *minv,
                          void *stream);
pp_status pp_matrix_right_blocks(pp_matrix B, int bs, const double *minv, void *stream);

/* Name of a chain-step variant ("tile8x1", "vec8x4", ...). */
const char *pp_chain_variant_name(int variant);

/* Transposed pattern of A for the adjoint solve (p(A)^T = p(A^T)).
 * Outputs (device, caller-allocated): rowptr_t int32[n+1], colind_t
 * int32[nnz], perm int32[nnz] with val_t[k] = val[perm[k]]. Entries of a
 * row of A^T are in ascending column order (stable counting sort). */
pp_status pp_matrix_transpose(pp_matrix A, int32_t *rowptr_t, int32_t *colind_t, int32_t *perm,
                              void *stream);

/* out[k] = in[perm[k]] for k < nnz (device double arrays). */
pp_status pp_gather(int64_t nnz, const double *in, const int32_t *perm, double *out, void *stream);

/* Gradient of a loss through A x = b with respect to the stored values:
 * dval[k] = -lam[row(k)] * x[col(k)]  (lam solves A^T lam = dL/dx).
 * lam, x: device double[n]; dval: device double[nnz]. */
pp_status pp_adjoint_values(pp_matrix A, const double *lam, const double *x, double *dval,
                            void *stream);

/* ------------------------------------------------------------------ */
/* Polynomial                                                           */
/* ------------------------------------------------------------------ */

/* Build the preconditioning polynomial (Algorithm 4 step 1): one GMRES(d)
 * cycle on A from v0 (FP64 Arnoldi with classical Gram-Schmidt applied
 * twice, on the device), harmonic Ritz values from the Hessenberg matrix
 * (host), modified Leja ordering and, if add_roots, Algorithm 2's added
 * roots (host).
 *   v0: device double[n], the random start vector (section 3.6 advises a
 *       random vector, not the right-hand side); not modified.
 *   d : requested degree, 1 <= d <= n and d <= 4096.
 * Returns PP_BREAKDOWN (with a valid polynomial of lower degree) if the
 * Krylov space became invariant, PP_ESINGULAR if H_dd is singular or a root
 * is zero. info may be NULL. */
pp_status pp_gmres_setup(pp_matrix A, const double *v0, int d, int add_roots, void *stream,
                         pp_poly *out, pp_setup_info *info);

/* The same polynomial setup (Algorithm 4 step 1) with the Krylov vectors of
 * the GMRES(d) cycle stored in `basis` precision: PP_F64 (as pp_gmres_setup)
 * or PP_F32 (binary32 vectors, half the bytes of the Gram-Schmidt sweeps and
 * the sparse products; dot products, norms and the Hessenberg matrix are
 * still accumulated in FP64). The harmonic Ritz values of a PP_F32 basis
 * differ from the FP64 ones by the rounding of the stored vectors (5e-8 to
 * 2e-7 relative on 2-D convection-diffusion); the polynomial is a
 * preconditioner, so a solve still reaches its tolerance through the FP64
 * residual and refinement. Arguments and returns as pp_gmres_setup;
 * PP_EINVAL for another basis. */
pp_status pp_gmres_setup_basis(pp_matrix A, const double *v0, int d, int add_roots, int basis, void *stream,
                               pp_poly *out, pp_setup_info *info);

/* Options of the stability check run by pp_gmres_setup_checked (section 3.5). */
typedef struct {
    const double *b; /* device double[n]: the problem right-hand side the check uses */
    double tol;      /* instability is predicted when StCh > tol * ||b|| */
    int d_step;      /* > 0: lower the degree by d_step while instability is predicted */
    int d_min;       /* lowest degree tried when lowering (values < 1 mean 1) */
} pp_stch_opts;

/* pp_gmres_setup followed by the stability check of section 3.5, which is
 * computed once the polynomial is known and lets the degree be lowered when
 * it predicts instability. The GMRES(d) cycle runs once; the polynomial of
 * degree k < d comes from the leading (k+1) x k block of its Hessenberg
 * matrix (the first k Arnoldi steps from v0 are the GMRES(k) cycle), so
 * lowering costs host eigenvalue work and one check per degree tried.
 * Degrees d, d - d_step, ... (not below d_min) are tried in turn; the first
 * with StCh <= tol ||b|| is returned with PP_OK (or PP_BREAKDOWN as for
 * pp_gmres_setup). If none passes, the one with the smallest StCh (NaN
 * counting as infinite) is returned with the warning PP_UNSTABLE: the
 * polynomial is valid. stch (host, may be NULL) receives its StCh. info->d
 * is the degree returned; info->mvps and info->dots include the checks. */
pp_status pp_gmres_setup_checked(pp_matrix A, const double *v0, int d, int add_roots, const pp_stch_opts *opts,
                                 void *stream, pp_poly *out, pp_setup_info *info, double *stch);

/* Double polynomial (section 6): one GMRES(d2) cycle with the operator
 * phi1(A), started at v0, gives the roots of phi2 (Algorithm 4 step 1 and
 * Algorithm 2 applied to phi1(A)). The result is the composite polynomial
 * phi2(phi1(A)): pp_apply and pp_solve then use phi(A) = phi2(phi1(A)) and
 * p(A) = p1(A) p2(phi1(A)), with phi1(a) = a p1(a) and phi2(a) = a p2(a)
 * (so A p(A) = phi(A)); its degree is d_eff(phi1) * d_eff(phi2). The
 * composite keeps its own copy of phi1 (p1 may be destroyed afterwards).
 * pp_poly_roots gives phi2's roots (PP_ROOTS_FINAL/THETA/LEJA) and phi1's
 * final roots (PP_ROOTS_INNER). info as for pp_gmres_setup, for phi2 (mvps
 * counts the sparse products: d2 applications of phi1). Not accepted by
 * pp_batch_solve. */
pp_status pp_gmres_setup_double(pp_matrix A, pp_poly p1, const double *v0, int d2, int add_roots, void *stream,
                                pp_poly *out, pp_setup_info *info);

/* Flags of pp_poly_from_roots. */
#define PP_ROOTS_ADD 1        /* add roots for stability (Algorithm 2) */
#define PP_ROOTS_KEEP_ORDER 2 /* use the list as given: no Leja ordering, no added
                                 roots; pairs must be adjacent (a+bi, a-bi) */

/* Build a polynomial from given roots (host arrays, conjugate pairs
 * present as exact conjugates): modified Leja ordering and, with
 * PP_ROOTS_ADD, added roots as in pp_gmres_setup; with PP_ROOTS_KEEP_ORDER
 * the list is applied in the given order. */
pp_status pp_poly_from_roots(int d, const double *re, const double *im, int flags, pp_poly *out);

/* Which root list pp_poly_roots copies. */
#define PP_ROOTS_FINAL 0  /* ordered list with added roots (what the chains apply) */
#define PP_ROOTS_THETA 1  /* harmonic Ritz values as the eigensolver returned them */
#define PP_ROOTS_LEJA 2   /* original roots in modified Leja order */
#define PP_ROOTS_INNER 3  /* composite polynomial: the final roots of the inner phi1 */

/* Copy a root list (host). cap: capacity of re/im (re/im may be NULL to
 * query sizes); len receives the list length (PP_EINVAL if cap < len).
 * d_orig / n_added may be NULL. */
pp_status pp_poly_roots(pp_poly p, int which, int cap, double *re, double *im, int *len, int *d_orig,
                        int *n_added);

void pp_poly_destroy(pp_poly p);

/* ------------------------------------------------------------------ */
/* Hot path                                                             */
/* ------------------------------------------------------------------ */

/* y = p(A) v, phi(A) v or pi(A) v by the root-product chain (Algorithms 1
 * and 3), every sparse product fused with its vector updates.
 *   v, y : device vectors of n elements of type prec (double, float or
 *          bfloat16 bits as uint16); v is not modified; y must not alias v.
 * Chains of float32/bfloat16 use the float32 copy of the values. */
pp_status pp_apply(pp_poly p, pp_matrix A, int kind, int prec, const void *v, void *y,
                   void *stream);

/* pp_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as pp_apply, with the chain's three temporary
 * vectors in a fixed 48 MiB scratch array that the library holds on each GPU
 * it runs on until the process ends. It calls no hipMalloc, hipFree or other
 * allocating routine.
 *   Limits: 3 vectors of n elements (rounded up to 64) of the precision must
 *   fit: n <= 2,097,152 in FP64, 4,194,304 in FP32, 8,388,608 in BF16;
 *   otherwise PP_EINVAL. The precision must already be tuned or set
 *   (pp_matrix_tune / pp_matrix_set_variant, not the persistent variant),
 *   and p must not be a double polynomial; otherwise PP_EINVAL.
 *   Nothing in the scratch needs to start at zero: every temporary is
 *   written before it is read. All calls on one GPU share its scratch, so
 *   calls that overlap in time on one GPU (other streams, other threads)
 *   race; order them on one stream. v, y as for pp_apply. */
pp_status pp_apply_noalloc(pp_poly p, pp_matrix A, int kind, int prec, const void *v, void *y, void *stream);

/* Device-memory traffic of one pp_apply(p, A, kind, prec) as the library runs
 * it now (the tuned chain variant and two-step fusion of that precision; the
 * precision is tuned first if it has not been): the bytes each launch must
 * move by its definition, summed over the launches of the chain
 * (Algorithms 1 and 3): the matrix data its storage format holds (values and
 * column indices, or diagonal values, or 1-byte value codes, or one pattern
 * byte per row and the pattern table; row pointers or slice offsets; partial
 * row sums between column bands), one read of the input vector, the aux and
 * final vectors a step reads, the accumulator of p (read unless the step
 * initialises it, then written) and one write of the output. A fused pair of
 * steps reads its input and matrix data once and does not store the first
 * step's result. This is the byte count a bandwidth figure of the chain is
 * divided by; it is not a hardware counter.
 *   bytes (host): the total; launches (host, may be NULL): kernel launches.
 * PP_EINVAL on a bad argument; tuning errors as pp_matrix_tune. */
pp_status pp_chain_bytes(pp_poly p, pp_matrix A, int kind, int prec, void *stream, int64_t *bytes,
                         int64_t *launches);

/* Launch floor, a measurement aid beside pp_chain_bytes: queue `launches`
 * back-to-back launches of an empty kernel of `blocks` workgroups of
 * `threads` threads on the stream (nothing is read or written). Timing them
 * with events on the same stream gives the cost of a kernel boundary at that
 * grid shape, which bounds a chain launch from below however few bytes it
 * moves. PP_EINVAL unless 1 <= launches <= 100000, 1 <= blocks < 2^31 and
 * threads is 64, 128, 256, 512 or 1024. */
pp_status pp_launch_floor(int launches, int64_t blocks, int threads, void *stream);

/* Solve A x = b by PP(d)-GMRES(m) (Algorithm 4 step 2), x_0 = 0.
 * Each cycle starts from the true residual r = b - A x computed in FP64;
 * the cycle runs GMRES(m) on phi(A) in opts->inner precision and adds
 * p(A)(V z) to x in FP64 (z minimises ||r|| e_1 - Hbar z) (iterative refinement when inner is not
 * FP64). A mixed cycle that fails to halve ||r|| is followed by an FP64 one.
 *   b, x : device double[n]; x is overwritten.
 * With opts->new_poly_degree > 0 each cycle uses its own polynomial (see
 * pp_solve_opts); info->mvps and info->dots then include those setups.
 * Returns PP_OK or PP_NOCONV (x is then the last iterate); info may be NULL. */
pp_status pp_solve(pp_poly p, pp_matrix A, const double *b, double *x, const pp_solve_opts *opts,
                   void *stream, pp_info *info);

/* Device memory of pp_solve, for a caller that must bound it beforehand. The
 * handle owns the solve's workspace and allocates it on first use (then keeps
 * it for later calls): the Krylov basis of m + 1 columns and 5 work vectors in
 * the inner precision and in FP64 (rows padded to a multiple of 64), 5 more
 * per precision for a composite (double) polynomial, the reduction buffers
 * of the widest Gram-Schmidt pass and, with ChPoly, each cycle's
 * Hessenberg matrix (see pp_solve_opts).
 *   total (host, may be NULL): bytes those buffers occupy for these options;
 *   additional (host, may be NULL): bytes a pp_solve call with these options
 *     would allocate on this handle now (0 when it already holds them).
 * The handle's matrix copies (made by pp_matrix_create) are not included.
 * PP_EINVAL on a bad argument (p may be NULL only with ChPoly). */
pp_status pp_solve_workspace_bytes(pp_poly p, pp_matrix A, const pp_solve_opts *opts, int64_t *total,
                                   int64_t *additional);

/* Stability check of section 3.5: StCh = ||(b - A p(A) b) - pi(A) b|| in
 * FP64. b: device double[n]; result to *stch (host). */
pp_status pp_stability_check(pp_poly p, pp_matrix A, const double *b, void *stream, double *stch);

/* ------------------------------------------------------------------ */
/* Batched systems                                                      */
/* ------------------------------------------------------------------ */

typedef struct pp_batch_s *pp_batch;

/* Wrap many independent square systems given as one block-diagonal CSR
 * matrix in device memory: system s owns rows and columns
 * [row_off[s], row_off[s+1]) (row_off: host int64[nsys+1], row_off[0] = 0),
 * and every stored entry of a row lies in its system's diagonal block
 * (checked; PP_EINVAL otherwise). rowptr: device int32[n+1], colind: device
 * int32[nnz] (global column indices), val: device double[nnz]; copied into a
 * sliced-ELL form (64-row slices inside each system), so the arrays may be
 * freed after the call. */
pp_status pp_batch_create(int nsys, const int64_t *row_off, int64_t nnz, const int32_t *rowptr,
                          const int32_t *colind, const double *val, void *stream, pp_batch *out);

/* New values for the same pattern (device double[nnz]). Drops the
 * pattern-coded copy (the batch goes back to format 0). */
pp_status pp_batch_set_values(pp_batch B, const double *val, void *stream);

/* Storage the batch's sparse products read. 0: sliced-ELL. 1: pattern-coded
 * diagonals, built by pp_batch_create when every system's entries lie on
 * the same number of diagonals (3, 5, 7, 9, 13, 19 or 27; the offsets may
 * differ per system), no row holds two entries of one column, and each
 * system's rows take at most 256 distinct value tuples: one byte per row
 * names the row's tuple in its system's table. pp_batch_create selects 1
 * when that copy exists. 2: constant-coefficient box stencils, built beside
 * 1 when every system is a 5-point stencil on a gx x gy grid (offsets -gx,
 * -1, 0, 1, gx; gx, gy >= 3) whose every row equals the interior row with
 * the entries that fall outside the grid dropped: each system keeps only
 * its interior tuple and gx, and a row's coefficients follow from its grid
 * position. All give the same sums in a different order. pp_batch_set_format
 * returns PP_EINVAL for a format the batch has no copy of; pp_batch_format
 * writes the current one (host int). */
pp_status pp_batch_set_format(pp_batch B, int format);
pp_status pp_batch_format(pp_batch B, int *format);

/* The batched autotuner: one chain step over the whole batch is timed, on
 * the batch's own matrix, precision (PP_F64/PP_F32/PP_BF16S) and nrhs (1, 2
 * or 4), for each storage format the batch has (only the one set by
 * pp_batch_set_format, if it was called), 1 or 2 64-row slices per wave
 * (pattern-coded and box formats) and the workgroup order (consecutive slices on one
 * XCD, or not); the fastest is kept for that precision and nrhs. Runs by
 * itself in the first pp_batch_solve of a (precision, nrhs);
 * pp_batch_set_values and pp_batch_set_format clear it.
 *   pp_batch_chain_config: the shape in use (tuned, or the default:
 *     pp_batch_format's format, 1 slice per wave, XCD order on): *format
 *     (host) 0 sliced-ELL, 1 pattern-coded or 2 box; spw, remap, us (host, may be
 *     NULL) slices per wave, XCD order, tuned microseconds per step (0 if not
 *     tuned).
 *   pp_batch_set_chain_config: use this shape for (prec, nrhs) instead of
 *     tuning (format 0, 1 or 2, spw 2 only with format 1 or 2, remap 0 or 1);
 *     PP_EINVAL for a format the batch has no copy of. */
pp_status pp_batch_tune(pp_batch B, int prec, int nrhs, void *stream);

/* Orthogonalisation of pp_batch_solve's cycles (Algorithm 4 step 2).
 * delayed = 1 (default): classical Gram-Schmidt with the second pass and the
 * normalisation delayed by one step, as in the polynomial setup: two sweeps
 * of every pair's basis per Arnoldi step; a column of the Hessenberg matrix
 * is complete one step later, so each pair's least-squares update and
 * stopping test run one step behind the phi(A) products (a pair that
 * converges at column k has applied phi(A) k + 1 times in that cycle).
 * delayed = 0: CGS2, three sweeps per step, no lag. Both give the same
 * Krylov spaces up to rounding. Cycles longer than 128 steps take CGS2. */
pp_status pp_batch_set_orth(pp_batch B, int delayed);
pp_status pp_batch_orth(pp_batch B, int *delayed);
pp_status pp_batch_set_chain_config(pp_batch B, int prec, int nrhs, int format, int spw, int remap);
pp_status pp_batch_chain_config(pp_batch B, int prec, int nrhs, int *format, int *spw, int *remap, double *us);

void pp_batch_destroy(pp_batch B);

/* One polynomial per system (Algorithm 4 step 1 for every system at once):
 * GMRES(d) on each diagonal block from the matching slice of v0 (device
 * double[n]), all systems advanced in lockstep; harmonic Ritz values, Leja
 * order and added roots per system on the host. polys: host array of nsys
 * handles to receive the polynomials (each freed with pp_poly_destroy);
 * infos: host array of nsys or NULL. PP_BREAKDOWN if some system's Krylov
 * space became invariant (its degree is lowered). */
pp_status pp_batch_setup(pp_batch B, const double *v0, int d, int add_roots, void *stream, pp_poly *polys,
                         pp_setup_info *infos);

/* Solve every system for nrhs (1, 2 or 4) right-hand sides by PP-GMRES,
 * all (system, right-hand side) pairs in lockstep: each pair has its own
 * Krylov basis, Hessenberg matrix and stopping test, each system its own
 * polynomial (polys: host array of nsys). b, x: device double[n * nrhs],
 * interleaved (entry (row i, rhs r) at i*nrhs + r), each aligned to
 * 8*nrhs bytes (PP_EINVAL otherwise; fresh allocations are); x is overwritten.
 * opts as for pp_solve (opts->history receives pair 0's residuals;
 * opts->new_poly_degree must be 0). infos:
 * host array of nsys*nrhs (pair s*nrhs + r) or NULL. PP_NOCONV if some pair
 * did not converge. */
pp_status pp_batch_solve(pp_batch B, const pp_poly *polys, int nrhs, const double *b, double *x,
                         const pp_solve_opts *opts, void *stream, pp_info *infos);

/* ------------------------------------------------------------------ */
/* Host-only building blocks (deterministic; no device work)            */
/* ------------------------------------------------------------------ */

/* Harmonic Ritz values from the (k+1) x k upper Hessenberg matrix Hbar
 * (column-major, leading dimension k+1): eigenvalues of H_kk + h^2 f e_k^T
 * with H_kk^T f = e_k (Algorithm 4 step 1b); if breakdown != 0 the last row
 * is ignored and the eigenvalues of H_kk are returned. re/im: host double[k];
 * a conjugate pair is returned as exact conjugates, +imag first. */
pp_status pp_harmonic_ritz(int k, const double *hbar, int breakdown, double *re, double *im);

/* Eigenvalues of a real upper Hessenberg matrix (column-major, ld >= k) by
 * the Francis double-shift QR iteration. */
pp_status pp_hessenberg_eig(int k, const double *h, int ld, double *re, double *im);

/* Modified Leja permutation (section 2, Algorithm 2 step 1): the ordered
 * roots are re[perm[i]] + i im[perm[i]]; conjugate pairs adjacent, +imag
 * first. Exact ties go to the lowest (real, imag)-sorted index. */
pp_status pp_leja_order(int d, const double *re, const double *im, int *perm);

/* Algorithm 2 steps 2-3 on Leja-ordered roots: pof per unit (mantissa in
 * [0.5,1) and binary exponent, one entry per root position: the +imag
 * member of a pair holds the pair's value, the -imag member a copy),
 * copies per unit n_add (same layout) and the final root list with the
 * copies inserted (re_out/im_out, capacity cap, length *d_eff). With
 * add == 0 no copies are inserted (pof and n_add are still reported). */
pp_status pp_add_roots(int d, const double *re, const double *im, int add, int cap, double *re_out,
                       double *im_out, int *d_eff, int *n_add, double *pof_mant, int *pof_exp);

/* Message of the last error on this thread. */
const char *pp_last_error(void);

/* Library version string. */
const char *pp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PPGMRES_H */
