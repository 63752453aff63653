// Launchers of the batched kernels (internal).
//
// A batch is a block-diagonal matrix: system s owns rows (and columns)
// [row_off[s], row_off[s+1]). Vectors hold R right-hand sides interleaved:
// element (row i, rhs r) sits at i*R + r. Every (system, rhs) pair runs its
// own Krylov process; pair p = s*R + r.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace ppg {

// Sliced-ELL of the whole batch: 64-row slices that never cross a system
// boundary. slice[k] = {row0, nrows, sys, 0}; entries of slice k are
// sptr[k] .. sptr[k+1] (width (sptr[k+1]-sptr[k])/64), columns global.
struct BatchSell {
    const int4 *slice;
    const int32_t *sptr;
    const int32_t *scol;
    const double *sval64;
    const float *sval32;
    int nslices;
    const int *active;  // per system: 0 = skip its slices (never null)
    // pattern-coded copy (used when bpat is not null): the rows of system s
    // lie on pnd diagonals with offsets poff[s*pnd + d]; row i of system s
    // holds ptab[ptoff[s] + bpat[i]*pnd + d] on diagonal d (0 where it has
    // no entry); system s owns rows sysoff[s] .. sysoff[s+1]-1
    const uint8_t *bpat;
    const int32_t *poff;
    const int32_t *ptoff;
    const int32_t *sysoff;
    const double *ptab64;
    const float *ptab32;
    int pnd;
    // constant-coefficient box copy (used when bgx is not null; pnd == 5 and
    // the pattern fields above set): system s is a 5-point stencil on a
    // bgx[s]-wide grid whose every row is its interior row (pattern bpint[s])
    // truncated at the grid
    const int32_t *bgx;
    const int32_t *bpint;
    // launch shape: slices per wave of the pattern-coded kernel (1 or 2) and
    // the XCD-aware workgroup order (consecutive slices on one XCD) on or off
    int spw;
    int remap;
};

// Rows per reduction block; a block never crosses a system boundary.
constexpr int kBatchBlockRows = 1024;

// System-aligned row blocks for reductions: block[b] = {row0, nrows, sys, 0}
// with nrows <= kBatchBlockRows; the blocks of system s are boff[s] ..
// boff[s+1]-1.
struct BatchBlocks {
    const int4 *block;
    const int32_t *boff;
    int nblocks;
    int nsys;
    const int *active;  // per system: 0 = skip its blocks (null: all run)
};

// One chain step k of every system (desc: nsys x K step table; a step with
// spmv == -1 is skipped for that system). bufs: input, output, ping, pong,
// temporary (each n_total*R elements of the precision's type).
hipError_t launch_bchain(const BatchSell &S, int prec, int R, const PStep *desc, int K, int k, void *const bufs[5],
                         hipStream_t st);
// partial[b*ldp + c*R + r] = sum over block b of V_c[i*R+r] * w[i*R+r], c < ncols
hipError_t launch_bdots(const BatchBlocks &B, int prec, int R, const void *V, long ldv, int ncols, const void *w,
                        double *partial, int ldp, hipStream_t st);
// h[s*ldh + t] = sum over the blocks of s of partial[b*ldp + t] (t < nt, fixed
// order); if H: H[p*pstride + t/R] (hmode 1: =, 2: +=) for pair p = s*R + t%R.
hipError_t launch_bred(const BatchBlocks &B, int R, const double *partial, int ldp, int nt, double *h, int ldh,
                       double *H, long pstride, int hmode, hipStream_t st);
// w[i*R+r] -= sum_c V_c[i*R+r] h[s*ldh + c*R + r], then times scale[s*R + r]
// if scale is not null; with npart, per-block sums of the new w^2 in
// npart[b*R + r].
hipError_t launch_bupdate(const BatchBlocks &B, int prec, int R, const void *V, long ldv, int ncols, const double *h,
                          int ldh, void *w, double *npart, const double *scale, hipStream_t st);
// Fused CGS2 pass (ncols <= bupdate_dots_max_cols(prec)): w -= V h as above,
// then partial[b*ldp + c*R + r] = block b's sum of V_c w (c < ncols) and
// partial[b*ldp + ncols*R + r] its sum of w^2.
int bupdate_dots_max_cols(int prec);
hipError_t launch_bupdate_dots(const BatchBlocks &B, int prec, int R, const void *V, long ldv, int ncols,
                               const double *h, int ldh, void *w, double *partial, int ldp, hipStream_t st);
// per pair p = s*R + r: H[p*pstride + c] += h2[s*ldh + c*R + r] (c < ncols),
// H[p*pstride + ncols] = sqrt(h2[s*ldh + ncols*R + r] - sum_c h2^2), inv[p] = its inverse (0 if 0)
hipError_t launch_bfinish(const BatchBlocks &B, int R, int ncols, const double *h2, int ldh, double *H, long pstride,
                          double *inv, hipStream_t st);
// per pair: norm = sqrt(sum_b npart[b*R + r]); H[p*pstride] = norm; inv[p] = 1/norm (0 if 0)
hipError_t launch_bnorm(const BatchBlocks &B, int R, const double *npart, double *H, long pstride, double *inv,
                        hipStream_t st);
// out[i*R+r] = (T_out)(in[i*R+r] * scale[p])
hipError_t launch_bscale(const BatchBlocks &B, int prec_in, int prec_out, int R, const void *in, const double *scale,
                         void *out, hipStream_t st);
// out[i*R+r] = sum_j V_j[i*R+r] z[p*ldz + j], j < k[p] (device int per pair)
hipError_t launch_bcombine(const BatchBlocks &B, int prec, int R, const void *V, long ldv, const int *k,
                           const double *z, int ldz, void *out, hipStream_t st);

// Givens least squares of every (system, rhs) pair on the device, the same
// arithmetic as the host's GivensLS (no contraction of multiply-adds): pair
// p's rotated Hessenberg matrix Rm + p (m+1) m (column-major, leading
// dimension m + 1), its rotations c, s + p m and right-hand side
// g + p (m+1). Per pair: fro2 (sum of squares of its Hessenberg entries),
// target (the cycle stops once the shortcut residual |g[j+1]| is at or
// below it), sc (the last shortcut residual), run (1 while its Arnoldi
// process runs), k (columns kept), steps (Arnoldi steps taken this cycle).
// act: per system, 1 while one of its pairs runs (the masked kernels' flags).
struct BGivens {
    double *Rm, *c, *s, *g, *fro2, *target, *sc;
    int *run, *k, *steps, *act;
    int m, R, nsys;
};
// The delayed Gram-Schmidt of a cycle (two basis sweeps per step; pair p's
// pending vector u, w = phi(A) u):
//  launch_bdots2: partial[b*ldp + c*R + r] = V_c^T u, [(ncols + c)*R + r] =
//    V_c^T w (c < ncols), [2 ncols R + r] = u^T u, [(2 ncols + 1) R + r] =
//    u^T w over block b (reduce per system with launch_bred, nt = 2 (ncols+1) R);
//  launch_bdcgs_step: per pair, completes Hessenberg column j-1 (Hf + p*ldhp
//    + (j-1)*ldc, rows 0..j) from pend and rho = sqrt(u^T u - |V^T u|^2), and
//    unless final_step forms the next pending coefficients pend, g (per pair,
//    stride ldc) and coef[2p] = 1/rho, coef[2p+1] = g_j;
//  launch_bupdate2: v_j = (u - V a) / rho into vout and u = w / rho - V g -
//    v_j g_j, one read of V (ncols <= bdcgs_max_cols()).
hipError_t launch_bdots2(const BatchBlocks &B, int prec, int R, const void *V, long ldv, int ncols, const void *u,
                         const void *w, double *partial, int ldp, hipStream_t st);
hipError_t launch_bdcgs_step(const BatchBlocks &B, int R, int j, const double *dd, int ldd, double *Hf, long ldhp,
                             int ldc, double *pend, double *g, double *coef, int final_step, hipStream_t st);
hipError_t launch_bupdate2(const BatchBlocks &B, int prec, int R, const void *V, long ldv, int ncols, const double *dd,
                           int ldd, const double *g, int ldc, const double *coef, void *u, const void *w, void *vout,
                           hipStream_t st);
int bdcgs_max_cols();
// Start of a cycle: g = beta e1, fro2 = 0, k = steps = 0, act from run.
hipError_t launch_bgivens_init(const BGivens &G, const double *beta, hipStream_t st);
// Arnoldi step j: for every running pair, its Hessenberg column
// Hc[p ldh .. p ldh + j + 1] joins its least squares; the pair stops on a
// non-finite column (the column is dropped), on breakdown
// (h_{j+1,j} <= tol_brk sqrt(fro2)) or when |g[j+1]| <= target.
hipError_t launch_bgivens_step(const BGivens &G, int j, const double *Hc, int ldh, double tol_brk, hipStream_t st);
// flag[0] (device int) = 1 if some system has a running pair (act), else 0.
hipError_t launch_bany(const int *act, int nsys, int *flag, hipStream_t st);
// z[p ldz + i] (i < k[p]) solves the pair's triangular system R z = g.
hipError_t launch_bgivens_solve(const BGivens &G, double *z, int ldz, hipStream_t st);

}  // namespace ppg
