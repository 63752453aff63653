// Launchers of the device kernels (internal). All launches are asynchronous
// on the given stream; pointers are device memory. Element types:
//   prec 0: double vectors, double matrix values, double arithmetic
//   prec 1: float vectors, float matrix values, float arithmetic
//   prec 2: bfloat16 vectors (uint16 bits), float values, float arithmetic
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace ppg {

// chain-step kernel variants (the autotuner picks one per matrix and precision)
enum ChainVariant : int {
    CV_TILE8 = 0,   // tiles of <= 256 rows / 2048 entries, LDS row sums
    CV_TILE16 = 1,  // tiles of <= 512 rows / 4096 entries
    CV_VEC1x4 = 2,  // one lane per row, 4 rows per lane
    CV_VEC4x4 = 3,  // 4 lanes per row, 4 rows in flight per lane group
    CV_VEC8x2 = 4,
    CV_VEC8x4 = 5,
    CV_VEC16x2 = 6,
    CV_VEC16x4 = 7,
    CV_VEC32x2 = 8,
    CV_TILEV8 = 9,    // tile8 plan, 16-byte non-temporal loads of the entry stream
    CV_TILEV16 = 10,  // tile16 plan, same loads
    CV_VK2x4x4 = 11,  // 2 lanes per row, 4 rows per group, 4 entries per lane per batch
    CV_VK4x4x2 = 12,
    CV_VK8x4x1 = 13,
    CV_VK16x2x2 = 14,
    CV_PERSIST = 15,  // one cooperative launch per chain, grid barrier between steps (opt-in)
    CV_TILEB8 = 16,   // tile8 kernel on a plan of whole occupancy rounds of equal tiles
    CV_TILEB16 = 17,  // tile16 kernel, same
    CV_SELL = 18,     // sliced-ELL copy (64-row slices): one lane per row, coalesced gathers
    CV_SELLT = 19,    // same with ordinary (cache-allocating) loads of the entry stream
    CV_SELL2 = 20,    // sell64 with 2 slices per wave
    CV_SELL4 = 21,    // sell64 with 4 slices per wave
    CV_SELLD = 22,    // sell64 with 16-bit column offsets (banded matrices only)
    CV_SELLD4 = 23,   // same, 4 slices per wave
    CV_DIA = 24,      // diagonal format (matrices on few diagonals): 2 rows per lane
    CV_DIA4 = 25,     // same, 1 row per lane
    CV_DIAC = 26,     // diagonal format with 1-byte codes into a table of the matrix's distinct values, 4 rows per lane
    CV_DIAP = 27,     // diagonal format with one byte per row: the row's pattern in a table of distinct rows
    CV_BAND2 = 28,    // tile8x1 on 2 column bands, one launch per band (partial row sums in between)
    CV_BAND4 = 29,    // the same with 4 column bands
    CV_DIAPV = 30,    // pattern-coded diagonals, 4 consecutive rows per lane with vector loads
    CV_BOX = 31,      // constant-coefficient box stencil: no per-row matrix data, 4 points of a grid line per lane
    CV_CSORT4 = 32,   // column-sorted tiles of kCsRows rows x one column band, 4 partial sums per row
    CV_CSORT2 = 33,   // the same, 2 partial sums per row (twice the bands per workgroup)
    CV_COUNT = 34
};

// A chain step as the persistent kernel reads it from device memory.
// Buffers: 0 = input, 1 = output, 2/3 = ping-pong, 4 = temporary, -1 = none.
struct PStep {
    int spmv, in, aux, out, acc, acc_init, fin, pad;
    double a0, a1, a2, b0, b1;
};
const char *chain_variant_name(int v);
constexpr int kRedBlock = 256;       // threads per reduction workgroup
constexpr int kDotRows = 1024;       // rows per dot-product workgroup
constexpr int kDotCols = 16;         // Krylov columns per dot-product pass
constexpr int kDotsWideCols = 16;    // the setup's dot and update passes switch layout at this width
constexpr int kDotsWideRows = 1024;  // partial rows of the wide dot pass

// Pointers of one fused chain step (see Step in poly.h).
struct StepPtrs {
    const void *in;
    const void *aux;
    const void *vfin;
    void *out;
    void *acc;
    int acc_init;
    int spmv;
    double a0, a1, a2, b0, b1;
    // spmv == 0: the product term a0 * prod[r] comes from this vector (null: none)
    const void *prod = nullptr;
};

// Column-sorted tiles: rows per block, the most partial sums per row, and
// the LDS bytes a tile's products may take (two workgroups per CU).
constexpr int kCsRows = 8192;
constexpr int kCsMaxParts = 4;
constexpr int kCsLdsBytes = 80 * 1024;

// Diagonals of the diagonal format, passed by value (uniform per launch).
constexpr int kMaxDiag = 32;
constexpr int kMaxPatEntries = 1024;
constexpr int kMaxRightBlock = 64;    // largest block of a block-Jacobi right preconditioner  // rows patterns x diagonals of the pattern-coded format
struct DiaOffsets {
    int nd;               // number of diagonals (0: no diagonal-format copy)
    int off[kMaxDiag];    // column - row of each diagonal, ascending
};

// CSR in the form the kernels read.
struct DevCSR {
    int n;
    int nnz;
    const int32_t *rowptr;
    const int32_t *colind;
    const double *val64;
    const float *val32;
    const int4 *tile8;   // {r0, r1, e0, e1} per tile of the CV_TILE8 plan
    int ntile8;
    const int4 *tile16;  // same for CV_TILE16
    int ntile16;
    const int4 *tileP;   // balanced plan of the persistent kernel
    int ntileP;
    const int4 *tileB8[3];  // per precision: plans of whole occupancy rounds
    int ntileB8[3];
    const int4 *tileB16[3];
    int ntileB16[3];
    // sliced-ELL copy (absent if nslices == 0): slice s holds rows
    // [64 s, 64 s + 64) as width_s columns of 64 entries, offsets sptr[s]
    const int32_t *sptr;
    const int32_t *scol;
    const int16_t *sdel;  // column - row per entry (null if some offset exceeds 16 bits)
    const double *sval64;
    const float *sval32;
    int nslices;
    // column-banded CSR copies (c = 0: 2 bands, c = 1: 4 bands; absent if
    // bandK[c] == 0): band k holds the entries with columns in
    // [k n / K, (k+1) n / K); its row pointers are brow[c][k (n + 1) ..]
    // (offsets into bcol[c] / bval[c]) and its 256-row tiles are
    // btile[c][btoff[c][k] .. btoff[c][k+1]). bpart: n partial row sums
    // (8 bytes each) carried from one band to the next.
    const int32_t *brow[2];
    const int32_t *bcol[2];
    const double *bval64[2];
    const float *bval32[2];
    const int4 *btile[2];
    int btoff[2][5];
    int bandK[2];
    void *bpart;
    // diagonal-format copy (absent if doff.nd == 0): the entry of row i on
    // diagonal d is dval[((i / 256) nd + d) 256 + i % 256] (0 where the
    // diagonal leaves the matrix or holds no stored entry), its column
    // i + doff.off[d]; ceil(n / 256) blocks
    DiaOffsets doff;
    const double *dval64;
    const float *dval32;
    // value-coded diagonal format (absent if dcode is null): row i's codes
    // for diagonals 8g .. 8g+7 are the 8 bytes dcode[(i * G + g) * 8 ..],
    // G = ceil(nd / 8); code c stands for the value dtab[c] (code 0: zero)
    const uint8_t *dcode;
    const double *dtab64;
    const float *dtab32;
    int ntab;
    // pattern-coded diagonal format (absent if pcode is null): byte q of
    // word pcode[b * 256 + t] is the pattern of row b * 1024 + q * 256 + t;
    // the entry of a row with pattern p on diagonal d is ptab[p * nd + d]
    // (npat * nd <= kMaxPatEntries values)
    const uint32_t *pcode;
    const uint8_t *pbyte;  // the same patterns one byte per row in row order (ceil(n/1024)*1024 bytes)
    const double *ptab64;
    const float *ptab32;
    int npat;
    // column-sorted tiles (absent if cs_nb == 0): rows in blocks of kCsRows,
    // columns in cs_nb bands of cs_W (every band non-empty); tile
    // t = block * cs_nb + band holds the block's entries in the band, entries
    // cs_toff[t] .. cs_toff[t+1], sorted by column. Entry e is the word
    // cs_code[e] = (column - band cs_W) << cs_sb | slot, slot = the entry's
    // rank in the tile in row-major (CSR) order, and the value cs_val[e];
    // cs_tptr[t (kCsRows + 1) + rl] is the first slot of the block's row rl.
    // cs_dg: every row's diagonal entry, held apart from the tiles (null:
    // the diagonal is in the tiles). cs_part: kCsMaxParts n partial row sums
    // (8 bytes each). cs_maxe: the largest tile.
    const uint32_t *cs_code;
    const double *cs_val64;
    const float *cs_val32;
    const int32_t *cs_toff;
    const uint16_t *cs_tptr;
    const double *cs_dg64;
    const float *cs_dg32;
    void *cs_part;
    int cs_nb, cs_sb, cs_W, cs_maxe;
    // box geometry (box_nd == 0: none): the rows are the points of a
    // box[0] x box[1] x box[2] grid, row x + box[0] (y + box[1] z), with
    // entries only on the diagonals 0, +-1, +-box[0] (and +-box[0] box[1]
    // when box_nd == 7) and none joining the end of a grid line to the start
    // of the next; the diagonal format's d order is that ascending order
    int box[3];
    int box_nd;
    // constant-coefficient box stencil: every row is the stencil of the row
    // with pattern box_pint (an interior point) truncated at the box; -1: no
    int box_pint;
    int variant[3];      // chain variant per precision
    int remap[3];        // 1: keep neighbouring workgroups on one XCD
};

// All steps of a chain program in one cooperative launch of `grid`
// workgroups (grid <= persist_max_grid). bar: monotonically growing barrier
// counter whose value before the launch is bar_base; it grows by
// (nsteps - 1) * grid. err: set to 1 if a barrier timed out.
hipError_t launch_chain_persist(const DevCSR &A, int prec, void *const bufs[5], const PStep *steps, int nsteps,
                                unsigned long long *bar, unsigned long long bar_base, int *err, int grid, int remap,
                                hipStream_t st);
// Largest co-resident grid of the persistent kernel.
hipError_t persist_max_grid(int prec, int *grid);
// Co-resident workgroups (whole GPU) of the tile kernels with EPT 8 or 16.
hipError_t tile_slots(int prec, int ept, int *slots);

// Sliced-ELL values from CSR values: sval[k] = sperm[k] >= 0 ? val[sperm[k]] : 0.
hipError_t launch_sell_values(long npad, const int32_t *sperm, const double *val, double *sval64, float *sval32,
                              hipStream_t st);

// Tile plan on the host: tiles of <= row_cap rows and <= nnz_cap entries
// (a longer row gets a tile of its own). Returns {r0, r1, e0, e1} per tile.
void build_tiles(const int32_t *rowptr, int n, int row_cap, int nnz_cap, std::vector<int4> &out);

size_t elem_size(int prec);

hipError_t launch_chain_step(const DevCSR &A, int prec, const StepPtrs &s, hipStream_t st);

// Two consecutive chain steps, each with one sparse product, the second
// reading the first's result and at most the first's input as its aux
// vector (two real roots of Algorithm 1 or 3, or one conjugate pair):
// for each row r
//     w1 = a01 (A in)_r + a11 in_r,   w2 = a02 (A w1)_r + a12 w1_r [+ a22 in_r if aux2]
//     acc_r = (init ? 0 : acc_r) [+ b01 in_r + b11 w1_r if acc1] [+ b02 w1_r + b12 w2_r if acc2]
//     out_r = vfin ? vfin_r - w2 : w2                       (if out)
// w1 is not stored. Needs the box geometry and the pattern-coded copy;
// out and acc must not alias in (other workgroups read in around their
// tiles). FP64 and FP32 vectors only.
struct PairPtrs {
    const void *in;
    void *out;
    void *acc;
    const void *vfin;
    int acc1, acc2, init, aux2;
    double a01, a11, b01, b11;
    double a02, a12, a22, b02, b12;
    // 0: the cube-tile kernel (k_chain_pair); 1: whole-line tiles
    // (k_chain_boxt, constant-coefficient 7-point stencils, box_tile_ok)
    int shape;
};
hipError_t launch_chain_pair(const DevCSR &A, int prec, const PairPtrs &p, int remap, hipStream_t st);

// 2 to kMarchMax consecutive chain steps in one launch on a box-stencil
// matrix, marching along the slowest grid dimension (z in 3-D, y in 2-D).
// Step k computes w_{k+1} = a0[k] (A w_k) + a1[k] w_k [+ a2[k] w_{k-1} if
// bit k of aux], w_0 = in (bit 0 must be clear); the last result is stored:
// out = vfin ? vfin - w_S : w_S. No intermediate result is stored. A
// workgroup owns an x-y tile (x tile in 2-D) and a chunk of cz planes; it
// keeps the last three planes of every intermediate result (on the tile and
// the points around it that later steps need) in LDS. Needs the box
// geometry and the pattern-coded copy; out must not alias in or vfin; FP64
// and FP32 vectors only.
constexpr int kMarchMax = 4;
struct MarchPtrs {
    const void *in;
    void *out;
    const void *vfin;
    int nsteps;
    int aux;
    int depth;  // planes of loads in flight per workgroup (1..3; constant-coefficient stencils only)
    // 0: the marching kernel; 1: whole-line tiles (k_chain_boxt: two steps,
    // constant-coefficient 7-point stencil, box_tile_ok)
    int shape;
    double a0[kMarchMax], a1[kMarchMax], a2[kMarchMax];
};
// The single-step box kernel (CV_BOX) applies: a constant-coefficient 5- or
// 7-point box stencil whose grid lines hold a multiple of 4 points.
bool box_step_ok(const DevCSR &A);
// One launch of an empty kernel of `blocks` workgroups of `threads` threads (the launch floor).
hipError_t launch_empty(long blocks, int threads, hipStream_t st);
// Whole-line tiles (MarchPtrs::shape 1) apply: a constant-coefficient
// 7-point box stencil whose grid lines hold 64, 128 or 256 points, FP64 or
// FP32 vectors.
bool box_tile_ok(const DevCSR &A, int prec);
hipError_t launch_chain_march(const DevCSR &A, int prec, const MarchPtrs &p, int cz, int remap, hipStream_t st);
// Planes per chunk that give the grid at least `target` workgroups (at most
// the marching extent; a multiple of 4 where possible).
int march_default_cz(const DevCSR &A, int target);

// partial[b * ldp + k] = sum over rows of block b of V[i, k] * w[i], k < ncols.
int dot_blocks(int n);
hipError_t launch_dots(int prec, int n, const void *V, long ldv, int ncols, const void *w, double *partial,
                       int ldp, hipStream_t st);
// h[k] = sum_b partial[b * ldp + k] in fixed order; H[k] (+)= h[k] (mode 1: =, 2: +=).
hipError_t launch_reduce(int nblk, const double *partial, int ldp, int ncols, double *h, double *H, int hmode,
                         hipStream_t st);
// w[i] -= sum_k V[i,k] h[k]; with norm_partial, also per-block sums of w^2.
hipError_t launch_update(int prec, int n, const void *V, long ldv, int ncols, const double *h, void *w,
                         double *norm_partial, hipStream_t st);
// Fused w -= V h and partial[b*ldp + k] = sum over block b of V[i,k] w[i]
// (one read of V). Only for ncols <= update_dots_max_cols(prec).
int update_dots_blocks(int n);
int update_dots_max_cols(int prec);
hipError_t launch_update_dots(int prec, int n, const void *V, long ldv, int ncols, const double *h, void *w,
                              double *partial, int ldp, hipStream_t st);
// (partial column ncols of launch_update_dots holds the block's ||w_new||^2)
// H[k] += h2[k]; H[ncols] = sqrt(h2[ncols] - ||h2||^2); inv[0] = 1/H[ncols] (0 if 0).
hipError_t launch_finish_col(int ncols, const double *h2, double *H, double *inv, hipStream_t st);
// w = (w - V h) * inv[0]
hipError_t launch_update_scale(int prec, int n, const void *V, long ldv, int ncols, const double *h, void *w,
                               const double *inv, hipStream_t st);
// norm = sqrt(sum_b partial[b]); writes H[0] = norm, inv[0] = 1/norm (0 if norm == 0).
hipError_t launch_reduce_norm(int nblk, const double *partial, double *H, double *inv, hipStream_t st);
// out[i] = (T_out)(in[i] * s) with s = scale[0] (device) or, if scale is null,
// s = scale_host; in and out may alias when the types match.
hipError_t launch_scale_cast(int prec_in, int prec_out, int n, const void *in, const double *scale, double scale_host,
                             void *out, hipStream_t st);
// out[i] = sum_k V[i,k] z[k]
hipError_t launch_combine(int prec, int n, const void *V, long ldv, int k, const double *z, void *out,
                          hipStream_t st);
// x[i] += beta * d[i]   (x double)
hipError_t launch_axpy_x(int prec, int n, double beta, const void *d, double *x, hipStream_t st);
// x[i] = value (double)
hipError_t launch_fill(int n, double value, double *x, hipStream_t st);
// Delayed Gram-Schmidt of the setup cycle (FP64): the dot pass
// (partial[b*ldp + 0..ncols) = V^T u, [ncols..2 ncols) = V^T w, then u^T u,
// u^T w), the one-workgroup coefficient step (dd after reduction, H column
// j-1, pending coefficients, coef = {1/rho, g_j}, g into dd[2j+2..]) and the
// update pass (v_j into vout, the next pending vector into u). The dot pass
// uses at most max_rows partial rows and returns their number in *rows.
// prec 0: binary64 vectors; prec 1: binary32 vectors (FP64 arithmetic).
hipError_t launch_dots_pair(int prec, int n, const void *V, long ldv, int ncols, const void *u, const void *w,
                            double *partial, int ldp, int max_rows, int *rows, hipStream_t st);
hipError_t launch_dcgs_step(int j, double *dd, double *H, int ldh, double *pend, double *coef, int final_step,
                            hipStream_t st);
hipError_t launch_update_pair(int prec, int n, const void *V, long ldv, int ncols, const double *a, const double *g,
                              const double *coef, void *u, const void *w, void *vout, hipStream_t st);
// s[i] = 1/a_ii (0 and *bad = 1 where the diagonal is missing or zero)
hipError_t launch_jacobi(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double *s, int *bad,
                         hipStream_t st);
// out[k] = val[k] * s[colind[k]]
hipError_t launch_scale_cols(int nnz, const int32_t *colind, const double *val, const double *s, double *out,
                             hipStream_t st);
// x[i] *= s[i]
hipError_t launch_vmul(int n, double *x, const double *s, hipStream_t st);
// copy with conversion
hipError_t launch_convert(int prec_in, int prec_out, int n, const void *in, void *out, hipStream_t st);
// val32[k] = (float) val64[k]
hipError_t launch_val_to_f32(int nnz, const double *val64, float *val32, hipStream_t st);
// x = M^{-1} x in place, M^{-1} block diagonal with blocks of bs rows
// (bs <= kMaxRightBlock; block k row-major with stride bs at minv + k bs bs)
hipError_t launch_block_apply(int n, int bs, const double *minv, double *x, hipStream_t st);
// New values for the coded copies with their codes kept: tab[c] = val[crep[c]]
// (tab[0] = 0), ptab[i] = tab[pcodes[i]] (i < nent), and *flag = 1 if some
// entry k differs from tab[ecode[k]] (the codes are then stale).
hipError_t launch_recode(long nnz, const double *val, const uint8_t *ecode, const int32_t *crep, int ntab,
                         double *tab64, float *tab32, int nent, const uint8_t *pcodes, double *ptab64, float *ptab32,
                         int *flag, hipStream_t st);
// out[k] = in[perm[k]]
hipError_t launch_gather(int nnz, const double *in, const int32_t *perm, double *out, hipStream_t st);
// dval[k] = -lam[row(k)] * x[col(k)]
hipError_t launch_adjoint_values(const DevCSR &A, const double *lam, const double *x, double *dval,
                                 hipStream_t st);

}  // namespace ppg
