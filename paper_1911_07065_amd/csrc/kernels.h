// Launchers of the device kernels (internal). All launches are asynchronous
// on the given stream; pointers are device memory. Element types:
//   prec 0: double vectors, double matrix values, double arithmetic
//   prec 1: float vectors, float matrix values, float arithmetic
//   prec 2: bfloat16 vectors (uint16 bits), float values, float arithmetic
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ppg {

constexpr int kChainBlock = 256;     // threads per chain-step workgroup
constexpr int kChainEpt = 8;         // stored entries per thread and tile
constexpr int kTileNnz = kChainBlock * kChainEpt;
constexpr int kTileRowsMax = 4 * kChainBlock;
constexpr int kRedBlock = 256;       // threads per reduction workgroup
constexpr int kDotRows = 2048;       // rows per dot-product workgroup
constexpr int kDotCols = 8;          // Krylov columns per dot-product pass

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
};

// CSR in the form the kernels read.
struct DevCSR {
    int n;
    int nnz;
    const int32_t *rowptr;
    const int32_t *colind;
    const double *val64;
    const float *val32;
    const int32_t *tiles;  // row tile starts, ntiles + 1 entries
    int ntiles;
    int xcd_remap;         // 1: keep neighbouring tiles on one XCD
};

size_t elem_size(int prec);

hipError_t launch_chain_step(const DevCSR &A, int prec, const StepPtrs &s, hipStream_t st);

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
// copy with conversion
hipError_t launch_convert(int prec_in, int prec_out, int n, const void *in, void *out, hipStream_t st);
// val32[k] = (float) val64[k]
hipError_t launch_val_to_f32(int nnz, const double *val64, float *val32, hipStream_t st);
// out[k] = in[perm[k]]
hipError_t launch_gather(int nnz, const double *in, const int32_t *perm, double *out, hipStream_t st);
// dval[k] = -lam[row(k)] * x[col(k)]
hipError_t launch_adjoint_values(const DevCSR &A, const double *lam, const double *x, double *dval,
                                 hipStream_t st);

}  // namespace ppg
