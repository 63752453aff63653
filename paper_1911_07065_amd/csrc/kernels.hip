// Device kernels of the polynomial-preconditioned GMRES hot path (gfx950).
//
// The hot path is memory bound (a CSR sparse product moves >= 8 bytes per
// stored entry for 2 flops), so the kernels are built for HBM bandwidth:
//  * chain step: one workgroup per row tile of <= 2048 stored entries. The
//    entries of a tile are streamed with fully coalesced loads (8 independent
//    loads in flight per lane), multiplied by the gathered input, staged in
//    LDS, summed per row, and the row result is finished in the same
//    kernel by the fused vector update of Algorithm 1 or 3 (no extra pass
//    over the vectors). Tiles are remapped so that neighbouring tiles run on
//    the same XCD and share its L2 for the gathered input.
//  * Gram-Schmidt: per-workgroup partial dot products over 2048 rows, then a
//    fixed-order second pass per column: deterministic, no float atomics.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace ppg {
namespace {

// ---------------------------------------------------------------------------
// element access: double, float, bfloat16 bits (uint16)
// ---------------------------------------------------------------------------

template <typename XT>
struct Arith;
template <>
struct Arith<double> {
    using T = double;
};
template <>
struct Arith<float> {
    using T = float;
};
template <>
struct Arith<uint16_t> {
    using T = float;
};

__device__ __forceinline__ double ldx(const double *p, long i) { return p[i]; }
__device__ __forceinline__ float ldx(const float *p, long i) { return p[i]; }
__device__ __forceinline__ float ldx(const uint16_t *p, long i) {
    return __uint_as_float(((uint32_t)p[i]) << 16);
}

// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f32_to_bf16(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void stx(double *p, long i, double v) { p[i] = v; }
__device__ __forceinline__ void stx(float *p, long i, float v) { p[i] = v; }
__device__ __forceinline__ void stx(uint16_t *p, long i, float v) { p[i] = f32_to_bf16(v); }

// the value a store of v into an array of the pointer's type keeps
__device__ __forceinline__ double stored_value(const double *, double v) { return v; }
__device__ __forceinline__ double stored_value(const float *, double v) { return (double)(float)v; }
__device__ __forceinline__ double stored_value(const uint16_t *, double v) {
    return (double)__uint_as_float(((uint32_t)f32_to_bf16((float)v)) << 16);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic sum over a 256-thread block; result valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum256(T v, T *sm /* [4] */) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    T r = T(0);
    if (threadIdx.x == 0) r = ((sm[0] + sm[1]) + sm[2]) + sm[3];
    __syncthreads();
    return r;
}

__device__ __forceinline__ int remap_tile(int b, int ntiles, int remap) {
    if (!remap) return b;
    constexpr int nx = 8;  // XCDs; workgroups are dispatched round-robin over them
    const int x = b % nx, q = ntiles / nx, rem = ntiles % nx;
    return x * q + min(x, rem) + b / nx;
}

// ---------------------------------------------------------------------------
// fused chain step
// ---------------------------------------------------------------------------

template <typename VT, typename XT>
struct ChainArgs {
    const int32_t *rowptr;
    const int32_t *colind;
    const VT *val;
    const int32_t *tiles;
    int ntiles;
    int xcd_remap;
    const XT *in;
    const XT *aux;
    const XT *vfin;
    XT *out;
    XT *acc;
    typename Arith<XT>::T a0, a1, a2, b0, b1;
    int acc_init;
    int spmv;
};

template <typename VT, typename XT>
__device__ __forceinline__ void chain_epilogue(const ChainArgs<VT, XT> &a, int r, typename Arith<XT>::T s) {
    using AT = typename Arith<XT>::T;
    const AT xin = ldx(a.in, r);
    AT w = a.a0 * s + a.a1 * xin;
    if (a.aux) w += a.a2 * ldx(a.aux, r);
    if (a.acc) {
        const AT old = a.acc_init ? AT(0) : ldx(a.acc, r);
        stx(a.acc, r, old + a.b0 * xin + a.b1 * w);
    }
    if (a.out) stx(a.out, r, a.vfin ? ldx(a.vfin, r) - w : w);
}

template <typename VT, typename XT>
__global__ __launch_bounds__(kChainBlock) void k_chain(ChainArgs<VT, XT> a) {
    using AT = typename Arith<XT>::T;
    __shared__ AT buf[kTileNnz];
    __shared__ AT red[4];
    const int t = remap_tile(blockIdx.x, a.ntiles, a.xcd_remap);
    const int r0 = a.tiles[t], r1 = a.tiles[t + 1];
    const int tid = threadIdx.x;
    if (!a.spmv) {
        for (int r = r0 + tid; r < r1; r += kChainBlock) chain_epilogue(a, r, AT(0));
        return;
    }
    const int e0 = a.rowptr[r0], e1 = a.rowptr[r1];
    if (e1 - e0 <= kTileNnz) {
        int col[kChainEpt];
        VT v[kChainEpt];
#pragma unroll
        for (int k = 0; k < kChainEpt; ++k) {
            const int e = e0 + k * kChainBlock + tid;
            col[k] = 0;
            v[k] = VT(0);
            if (e < e1) {
                col[k] = a.colind[e];
                v[k] = a.val[e];
            }
        }
#pragma unroll
        for (int k = 0; k < kChainEpt; ++k) {
            const int e = e0 + k * kChainBlock + tid;
            if (e < e1) buf[k * kChainBlock + tid] = (AT)v[k] * ldx(a.in, col[k]);
        }
        __syncthreads();
        for (int r = r0 + tid; r < r1; r += kChainBlock) {
            const int s0 = a.rowptr[r] - e0, s1 = a.rowptr[r + 1] - e0;
            AT s = AT(0);
            for (int q = s0; q < s1; ++q) s += buf[q];
            chain_epilogue(a, r, s);
        }
    } else {
        // a tile with a single long row
        AT s = AT(0);
        for (int e = e0 + tid; e < e1; e += kChainBlock) s += (AT)a.val[e] * ldx(a.in, a.colind[e]);
        s = block_sum256(s, red);
        if (tid == 0) chain_epilogue(a, r0, s);
    }
}

template <typename VT, typename XT>
hipError_t chain_launch(const DevCSR &A, const VT *val, const StepPtrs &s, hipStream_t st) {
    using AT = typename Arith<XT>::T;
    ChainArgs<VT, XT> a;
    a.rowptr = A.rowptr;
    a.colind = A.colind;
    a.val = val;
    a.tiles = A.tiles;
    a.ntiles = A.ntiles;
    a.xcd_remap = A.xcd_remap;
    a.in = (const XT *)s.in;
    a.aux = (const XT *)s.aux;
    a.vfin = (const XT *)s.vfin;
    a.out = (XT *)s.out;
    a.acc = (XT *)s.acc;
    a.a0 = (AT)s.a0;
    a.a1 = (AT)s.a1;
    a.a2 = (AT)s.a2;
    a.b0 = (AT)s.b0;
    a.b1 = (AT)s.b1;
    a.acc_init = s.acc_init;
    a.spmv = s.spmv;
    if (A.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL((k_chain<VT, XT>), dim3(A.ntiles), dim3(kChainBlock), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram-Schmidt pieces
// ---------------------------------------------------------------------------

template <typename XT>
__global__ __launch_bounds__(256) void k_dots(int n, const XT *V, long ldv, int ncols, const XT *w,
                                              double *partial, int ldp) {
    constexpr int RPT = kDotRows / 256;
    __shared__ double sm[4][kDotCols];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long base = (long)blockIdx.x * kDotRows;
    double wv[RPT];
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
        const long i = base + s * 256 + tid;
        wv[s] = (i < n) ? (double)ldx(w, i) : 0.0;
    }
    for (int c0 = 0; c0 < ncols; c0 += kDotCols) {
        double acc[kDotCols];
#pragma unroll
        for (int kc = 0; kc < kDotCols; ++kc) acc[kc] = 0.0;
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
            const long i = base + s * 256 + tid;
            if (i < n) {
#pragma unroll
                for (int kc = 0; kc < kDotCols; ++kc)
                    if (c0 + kc < ncols) acc[kc] += (double)ldx(V, i + (long)(c0 + kc) * ldv) * wv[s];
            }
        }
#pragma unroll
        for (int kc = 0; kc < kDotCols; ++kc) acc[kc] = wave_sum(acc[kc]);
        if (lane == 0) {
#pragma unroll
            for (int kc = 0; kc < kDotCols; ++kc) sm[wave][kc] = acc[kc];
        }
        __syncthreads();
        if (tid < kDotCols && c0 + tid < ncols)
            partial[(long)blockIdx.x * ldp + c0 + tid] = ((sm[0][tid] + sm[1][tid]) + sm[2][tid]) + sm[3][tid];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kRedBlock) void k_reduce(int nblk, const double *partial, int ldp, double *h,
                                                      double *H, int hmode) {
    __shared__ double red[4];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kRedBlock) s += partial[(long)b * ldp + k];
    s = block_sum256(s, red);
    if (threadIdx.x == 0) {
        if (h) h[k] = s;
        if (hmode == 1)
            H[k] = s;
        else if (hmode == 2)
            H[k] += s;
    }
}

template <typename XT>
__global__ __launch_bounds__(256) void k_update(int n, const XT *V, long ldv, int ncols, const double *h, XT *w,
                                                double *norm_partial) {
    __shared__ double red[4];
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    double sq = 0.0;
    if (i < n) {
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
        int k = 0;
        for (; k + 4 <= ncols; k += 4) {
            acc0 += (double)ldx(V, i + (long)k * ldv) * h[k];
            acc1 += (double)ldx(V, i + (long)(k + 1) * ldv) * h[k + 1];
            acc2 += (double)ldx(V, i + (long)(k + 2) * ldv) * h[k + 2];
            acc3 += (double)ldx(V, i + (long)(k + 3) * ldv) * h[k + 3];
        }
        for (; k < ncols; ++k) acc0 += (double)ldx(V, i + (long)k * ldv) * h[k];
        const double wn = (double)ldx(w, i) - ((acc0 + acc1) + (acc2 + acc3));
        stx(w, i, (typename Arith<XT>::T)wn);
        const double stored = stored_value(w, wn);
        sq = stored * stored;
    }
    if (norm_partial) {
        sq = block_sum256(sq, red);
        if (threadIdx.x == 0) norm_partial[blockIdx.x] = sq;
    }
}

__global__ __launch_bounds__(kRedBlock) void k_reduce_norm(int nblk, const double *partial, double *H,
                                                           double *inv) {
    __shared__ double red[4];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kRedBlock) s += partial[b];
    s = block_sum256(s, red);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(s);
        if (H) H[0] = nrm;
        if (inv) inv[0] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    }
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_scale_cast(int n, const TI *in, const double *scale, double scale_host,
                                                    TO *out) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const double v = (double)ldx(in, i) * (scale ? scale[0] : scale_host);
        stx(out, i, (typename Arith<TO>::T)v);
    }
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_convert(int n, const TI *in, TO *out) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) stx(out, i, (typename Arith<TO>::T)ldx(in, i));
}

template <typename XT>
__global__ __launch_bounds__(256) void k_combine(int n, const XT *V, long ldv, int k, const double *z, XT *out) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double acc0 = 0.0, acc1 = 0.0;
    int j = 0;
    for (; j + 2 <= k; j += 2) {
        acc0 += (double)ldx(V, i + (long)j * ldv) * z[j];
        acc1 += (double)ldx(V, i + (long)(j + 1) * ldv) * z[j + 1];
    }
    if (j < k) acc0 += (double)ldx(V, i + (long)j * ldv) * z[j];
    stx(out, i, (typename Arith<XT>::T)(acc0 + acc1));
}

template <typename XT>
__global__ __launch_bounds__(256) void k_axpy_x(int n, double beta, const XT *d, double *x) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] += beta * (double)ldx(d, i);
}

__global__ __launch_bounds__(256) void k_fill(int n, double value, double *x) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = value;
}

__global__ __launch_bounds__(256) void k_val_to_f32(int nnz, const double *v, float *o) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < nnz) o[i] = (float)v[i];
}

__global__ __launch_bounds__(256) void k_gather(int nnz, const double *in, const int32_t *perm, double *out) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < nnz) out[i] = in[perm[i]];
}

__global__ __launch_bounds__(256) void k_adjoint_values(int n, const int32_t *rowptr, const int32_t *colind,
                                                        const double *lam, const double *x, double *dval) {
    const long r = (long)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    const double l = lam[r];
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) dval[e] = -l * x[colind[e]];
}

inline unsigned blocks_for(long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

size_t elem_size(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }

hipError_t launch_chain_step(const DevCSR &A, int prec, const StepPtrs &s, hipStream_t st) {
    switch (prec) {
        case 0:
            return chain_launch<double, double>(A, A.val64, s, st);
        case 1:
            return chain_launch<float, float>(A, A.val32, s, st);
        case 2:
            return chain_launch<float, uint16_t>(A, A.val32, s, st);
    }
    return hipErrorInvalidValue;
}

int dot_blocks(int n) { return (int)blocks_for(n, kDotRows); }

hipError_t launch_dots(int prec, int n, const void *V, long ldv, int ncols, const void *w, double *partial, int ldp,
                       hipStream_t st) {
    const unsigned g = blocks_for(n, kDotRows);
    if (g == 0 || ncols == 0) return hipSuccess;
    switch (prec) {
        case 0:
            hipLaunchKernelGGL(k_dots<double>, dim3(g), dim3(256), 0, st, n, (const double *)V, ldv, ncols,
                               (const double *)w, partial, ldp);
            break;
        case 1:
            hipLaunchKernelGGL(k_dots<float>, dim3(g), dim3(256), 0, st, n, (const float *)V, ldv, ncols,
                               (const float *)w, partial, ldp);
            break;
        case 2:
            hipLaunchKernelGGL(k_dots<uint16_t>, dim3(g), dim3(256), 0, st, n, (const uint16_t *)V, ldv, ncols,
                               (const uint16_t *)w, partial, ldp);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce(int nblk, const double *partial, int ldp, int ncols, double *h, double *H, int hmode,
                         hipStream_t st) {
    if (ncols == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(ncols), dim3(kRedBlock), 0, st, nblk, partial, ldp, h, H, hmode);
    return hipGetLastError();
}

hipError_t launch_update(int prec, int n, const void *V, long ldv, int ncols, const double *h, void *w,
                         double *norm_partial, hipStream_t st) {
    const unsigned g = blocks_for(n, 256);
    if (g == 0) return hipSuccess;
    switch (prec) {
        case 0:
            hipLaunchKernelGGL(k_update<double>, dim3(g), dim3(256), 0, st, n, (const double *)V, ldv, ncols, h,
                               (double *)w, norm_partial);
            break;
        case 1:
            hipLaunchKernelGGL(k_update<float>, dim3(g), dim3(256), 0, st, n, (const float *)V, ldv, ncols, h,
                               (float *)w, norm_partial);
            break;
        case 2:
            hipLaunchKernelGGL(k_update<uint16_t>, dim3(g), dim3(256), 0, st, n, (const uint16_t *)V, ldv, ncols,
                               h, (uint16_t *)w, norm_partial);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_norm(int nblk, const double *partial, double *H, double *inv, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_norm, dim3(1), dim3(kRedBlock), 0, st, nblk, partial, H, inv);
    return hipGetLastError();
}

template <typename TI>
static hipError_t scale_cast_to(int prec_out, int n, const TI *in, const double *scale, double scale_host, void *out,
                                hipStream_t st) {
    const unsigned g = blocks_for(n, 256);
    if (g == 0) return hipSuccess;
    switch (prec_out) {
        case 0:
            hipLaunchKernelGGL((k_scale_cast<TI, double>), dim3(g), dim3(256), 0, st, n, in, scale, scale_host, (double *)out);
            break;
        case 1:
            hipLaunchKernelGGL((k_scale_cast<TI, float>), dim3(g), dim3(256), 0, st, n, in, scale, scale_host, (float *)out);
            break;
        case 2:
            hipLaunchKernelGGL((k_scale_cast<TI, uint16_t>), dim3(g), dim3(256), 0, st, n, in, scale, scale_host,
                               (uint16_t *)out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_scale_cast(int prec_in, int prec_out, int n, const void *in, const double *scale, double scale_host,
                             void *out, hipStream_t st) {
    switch (prec_in) {
        case 0:
            return scale_cast_to<double>(prec_out, n, (const double *)in, scale, scale_host, out, st);
        case 1:
            return scale_cast_to<float>(prec_out, n, (const float *)in, scale, scale_host, out, st);
        case 2:
            return scale_cast_to<uint16_t>(prec_out, n, (const uint16_t *)in, scale, scale_host, out, st);
    }
    return hipErrorInvalidValue;
}

template <typename TI>
static hipError_t convert_to(int prec_out, int n, const TI *in, void *out, hipStream_t st) {
    const unsigned g = blocks_for(n, 256);
    if (g == 0) return hipSuccess;
    switch (prec_out) {
        case 0:
            hipLaunchKernelGGL((k_convert<TI, double>), dim3(g), dim3(256), 0, st, n, in, (double *)out);
            break;
        case 1:
            hipLaunchKernelGGL((k_convert<TI, float>), dim3(g), dim3(256), 0, st, n, in, (float *)out);
            break;
        case 2:
            hipLaunchKernelGGL((k_convert<TI, uint16_t>), dim3(g), dim3(256), 0, st, n, in, (uint16_t *)out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_convert(int prec_in, int prec_out, int n, const void *in, void *out, hipStream_t st) {
    switch (prec_in) {
        case 0:
            return convert_to<double>(prec_out, n, (const double *)in, out, st);
        case 1:
            return convert_to<float>(prec_out, n, (const float *)in, out, st);
        case 2:
            return convert_to<uint16_t>(prec_out, n, (const uint16_t *)in, out, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_combine(int prec, int n, const void *V, long ldv, int k, const double *z, void *out,
                          hipStream_t st) {
    const unsigned g = blocks_for(n, 256);
    if (g == 0) return hipSuccess;
    switch (prec) {
        case 0:
            hipLaunchKernelGGL(k_combine<double>, dim3(g), dim3(256), 0, st, n, (const double *)V, ldv, k, z,
                               (double *)out);
            break;
        case 1:
            hipLaunchKernelGGL(k_combine<float>, dim3(g), dim3(256), 0, st, n, (const float *)V, ldv, k, z,
                               (float *)out);
            break;
        case 2:
            hipLaunchKernelGGL(k_combine<uint16_t>, dim3(g), dim3(256), 0, st, n, (const uint16_t *)V, ldv, k, z,
                               (uint16_t *)out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_axpy_x(int prec, int n, double beta, const void *d, double *x, hipStream_t st) {
    const unsigned g = blocks_for(n, 256);
    if (g == 0) return hipSuccess;
    switch (prec) {
        case 0:
            hipLaunchKernelGGL(k_axpy_x<double>, dim3(g), dim3(256), 0, st, n, beta, (const double *)d, x);
            break;
        case 1:
            hipLaunchKernelGGL(k_axpy_x<float>, dim3(g), dim3(256), 0, st, n, beta, (const float *)d, x);
            break;
        case 2:
            hipLaunchKernelGGL(k_axpy_x<uint16_t>, dim3(g), dim3(256), 0, st, n, beta, (const uint16_t *)d, x);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fill(int n, double value, double *x, hipStream_t st) {
    const unsigned g = blocks_for(n, 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(g), dim3(256), 0, st, n, value, x);
    return hipGetLastError();
}

hipError_t launch_val_to_f32(int nnz, const double *val64, float *val32, hipStream_t st) {
    const unsigned g = blocks_for(nnz, 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_val_to_f32, dim3(g), dim3(256), 0, st, nnz, val64, val32);
    return hipGetLastError();
}

hipError_t launch_gather(int nnz, const double *in, const int32_t *perm, double *out, hipStream_t st) {
    const unsigned g = blocks_for(nnz, 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(256), 0, st, nnz, in, perm, out);
    return hipGetLastError();
}

hipError_t launch_adjoint_values(const DevCSR &A, const double *lam, const double *x, double *dval, hipStream_t st) {
    const unsigned g = blocks_for(A.n, 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adjoint_values, dim3(g), dim3(256), 0, st, A.n, A.rowptr, A.colind, lam, x, dval);
    return hipGetLastError();
}

}  // namespace ppg
