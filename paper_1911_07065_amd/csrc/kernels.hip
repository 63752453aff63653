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
#include <cstring>
#include <type_traits>

#include "devutil.h"
#include "kernels.h"

namespace ppg {
namespace {

// ---------------------------------------------------------------------------
// fused chain step
//
// Every launch computes, for each row r,
//     w = a0 (A in)_r + a1 in_r + a2 aux_r
//     acc_r = (acc_init ? 0 : acc_r) + b0 in_r + b1 w      (if acc)
//     out_r = fin ? vfin_r - w : w                          (if out)
// which covers one factor of Algorithm 1 or 3 (see poly.cpp). Several kernel
// families compute (A in)_r, each on its own copy of the matrix; the
// autotuner picks one per matrix and precision:
//  * tile (CSR): a workgroup owns a tile of <= 256*RPT rows holding
//    <= 256*EPT stored entries; the entries are streamed with coalesced
//    loads, the products staged in LDS and summed per row. Row data of the
//    epilogue is prefetched before the stream so that it overlaps it. The
//    column-banded variants run it once per band of columns.
//  * vec (CSR): LPR lanes per row, U rows in flight per lane group, sums
//    reduced with cross-lane shuffles; no LDS and no barrier.
//  * sliced-ELL: one lane per row of a 64-row slice, entries stored column
//    by column (32-bit columns or 16-bit offsets).
//  * diagonal formats (matrices on few diagonals): stored values per
//    diagonal, 1-byte codes into the distinct values, or 1 byte per row
//    naming its pattern among the distinct rows; the gather is x[r + off].
//  * persistent: a whole chain in one cooperative launch (opt-in).
// ---------------------------------------------------------------------------

template <typename VT, typename XT>
struct ChainArgs {
    const int32_t *rowptr;
    const int32_t *colind;
    const VT *val;
    const XT *in;
    const XT *aux;
    const XT *vfin;
    XT *out;
    XT *acc;
    typename Arith<XT>::T a0, a1, a2, b0, b1;
    int acc_init;
    int n;
    // banded products (kernels compiled with BAND): add pin[r] to the row's
    // sum; with pout, store the sum there instead of finishing the row
    const typename Arith<XT>::T *pin;
    typename Arith<XT>::T *pout;
};

template <typename AT>
struct RowPre {
    AT xin, aux, vf, acc;
};

// BAND: a kernel that may run one band of a column-banded product (pin,
// pout); the other kernels are compiled without those tests
template <typename VT, typename XT, bool BAND = false>
__device__ __forceinline__ RowPre<typename Arith<XT>::T> row_prefetch(const ChainArgs<VT, XT> &a, int r) {
    using AT = typename Arith<XT>::T;
    RowPre<AT> p;
    if constexpr (BAND) {
        if (a.pout) {  // a partial pass reads nothing but its entries
            p.xin = p.aux = p.vf = p.acc = AT(0);
            return p;
        }
    }
    p.xin = ldx(a.in, r);
    p.aux = a.aux ? (AT)ldx(a.aux, r) : AT(0);
    p.vf = a.vfin ? (AT)ldx(a.vfin, r) : AT(0);
    p.acc = (a.acc && !a.acc_init) ? (AT)ldx(a.acc, r) : AT(0);
    return p;
}

template <typename VT, typename XT, bool BAND = false>
__device__ __forceinline__ void row_finish(const ChainArgs<VT, XT> &a, int r, typename Arith<XT>::T s,
                                           const RowPre<typename Arith<XT>::T> &p) {
    using AT = typename Arith<XT>::T;
    if constexpr (BAND) {
        if (a.pin) s += a.pin[r];
        if (a.pout) {
            a.pout[r] = s;
            return;
        }
    }
    AT w = a.a0 * s + a.a1 * p.xin;
    if (a.aux) w += a.a2 * p.aux;
    if (a.acc) stx(a.acc, r, p.acc + a.b0 * p.xin + a.b1 * w);
    if (a.out) stx(a.out, r, a.vfin ? p.vf - w : w);
}

// steps without a sparse product: the product term is a0 * prod[r] when a
// product vector is given (a composite polynomial's outer step, whose
// operator was applied by another chain), else zero
template <typename VT, typename XT>
__global__ __launch_bounds__(256) void k_chain_elem(ChainArgs<VT, XT> a, const XT *prod) {
    using AT = typename Arith<XT>::T;
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < a.n) row_finish(a, r, prod ? (AT)ldx(prod, r) : AT(0), row_prefetch(a, r));
}

// One row tile of a chain step (r0, r1, e0, e1 in ti); buf: LDS of 256*EPT
// entries, red: LDS of 4. With spmv == 0 only the epilogue runs.
template <typename VT, typename XT, int EPT, int RPT, bool BAND = false>
__device__ __forceinline__ void tile_body(const ChainArgs<VT, XT> &a, const int4 ti, int spmv,
                                          typename Arith<XT>::T *buf, typename Arith<XT>::T *red) {
    using AT = typename Arith<XT>::T;
    constexpr int TILE = 256 * EPT;
    const int r0 = ti.x, r1 = ti.y, e0 = ti.z, e1 = ti.w;
    const int tid = threadIdx.x;
    if (!spmv) {
        for (int r = r0 + tid; r < r1; r += 256) row_finish<VT, XT, BAND>(a, r, AT(0), row_prefetch<VT, XT, BAND>(a, r));
        return;
    }
    if (e1 - e0 <= TILE) {
        int rs[RPT], rl[RPT];
        RowPre<AT> pre[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = r0 + tid + q * 256;
            rs[q] = 0;
            rl[q] = 0;
            if (r < r1) {
                rs[q] = a.rowptr[r] - e0;
                rl[q] = a.rowptr[r + 1] - e0;
                pre[q] = row_prefetch<VT, XT, BAND>(a, r);
            }
        }
        int col[EPT];
        VT v[EPT];
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = e0 + k * 256 + tid;
            col[k] = 0;
            v[k] = VT(0);
            if (e < e1) {
                col[k] = a.colind[e];
                v[k] = a.val[e];
            }
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const int e = e0 + k * 256 + tid;
            if (e < e1) buf[k * 256 + tid] = (AT)v[k] * ldx(a.in, col[k]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = r0 + tid + q * 256;
            if (r < r1) {
                AT s = AT(0);
                for (int k = rs[q]; k < rl[q]; ++k) s += buf[k];
                row_finish<VT, XT, BAND>(a, r, s, pre[q]);
            }
        }
    } else {
        // a tile holding one row longer than the tile capacity
        AT s = AT(0);
        for (int e = e0 + tid; e < e1; e += 256) s += (AT)a.val[e] * ldx(a.in, a.colind[e]);
        s = block_sum256(s, red);
        if (tid == 0) row_finish<VT, XT, BAND>(a, r0, s, row_prefetch<VT, XT, BAND>(a, r0));
    }
}

template <typename VT, typename XT, int EPT, int RPT, bool BAND = false>
__global__ __launch_bounds__(256) void k_chain_tile(ChainArgs<VT, XT> a, const int4 *__restrict__ tinfo, int ntiles,
                                                    int remap) {
    using AT = typename Arith<XT>::T;
    __shared__ AT buf[256 * EPT];
    __shared__ AT red[4];
    const int t = remap_tile(blockIdx.x, ntiles, remap);
    tile_body<VT, XT, EPT, RPT, BAND>(a, tinfo[t], 1, buf, red);
}

// ---------------------------------------------------------------------------
// persistent chain: all steps of a program in one cooperative launch
//
// Every workgroup owns a fixed contiguous range of row tiles (balanced in
// stored entries) and runs each step of the program over it; consecutive
// steps are separated by a grid-wide barrier (the next step gathers rows
// written by other workgroups). The barrier counter only grows: the host
// passes the value it had before the launch. A barrier that does not
// complete within a bounded number of polls sets *err and lets the kernel
// run to its end, so every wave exits.
// ---------------------------------------------------------------------------

template <typename VT, typename XT>
struct PArgs {
    const int32_t *rowptr;
    const int32_t *colind;
    const VT *val;
    const int4 *tiles;
    int ntiles;
    int n;
    XT *bufs[5];
    const PStep *steps;
    int nsteps;
    int remap;
    unsigned long long *bar;
    unsigned long long bar_base;
    int *err;
};

__device__ __forceinline__ void grid_barrier(unsigned long long *bar, unsigned long long target, int *err) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            // bounded wait (~0.2 s); after a timeout every later barrier of
            // the launch returns at once
            if (++spins > (1u << 23) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <typename VT, typename XT, int EPT>
__global__ __launch_bounds__(256) void k_chain_persist(PArgs<VT, XT> p) {
    using AT = typename Arith<XT>::T;
    __shared__ AT buf[256 * EPT];
    __shared__ AT red[4];
    const int G = gridDim.x;
    const int w = remap_tile(blockIdx.x, G, p.remap);
    const int t0 = (int)((long)w * p.ntiles / G), t1 = (int)((long)(w + 1) * p.ntiles / G);
    for (int s = 0; s < p.nsteps; ++s) {
        const PStep st = p.steps[s];
        ChainArgs<VT, XT> a;
        a.rowptr = p.rowptr;
        a.colind = p.colind;
        a.val = p.val;
        a.in = p.bufs[st.in];
        a.aux = st.aux >= 0 ? p.bufs[st.aux] : nullptr;
        a.vfin = st.fin ? p.bufs[0] : nullptr;
        a.out = st.out >= 0 ? p.bufs[st.out] : nullptr;
        a.acc = st.acc >= 0 ? p.bufs[st.acc] : nullptr;
        a.a0 = (AT)st.a0;
        a.a1 = (AT)st.a1;
        a.a2 = (AT)st.a2;
        a.b0 = (AT)st.b0;
        a.b1 = (AT)st.b1;
        a.acc_init = st.acc_init;
        a.n = p.n;
        a.pin = nullptr;
        a.pout = nullptr;
        for (int t = t0; t < t1; ++t) {
            tile_body<VT, XT, EPT, 1>(a, p.tiles[t], st.spmv, buf, red);
            __syncthreads();
        }
        if (s + 1 < p.nsteps) grid_barrier(p.bar, p.bar_base + (unsigned long long)(s + 1) * G, p.err);
    }
}

// 16-byte non-temporal loads of 4 consecutive stored entries (streamed once
// per launch: kept out of the way of the gathered input vector in L2)
typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void load4(const int32_t *p, int *c) {
    const v4i q = __builtin_nontemporal_load((const v4i *)p);
    c[0] = q.x;
    c[1] = q.y;
    c[2] = q.z;
    c[3] = q.w;
}
__device__ __forceinline__ void load4(const float *p, float *v) {
    const v4f q = __builtin_nontemporal_load((const v4f *)p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
}
__device__ __forceinline__ void load4(const double *p, double *v) {
    const v2d a = __builtin_nontemporal_load((const v2d *)p);
    const v2d b = __builtin_nontemporal_load((const v2d *)p + 1);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
}

// Tile kernel with 16-byte streaming loads: the tile's entries are read in
// aligned chunks of 4 from e0 rounded down to a multiple of 4 (entries of
// the neighbouring tiles in the first/last chunk are masked out). A chunk
// that would cross the end of the arrays is read element by element.
template <typename VT, typename XT, int EPT, int RPT>
__global__ __launch_bounds__(256) void k_chain_tilev(ChainArgs<VT, XT> a, const int4 *__restrict__ tinfo, int ntiles,
                                                     int remap, int nnz) {
    using AT = typename Arith<XT>::T;
    constexpr int TILE = 256 * EPT;
    constexpr int CH = EPT / 4;  // chunks of 4 per thread
    __shared__ AT buf[TILE];
    __shared__ AT red[4];
    const int t = remap_tile(blockIdx.x, ntiles, remap);
    const int4 ti = tinfo[t];
    const int r0 = ti.x, r1 = ti.y, e0 = ti.z, e1 = ti.w;
    const int ea = e0 & ~3;
    const int tid = threadIdx.x;
    if (e1 - ea <= TILE) {
        int rs[RPT], rl[RPT];
        RowPre<AT> pre[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = r0 + tid + q * 256;
            rs[q] = 0;
            rl[q] = 0;
            if (r < r1) {
                rs[q] = a.rowptr[r] - ea;
                rl[q] = a.rowptr[r + 1] - ea;
                pre[q] = row_prefetch(a, r);
            }
        }
        int col[CH][4];
        VT v[CH][4];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int c = ea + (k * 256 + tid) * 4;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                col[k][j] = 0;
                v[k][j] = VT(0);
            }
            if (c < e1) {
                if (c + 4 <= nnz) {
                    load4(a.colind + c, col[k]);
                    load4(a.val + c, v[k]);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (c + j < nnz) {
                            col[k][j] = a.colind[c + j];
                            v[k][j] = a.val[c + j];
                        }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int c = ea + (k * 256 + tid) * 4;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = c + j;
                if (e >= e0 && e < e1) buf[e - ea] = (AT)v[k][j] * ldx(a.in, col[k][j]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = r0 + tid + q * 256;
            if (r < r1) {
                AT s = AT(0);
                for (int k = rs[q]; k < rl[q]; ++k) s += buf[k];
                row_finish(a, r, s, pre[q]);
            }
        }
    } else {
        AT s = AT(0);
        for (int e = e0 + tid; e < e1; e += 256) s += (AT)a.val[e] * ldx(a.in, a.colind[e]);
        s = block_sum256(s, red);
        if (tid == 0) row_finish(a, r0, s, row_prefetch(a, r0));
    }
}

// LPR lanes per row, U rows per lane group, K entries per lane loaded in
// one batch (rows longer than LPR*K finish in a loop).
template <typename VT, typename XT, int LPR, int U, int K>
__global__ __launch_bounds__(256) void k_chain_vk(ChainArgs<VT, XT> a, int nblocks, int remap) {
    using AT = typename Arith<XT>::T;
    constexpr int GPW = 64 / LPR;
    constexpr int RPW = GPW * U;
    const int blk = remap_tile(blockIdx.x, nblocks, remap);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / LPR, l = lane % LPR;
    const int base = (blk * 4 + wave) * RPW + g;
    int e0[U], e1[U];
    RowPre<AT> pre[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = base + u * GPW;
        e0[u] = 0;
        e1[u] = 0;
        if (r < a.n) {
            e0[u] = a.rowptr[r];
            e1[u] = a.rowptr[r + 1];
            if (l == 0) pre[u] = row_prefetch(a, r);
        }
    }
    int col[U][K];
    VT v[U][K];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = e0[u] + l + k * LPR;
            col[u][k] = 0;
            v[u][k] = VT(0);
            if (e < e1[u]) {
                col[u][k] = __builtin_nontemporal_load(a.colind + e);
                v[u][k] = __builtin_nontemporal_load(a.val + e);
            }
        }
    AT s[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        s[u] = AT(0);
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (e0[u] + l + k * LPR < e1[u]) s[u] += (AT)v[u][k] * ldx(a.in, col[u][k]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
        for (int e = e0[u] + l + K * LPR; e < e1[u]; e += LPR) s[u] += (AT)a.val[e] * ldx(a.in, a.colind[e]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int off = LPR / 2; off > 0; off >>= 1) s[u] += __shfl_xor(s[u], off, 64);
    }
    if (l == 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = base + u * GPW;
            if (r < a.n) row_finish(a, r, s[u], pre[u]);
        }
    }
}

template <typename VT, typename XT, int LPR, int U>
__global__ __launch_bounds__(256) void k_chain_vec(ChainArgs<VT, XT> a, int nblocks, int remap) {
    using AT = typename Arith<XT>::T;
    constexpr int GPW = 64 / LPR;  // row groups per wave
    constexpr int RPW = GPW * U;   // rows per wave
    const int blk = remap_tile(blockIdx.x, nblocks, remap);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / LPR, l = lane % LPR;
    const int base = (blk * 4 + wave) * RPW + g;
    int e0[U], e1[U];
    RowPre<AT> pre[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = base + u * GPW;
        e0[u] = 0;
        e1[u] = 0;
        if (r < a.n) {
            e0[u] = a.rowptr[r];
            e1[u] = a.rowptr[r + 1];
            if (l == 0) pre[u] = row_prefetch(a, r);
        }
    }
    int col[U];
    VT v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int e = e0[u] + l;
        col[u] = 0;
        v[u] = VT(0);
        if (e < e1[u]) {
            col[u] = a.colind[e];
            v[u] = a.val[e];
        }
    }
    AT s[U];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = (e0[u] + l < e1[u]) ? (AT)v[u] * ldx(a.in, col[u]) : AT(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
        for (int e = e0[u] + l + LPR; e < e1[u]; e += LPR) s[u] += (AT)a.val[e] * ldx(a.in, a.colind[e]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int off = LPR / 2; off > 0; off >>= 1) s[u] += __shfl_xor(s[u], off, 64);
    }
    if (l == 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = base + u * GPW;
            if (r < a.n) row_finish(a, r, s[u], pre[u]);
        }
    }
}

// Sliced ELL: wave w handles slice w (64 rows, lane j -> row 64 w + j). The
// k-th entries of the slice's rows are contiguous, so the index and value
// loads are coalesced and, for stencil-like matrices, so is the gather of
// the input (neighbouring rows have neighbouring columns). Entries are
// consumed 8 at a time (loads issued together).
template <typename T>
__device__ __forceinline__ T stream_load(const T *p, bool nt) {
    return nt ? __builtin_nontemporal_load(p) : *p;
}

// One 64-row slice of a sliced-ELL matrix; lane j owns row 64 w + j. Entries
// are consumed 8 at a time: all 16 loads of a block are issued before the
// first is used (positions past the slice width re-read its last column and
// are dropped by a select, so no load sits behind a branch). IT = int32_t:
// the index is the column; IT = int16_t: the index is column - row (rows
// past n store 0 relative to row 0).
template <typename VT, typename XT, bool NT, typename IT>
__device__ __forceinline__ void sell_slice(const ChainArgs<VT, XT> &a, const int32_t *__restrict__ sptr,
                                           const IT *__restrict__ sidx, const VT *__restrict__ sval, int w,
                                           int lane) {
    using AT = typename Arith<XT>::T;
    constexpr int U = 8;
    const int r = w * 64 + lane;
    const int base = (sizeof(IT) == 4 || r < a.n) ? r : 0;
    const int o0 = sptr[w];
    const int width = (sptr[w + 1] - o0) >> 6;
    RowPre<AT> pre;
    if (r < a.n) pre = row_prefetch(a, r);
    AT s = AT(0);
    for (int k0 = 0; k0 < width; k0 += U) {
        int c[U];
        VT v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int o = o0 + min(k0 + u, width - 1) * 64 + lane;
            const int id = (int)stream_load(sidx + o, NT);
            c[u] = sizeof(IT) == 4 ? id : base + id;
            v[u] = stream_load(sval + o, NT);
        }
        AT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = ldx(a.in, c[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const AT t = (AT)v[u] * xv[u];
            s += (k0 + u < width) ? t : AT(0);
        }
    }
    if (r < a.n) row_finish(a, r, s, pre);
}

// Sliced ELL: wave w handles SPW consecutive slices of 64 rows (lane j -> row
// 64 w' + j). The k-th entries of the slice's rows are contiguous, so the
// index and value loads are coalesced and, for stencil-like matrices, so is
// the gather of the input (neighbouring rows have neighbouring columns).
// With IT = int16_t the indices are 16-bit column offsets from the row, for
// matrices whose entries all lie within 32767 of the diagonal (banded,
// stencils): the entry stream shrinks from 4 + s_val to 2 + s_val bytes.
template <typename VT, typename XT, bool NT, int SPW, typename IT>
__global__ __launch_bounds__(256) void k_chain_sell(ChainArgs<VT, XT> a, const int32_t *__restrict__ sptr,
                                                    const IT *__restrict__ sidx, const VT *__restrict__ sval,
                                                    int nslices, int nblocks, int remap) {
    const int blk = remap_tile(blockIdx.x, nblocks, remap);
    const int lane = threadIdx.x & 63;
    const int w0 = (blk * 4 + (threadIdx.x >> 6)) * SPW;
#pragma unroll
    for (int q = 0; q < SPW; ++q)
        if (w0 + q < nslices) sell_slice<VT, XT, NT, IT>(a, sptr, sidx, sval, w0 + q, lane);
}

// Diagonal format: each lane owns RPT rows (256 apart); the diagonals are
// consumed DU at a time with every load of a block issued before the first
// is used. Diagonal positions past nd re-read the last diagonal and columns
// outside [0, n) read a clamped column; both carry a zero value or are
// dropped by a select. Values are stored per 256-row block, diagonal after
// diagonal (entry of row r on diagonal d at ((r/256) nd + d) 256 + r%256),
// so a workgroup streams contiguous memory; the gather is coalesced too:
// lane i reads x[i + off].
template <typename VT, typename XT, int RPT, int DU>
__global__ __launch_bounds__(256) void k_chain_dia(ChainArgs<VT, XT> a, const VT *__restrict__ dval, DiaOffsets doff,
                                                   int nblocks, int remap) {
    using AT = typename Arith<XT>::T;
    const int blk = remap_tile(blockIdx.x, nblocks, remap);
    const int base = blk * 256 * RPT + (int)threadIdx.x;
    const int n = a.n, nd = doff.nd;
    // 32-bit index math: n and the number of stored slots are below 2^31
    int rr[RPT], vb[RPT];
    AT s[RPT];
    RowPre<AT> pre[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = base + q * 256;
        rr[q] = r < n ? r : n - 1;
        vb[q] = (rr[q] >> 8) * nd * 256 + (rr[q] & 255);
        s[q] = AT(0);
        if (r < n) pre[q] = row_prefetch(a, r);
    }
    for (int d0 = 0; d0 < nd; d0 += DU) {
        VT v[DU][RPT];
        AT x[DU][RPT];
#pragma unroll
        for (int u = 0; u < DU; ++u) {
            const int d = min(d0 + u, nd - 1);
            const int off = doff.off[d];
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int c = min(max(rr[q] + off, 0), n - 1);
                v[u][q] = __builtin_nontemporal_load(dval + vb[q] + d * 256);
                x[u][q] = ldx(a.in, c);
            }
        }
#pragma unroll
        for (int u = 0; u < DU; ++u)
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const AT t = (AT)v[u][q] * x[u][q];
                s[q] += (d0 + u < nd) ? t : AT(0);
            }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = base + q * 256;
        if (r < n) row_finish(a, r, s[q], pre[q]);
    }
}

// Diagonal format with the diagonal count ND known at compile time (common
// stencils: 3, 5, 7, 9, 13, 19, 27): one row per lane, all 2 ND loads issued
// together, no clamp of the diagonal index and no select.
template <typename VT, typename XT, int ND>
__global__ __launch_bounds__(256) void k_chain_dia_nd(ChainArgs<VT, XT> a, const VT *__restrict__ dval, DiaOffsets doff,
                                                      int nblocks, int remap) {
    using AT = typename Arith<XT>::T;
    const int blk = remap_tile(blockIdx.x, nblocks, remap);
    const int r = blk * 256 + (int)threadIdx.x;
    const int n = a.n;
    const int rr = r < n ? r : n - 1;
    const int vb = (rr >> 8) * ND * 256 + (rr & 255);
    RowPre<AT> pre;
    if (r < n) pre = row_prefetch(a, r);
    VT v[ND];
    AT x[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        v[d] = __builtin_nontemporal_load(dval + vb + d * 256);
        x[d] = ldx(a.in, min(max(rr + doff.off[d], 0), n - 1));
    }
    AT s = AT(0);
#pragma unroll
    for (int d = 0; d < ND; ++d) s += (AT)v[d] * x[d];
    if (r < n) row_finish(a, r, s, pre);
}

// Value-coded diagonal format: as k_chain_dia_nd, but the entry of row r on
// diagonal d is the byte code dcode[(r G + d/8) 8 + d%8] into a table of the
// matrix's distinct values (staged in LDS), so a row's entries cost 8 bytes
// per 8 diagonals. Rows past n read row n - 1 and are not written.
template <typename VT, typename XT, int ND, int RPT>
__global__ __launch_bounds__(256) void k_chain_diac(ChainArgs<VT, XT> a, const uint8_t *__restrict__ dcode,
                                                    const VT *__restrict__ dtab, int ntab, DiaOffsets doff,
                                                    int nblocks, int remap) {
    using AT = typename Arith<XT>::T;
    constexpr int G = (ND + 7) / 8;
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __shared__ AT tab[256];
    const int blk = remap_tile(blockIdx.x, nblocks, remap);
    const int base = blk * 256 * RPT + (int)threadIdx.x;
    const int n = a.n;
    // the block's loads go out before the table is staged (it waits once)
    int rr[RPT];
    u32x2 cw[RPT][G];
    AT x[RPT][ND];
    RowPre<AT> pre[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = base + q * 256;
        rr[q] = r < n ? r : n - 1;
#pragma unroll
        for (int g = 0; g < G; ++g)
            cw[q][g] = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(dcode) + (long)rr[q] * G + g);
#pragma unroll
        for (int d = 0; d < ND; ++d) x[q][d] = ldx(a.in, min(max(rr[q] + doff.off[d], 0), n - 1));
        if (r < n) pre[q] = row_prefetch(a, r);
    }
    if ((int)threadIdx.x < ntab) tab[threadIdx.x] = (AT)dtab[threadIdx.x];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        AT s = AT(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const unsigned word = (d & 7) < 4 ? cw[q][d >> 3].x : cw[q][d >> 3].y;
            const unsigned code = (word >> (8 * (d & 3))) & 0xffu;
            s += tab[code] * x[q][d];
        }
        const int r = base + q * 256;
        if (r < n) row_finish(a, r, s, pre[q]);
    }
}

// Pattern-coded diagonal format: the ND entries of a row are one of the
// matrix's distinct row patterns (a constant-coefficient stencil on a box
// has one per boundary class), so a row costs one byte. Lane t of block b
// takes rows b*1024 + q*256 + t (q = 0..3), whose pattern ids are the bytes
// of pcode[b*256 + t]; the pattern table is staged in LDS. Rows past n read
// row n - 1 and are not written.
template <typename VT, typename XT, int ND>
__global__ __launch_bounds__(256) void k_chain_diap(ChainArgs<VT, XT> a, const uint32_t *__restrict__ pcode,
                                                    const VT *__restrict__ ptab, int nent, DiaOffsets doff,
                                                    int nblocks, int remap) {
    using AT = typename Arith<XT>::T;
    constexpr int RPT = 4;
    __shared__ AT tab[kMaxPatEntries];
    const int blk = remap_tile(blockIdx.x, nblocks, remap);
    const int base = blk * 256 * RPT + (int)threadIdx.x;
    const int n = a.n;
    const uint32_t pw = __builtin_nontemporal_load(pcode + (long)blk * 256 + threadIdx.x);
    int rr[RPT];
    AT x[RPT][ND];
    RowPre<AT> pre[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = base + q * 256;
        rr[q] = r < n ? r : n - 1;
#pragma unroll
        for (int d = 0; d < ND; ++d) x[q][d] = ldx(a.in, min(max(rr[q] + doff.off[d], 0), n - 1));
        if (r < n) pre[q] = row_prefetch(a, r);
    }
    for (int i = (int)threadIdx.x; i < nent; i += 256) tab[i] = (AT)ptab[i];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const AT *t = tab + ((pw >> (8 * q)) & 0xffu) * ND;
        AT s = AT(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) s += t[d] * x[q][d];
        const int r = base + q * 256;
        if (r < n) row_finish(a, r, s, pre[q]);
    }
}

// Four consecutive elements of a vector as one access; the pointer need only
// be aligned to its element (dword-aligned vector loads).
__device__ __forceinline__ double elem_in(double v) { return v; }
__device__ __forceinline__ float elem_in(float v) { return v; }
__device__ __forceinline__ float elem_in(uint16_t v) { return __uint_as_float(((uint32_t)v) << 16); }
__device__ __forceinline__ double elem_out(const double *, double v) { return v; }
__device__ __forceinline__ float elem_out(const float *, float v) { return v; }
__device__ __forceinline__ uint16_t elem_out(const uint16_t *, float v) { return f32_to_bf16(v); }

template <typename XT>
__device__ __forceinline__ void ld4(const XT *__restrict__ p, long i, typename Arith<XT>::T *o) {
    typedef XT V4 __attribute__((ext_vector_type(4), aligned(sizeof(XT))));
    const V4 v = *reinterpret_cast<const V4 *>(p + i);
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = elem_in(v[k]);
}

template <typename XT>
__device__ __forceinline__ void st4(XT *__restrict__ p, long i, const typename Arith<XT>::T *v) {
    typedef XT V4 __attribute__((ext_vector_type(4), aligned(sizeof(XT))));
    V4 t;
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = elem_out(p, v[k]);
    *reinterpret_cast<V4 *>(p + i) = t;
}

// Pattern-coded diagonal format with 4 consecutive rows per lane: lane t of
// block b owns rows r .. r+3, r = b*1024 + 4t, whose pattern ids are the
// bytes pbyte[r .. r+3] (one 4-byte load). In a block whose every window
// x[r + off .. r + off + 3] lies inside [0, n) (omin <= 0 <= omax bound the
// offsets), each diagonal's window, the row data and the results move as
// one vector access each; the blocks at the two ends of the matrix read
// element by element with clamped indices and write only rows below n.
template <typename VT, typename XT, int ND>
__global__ __launch_bounds__(256) void k_chain_diapv(ChainArgs<VT, XT> a, const uint8_t *__restrict__ pbyte,
                                                     const VT *__restrict__ ptab, int nent, DiaOffsets doff,
                                                     int omin, int omax, int nblocks, int remap) {
    using AT = typename Arith<XT>::T;
    __shared__ AT tab[kMaxPatEntries];
    const int blk = remap_tile(blockIdx.x, nblocks, remap);
    const int n = a.n;
    const long b0 = (long)blk * 1024;
    const int r = (int)b0 + 4 * (int)threadIdx.x;
    // (bfloat16 storage always reads element by element: its windows are
    // only 2-byte aligned)
    const bool inner = sizeof(XT) >= 4 && b0 + omin >= 0 && b0 + 1023 + omax <= (long)n - 1;
    const uint32_t pw = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(pbyte) + (r >> 2));
    AT x[ND][4], xin[4], aux[4], vf[4], acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) aux[k] = vf[k] = acc[k] = AT(0);
    if (inner) {
#pragma unroll
        for (int d = 0; d < ND; ++d) ld4(a.in, (long)r + doff.off[d], x[d]);
        ld4(a.in, r, xin);
        if (a.aux) ld4(a.aux, r, aux);
        if (a.vfin) ld4(a.vfin, r, vf);
        if (a.acc && !a.acc_init) ld4(a.acc, r, acc);
    } else {
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
            for (int k = 0; k < 4; ++k) x[d][k] = ldx(a.in, min(max(r + k + doff.off[d], 0), n - 1));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int rk = min(r + k, n - 1);
            xin[k] = ldx(a.in, rk);
            if (a.aux) aux[k] = ldx(a.aux, rk);
            if (a.vfin) vf[k] = ldx(a.vfin, rk);
            if (a.acc && !a.acc_init) acc[k] = ldx(a.acc, rk);
        }
    }
    for (int i = (int)threadIdx.x; i < nent; i += 256) tab[i] = (AT)ptab[i];
    __syncthreads();
    AT ov[4], av[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const AT *t = tab + ((pw >> (8 * k)) & 0xffu) * ND;
        AT s = AT(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) s += t[d] * x[d][k];
        AT w = a.a0 * s + a.a1 * xin[k];
        if (a.aux) w += a.a2 * aux[k];
        av[k] = acc[k] + a.b0 * xin[k] + a.b1 * w;
        ov[k] = a.vfin ? vf[k] - w : w;
    }
    if (inner) {
        if (a.acc) st4(a.acc, r, av);
        if (a.out) st4(a.out, r, ov);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (r + k < n) {
                if (a.acc) stx(a.acc, r + k, av[k]);
                if (a.out) stx(a.out, r + k, ov[k]);
            }
    }
}

// Constant-coefficient box stencil (every row is the interior row's stencil
// truncated at the box, DevCSR::box_pint), one chain step with the update of
// the other chain kernels. The line length gx is a multiple of 4: lane t of
// block b owns the 4 points r .. r+3 of one grid line, r = 4 (256 b + t).
// Its own values and each neighbouring line's 4 values move as one vector
// access, the two neighbours along the line as single loads; no per-row
// matrix data is read. The ND coefficients (the interior row's pattern, a
// uniform load) multiply the neighbours in ascending diagonal order; a
// neighbour outside the box counts as zero, which is what the truncated row
// holds, so a row's sum has the pattern-coded kernels' terms in their order
// (the fused update may round differently by an ulp). Addresses of
// neighbours outside the box are clamped to the point itself and the loaded
// value is dropped, so every load of a lane goes out at once.
template <typename VT, typename XT, int ND>
__global__ __launch_bounds__(256) void k_chain_box(ChainArgs<VT, XT> a, const VT *__restrict__ ptab, int pint,
                                                   int gx, int gy, int gz, int nblocks, int remap) {
    using AT = typename Arith<XT>::T;
    static_assert(ND == 5 || ND == 7, "5- or 7-point box stencils");
    const int blk = remap_tile(blockIdx.x, nblocks, remap);
    const int n = a.n;
    const int r = 4 * (blk * 256 + (int)threadIdx.x);
    if (r >= n) return;
    const int P = gx * gy;
    const int x = r % gx, y = (r / gx) % gy, z = ND == 7 ? r / P : 0;
    AT c[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) c[d] = (AT)ptab[pint * ND + d];
    const bool hx0 = x > 0, hx1 = x + 4 < gx, hy0 = y > 0, hy1 = y + 1 < gy;
    const bool hz0 = ND == 7 && z > 0, hz1 = ND == 7 && z + 1 < gz;
    AT xc[4], ym[4], yp[4], zm[4], zp[4], aux[4], vf[4], acc[4];
    ld4(a.in, r, xc);
    ld4(a.in, hy0 ? r - gx : r, ym);
    ld4(a.in, hy1 ? r + gx : r, yp);
    if constexpr (ND == 7) {
        ld4(a.in, hz0 ? r - P : r, zm);
        ld4(a.in, hz1 ? r + P : r, zp);
    }
    AT xl = ldx(a.in, hx0 ? r - 1 : r), xr = ldx(a.in, hx1 ? r + 4 : r);
#pragma unroll
    for (int k = 0; k < 4; ++k) aux[k] = vf[k] = acc[k] = AT(0);
    if (a.aux) ld4(a.aux, r, aux);
    if (a.vfin) ld4(a.vfin, r, vf);
    if (a.acc && !a.acc_init) ld4(a.acc, r, acc);
    xl = hx0 ? xl : AT(0);
    xr = hx1 ? xr : AT(0);
    AT ov[4], av[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const AT left = k == 0 ? xl : xc[k - 1], right = k == 3 ? xr : xc[k + 1];
        AT s = AT(0);
        if constexpr (ND == 7) s += c[0] * (hz0 ? zm[k] : AT(0));
        constexpr int o = ND == 7 ? 1 : 0;
        s += c[o] * (hy0 ? ym[k] : AT(0));
        s += c[o + 1] * left;
        s += c[o + 2] * xc[k];
        s += c[o + 3] * right;
        s += c[o + 4] * (hy1 ? yp[k] : AT(0));
        if constexpr (ND == 7) s += c[6] * (hz1 ? zp[k] : AT(0));
        AT w = a.a0 * s + a.a1 * xc[k];
        if (a.aux) w += a.a2 * aux[k];
        av[k] = acc[k] + a.b0 * xc[k] + a.b1 * w;
        ov[k] = a.vfin ? vf[k] - w : w;
    }
    if (a.acc) st4(a.acc, r, av);
    if (a.out) st4(a.out, r, ov);
}

template <typename VT>
const VT *diap_tab(const DevCSR &A);
template <>
const double *diap_tab<double>(const DevCSR &A) {
    return A.ptab64;
}
template <>
const float *diap_tab<float>(const DevCSR &A) {
    return A.ptab32;
}

template <typename VT>
const VT *diac_tab(const DevCSR &A);
template <>
const double *diac_tab<double>(const DevCSR &A) {
    return A.dtab64;
}
template <>
const float *diac_tab<float>(const DevCSR &A) {
    return A.dtab32;
}

template <typename VT>
const VT *dia_vals(const DevCSR &A);
template <>
const double *dia_vals<double>(const DevCSR &A) {
    return A.dval64;
}
template <>
const float *dia_vals<float>(const DevCSR &A) {
    return A.dval32;
}

// ---------------------------------------------------------------------------
// column-sorted tiles (CV_CSORT4 / CV_CSORT2)
//
// On a matrix whose entries scatter over all columns, the 64 gathers of one
// wave of a CSR stream land on 64 different cache lines, and the L2 request
// rate, not HBM, bounds the product. Here the rows form blocks of kCsRows
// and the columns cs_nb bands; the entries of a (block, band) tile are
// stored sorted by column, so 64 consecutive entries of a tile span a narrow
// column range and share cache lines (a block of 8192 rows with 16 entries
// each: about 2 columns apart on average). The order of each row's sum
// stays fixed: a product goes to LDS at its slot (the entry's rank in
// row-major order) and every row adds its slots in order.
//
// k_chain_cs_tiles: a workgroup of 1024 threads takes G consecutive bands
// of one block, keeps its rows' running sums in registers (kCsRows / 1024
// rows per thread) and stores them as partial sum k of nsb = cs_nb / G.
// k_chain_cs_finish: per row, the diagonal product (when held apart), then
// the partial sums in band order, then the step's vector update.
// ---------------------------------------------------------------------------

constexpr int kCsThreads = 1024;
constexpr int kCsRPT = kCsRows / kCsThreads;

// DB (4-byte sums): two product areas in LDS; while the rows of band g add
// their slots from one, the gathers of band g+1 fill the other, and the
// workgroup meets once per band. 8-byte sums keep one area (its products
// fill the LDS budget): gather, meet, add, meet. Either way the words and
// values of band g+1 are loaded before band g's slots are added.
//
// WIDE: one workgroup per CU (up to 128 VGPRs): 8 entries in flight per
// thread with 8-byte sums too, slot ranges loaded one band ahead, and
// (FP64, BF16 storage) words two bands ahead.
template <typename VT, typename XT, bool WIDE>
__global__ __launch_bounds__(kCsThreads, WIDE ? 4 : 8) void k_chain_cs_tiles(
    const uint32_t *__restrict__ code, const VT *__restrict__ val, const int32_t *__restrict__ toff,
    const uint16_t *__restrict__ tptr, int nb, int sb, int W, int n, int G, int maxe, const XT *__restrict__ in,
    typename Arith<XT>::T *__restrict__ part, int remap) {
    using AT = typename Arith<XT>::T;
    constexpr bool DB = sizeof(AT) == 4;
    // entries in flight per thread (64 VGPRs; 128 when WIDE)
    constexpr int kCsUnroll = sizeof(AT) == 8 && !WIDE ? 4 : 8;
    // words two bands ahead (measured: FP32 storage one band ahead is faster)
    constexpr bool kAhead2 = WIDE && !std::is_same<XT, float>::value;
    extern __shared__ __align__(16) unsigned char cs_lds[];
    AT *prod0 = reinterpret_cast<AT *>(cs_lds);
    AT *prod1 = DB ? prod0 + maxe : prod0;
    const int nsb = nb / G;
    const int w = remap_tile(blockIdx.x, gridDim.x, remap);
    const int b = w / nsb, k = w - b * nsb;
    const int tid = threadIdx.x;
    const int r0 = b * kCsRows, rows = min(kCsRows, n - r0);
    const uint32_t mask = (1u << sb) - 1u;
    // first pass of band (k G + g): this thread's words and values
    auto load = [&](int g, uint32_t (&cd)[kCsUnroll], VT (&v)[kCsUnroll]) {
        const int t = b * nb + k * G + g;
        const int e1 = toff[t + 1];
#pragma unroll
        for (int u = 0; u < kCsUnroll; ++u) {
            const int ee = toff[t] + tid + u * kCsThreads;
            cd[u] = ee < e1 ? __builtin_nontemporal_load(code + ee) : 0u;
            v[u] = ee < e1 ? __builtin_nontemporal_load(val + ee) : VT(0);
        }
    };
    // the products of band (k G + g) into dst at their slots, the first
    // pass from words and values already loaded
    auto gather = [&](int g, AT *dst, uint32_t (&cd)[kCsUnroll], VT (&v)[kCsUnroll]) {
        const int band = k * G + g, t = b * nb + band;
        const int e0 = toff[t], e1 = toff[t + 1];
        const XT *xb = in + (long)band * W;
        // an empty tile reads nothing (its band may start past the last column)
        for (int e = e0 + tid; e < e1;) {
            AT xv[kCsUnroll];
#pragma unroll
            for (int u = 0; u < kCsUnroll; ++u) xv[u] = ldx(xb, (long)(cd[u] >> sb));
#pragma unroll
            for (int u = 0; u < kCsUnroll; ++u)
                if (e + u * kCsThreads < e1) dst[cd[u] & mask] = (AT)v[u] * xv[u];
            e += kCsThreads * kCsUnroll;
            if (e >= e1) break;
#pragma unroll
            for (int u = 0; u < kCsUnroll; ++u) {
                const int ee = e + u * kCsThreads;
                cd[u] = ee < e1 ? __builtin_nontemporal_load(code + ee) : 0u;
                v[u] = ee < e1 ? __builtin_nontemporal_load(val + ee) : VT(0);
            }
        }
    };
    AT acc[kCsRPT];
#pragma unroll
    for (int q = 0; q < kCsRPT; ++q) acc[q] = AT(0);
    // this thread's rows' first and end slots in tile (k G + g), two 16-bit
    // values per word
    auto load_span = [&](int g, uint32_t (&span)[kCsRPT]) {
        const uint16_t *tp = tptr + (size_t)(b * nb + k * G + g) * (kCsRows + 1);
#pragma unroll
        for (int q = 0; q < kCsRPT; ++q) {
            const int rl = tid + q * kCsThreads;
            span[q] = rl < rows ? (uint32_t)tp[rl] | ((uint32_t)tp[rl + 1] << 16) : 0u;
        }
    };
    // each row adds its slots of one band, in slot order
    auto add_slots = [&](const uint32_t (&span)[kCsRPT], const AT *src) {
#pragma unroll
        for (int q = 0; q < kCsRPT; ++q) {
            const int p0 = (int)(span[q] & 0xFFFFu), p1 = (int)(span[q] >> 16);
            AT s = acc[q];
            for (int j = p0; j < p1; ++j) s += src[j];
            acc[q] = s;
        }
    };
    using Words = uint32_t[kCsUnroll];
    using Vals = VT[kCsUnroll];
    using Span = uint32_t[kCsRPT];
    if constexpr (kAhead2) {
        // words two bands ahead, in two register sets that trade roles from
        // one band to the next (the band loop runs two bands per turn, so
        // no set is copied while its loads are in flight)
        Words cA, cB;
        Vals vA, vB;
        Span sA, sB;
        if constexpr (DB) {
            // turn g: the products of band g are in area g & 1, band g+1's
            // words in (cx, vx), set (cy, vy) free
            auto turn = [&](int g, Words &cx, Vals &vx, Words &cy, Vals &vy, const Span &sx, Span &sy) {
                if (g + 2 < G) load(g + 2, cy, vy);
                if (g + 1 < G) load_span(g + 1, sy);
                add_slots(sx, (g & 1) ? prod1 : prod0);
                if (g + 1 < G) gather(g + 1, (g & 1) ? prod0 : prod1, cx, vx);
                __syncthreads();
            };
            load(0, cA, vA);
            if (G > 1) load(1, cB, vB);
            load_span(0, sA);
            gather(0, prod0, cA, vA);
            __syncthreads();
            for (int g = 0; g < G; g += 2) {
                turn(g, cB, vB, cA, vA, sA, sB);
                if (g + 1 < G) turn(g + 1, cA, vA, cB, vB, sB, sA);
            }
        } else {
            // turn g: band g's words in (cx, vx), band g+1's in (cy, vy)
            auto turn = [&](int g, Words &cx, Vals &vx, Words &cy, Vals &vy, const Span &sx, Span &sy) {
                (void)cy;
                (void)vy;
                gather(g, prod0, cx, vx);
                __syncthreads();
                if (g + 2 < G) load(g + 2, cx, vx);
                if (g + 1 < G) load_span(g + 1, sy);
                add_slots(sx, prod0);
                __syncthreads();
            };
            load(0, cA, vA);
            if (G > 1) load(1, cB, vB);
            load_span(0, sA);
            for (int g = 0; g < G; g += 2) {
                turn(g, cA, vA, cB, vB, sA, sB);
                if (g + 1 < G) turn(g + 1, cB, vB, cA, vA, sB, sA);
            }
        }
    } else {
        Words cd;
        Vals v;
        load(0, cd, v);
        if constexpr (DB) {
            gather(0, prod0, cd, v);
            __syncthreads();
        }
        Span span;
        if constexpr (WIDE) load_span(0, span);
        for (int g = 0; g < G; ++g) {
            // slot ranges: loaded before the gathers so that they arrive
            // with them (WIDE: one band ahead, with the words)
            Span span_next;
            if constexpr (!WIDE) load_span(g, span);
            const AT *src = (g & 1) ? prod1 : prod0;
            if constexpr (!DB) {
                gather(g, prod0, cd, v);
                __syncthreads();
            }
            // the next band's words travel while this band's slots are added
            if (g + 1 < G) {
                load(g + 1, cd, v);
                if constexpr (WIDE) load_span(g + 1, span_next);
            }
            add_slots(span, src);
            if constexpr (DB) {
                if (g + 1 < G) gather(g + 1, (g & 1) ? prod0 : prod1, cd, v);
            }
            __syncthreads();
            if constexpr (WIDE) {
#pragma unroll
                for (int q = 0; q < kCsRPT; ++q) span[q] = span_next[q];
            }
        }
    }
    AT *pk = part + (size_t)k * n + r0;
#pragma unroll
    for (int q = 0; q < kCsRPT; ++q) {
        const int rl = tid + q * kCsThreads;
        if (rl < rows) pk[rl] = acc[q];
    }
}

template <typename VT, typename XT>
__global__ __launch_bounds__(256) void k_chain_cs_finish(ChainArgs<VT, XT> a, const VT *__restrict__ dg,
                                                         const typename Arith<XT>::T *__restrict__ part, int nsb) {
    using AT = typename Arith<XT>::T;
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= a.n) return;
    const RowPre<AT> p = row_prefetch(a, r);
    AT s = dg ? (AT)dg[r] * p.xin : AT(0);
    for (int k = 0; k < nsb; ++k) s += part[(size_t)k * a.n + r];
    row_finish(a, r, s, p);
}

template <typename VT>
const VT *cs_vals(const DevCSR &A);
template <>
const double *cs_vals<double>(const DevCSR &A) {
    return A.cs_val64;
}
template <>
const float *cs_vals<float>(const DevCSR &A) {
    return A.cs_val32;
}
template <typename VT>
const VT *cs_diag(const DevCSR &A);
template <>
const double *cs_diag<double>(const DevCSR &A) {
    return A.cs_dg64;
}
template <>
const float *cs_diag<float>(const DevCSR &A) {
    return A.cs_dg32;
}

// The tile launch of one column-sorted product (lds: its dynamic LDS bytes).
template <typename VT, typename XT, bool WIDE>
hipError_t cs_tiles_launch(const DevCSR &A, const ChainArgs<VT, XT> &a, int nsb, size_t lds, int remap,
                           hipStream_t st) {
    using AT = typename Arith<XT>::T;
    static bool attr_set = false;  // one per instantiation; the call is idempotent
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_chain_cs_tiles<VT, XT, WIDE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kCsLdsBytes);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int nblk = (A.n + kCsRows - 1) / kCsRows;
    hipLaunchKernelGGL((k_chain_cs_tiles<VT, XT, WIDE>), dim3(nblk * nsb), dim3(kCsThreads), lds, st, A.cs_code,
                       cs_vals<VT>(A), A.cs_toff, A.cs_tptr, A.cs_nb, A.cs_sb, A.cs_W, A.n, A.cs_nb / nsb, A.cs_maxe,
                       a.in, (AT *)A.cs_part, remap);
    return hipGetLastError();
}

// Both launches of one column-sorted product with `nsb` partial sums per
// row; two partial sums (half the workgroups) take the WIDE tile kernel.
template <typename VT, typename XT>
hipError_t cs_launch(const DevCSR &A, const ChainArgs<VT, XT> &a, int nsb, int remap, hipStream_t st) {
    using AT = typename Arith<XT>::T;
    if (A.cs_nb <= 0 || !A.cs_part || nsb < 1 || nsb > kCsMaxParts || A.cs_nb % nsb != 0) return hipErrorInvalidValue;
    // two product areas for 4-byte sums, one for 8-byte: within the bound
    // the copy is built for (a tile's FP64 products in kCsLdsBytes)
    const size_t lds = (size_t)A.cs_maxe * sizeof(AT) * (sizeof(AT) == 4 ? 2 : 1);
    if (lds > (size_t)kCsLdsBytes) return hipErrorInvalidValue;
    hipError_t e = nsb == 2 ? cs_tiles_launch<VT, XT, true>(A, a, nsb, lds, remap, st)
                            : cs_tiles_launch<VT, XT, false>(A, a, nsb, lds, remap, st);
    if (e != hipSuccess) return e;
    AT *part = (AT *)A.cs_part;
    hipLaunchKernelGGL((k_chain_cs_finish<VT, XT>), dim3((A.n + 255) / 256), dim3(256), 0, st, a, cs_diag<VT>(A), part,
                       nsb);
    return hipGetLastError();
}

template <typename VT>
const VT *band_vals(const DevCSR &A, int c);
template <>
const double *band_vals<double>(const DevCSR &A, int c) {
    return A.bval64[c];
}
template <>
const float *band_vals<float>(const DevCSR &A, int c) {
    return A.bval32[c];
}

template <typename VT>
const VT *sell_vals(const DevCSR &A);
template <>
const double *sell_vals<double>(const DevCSR &A) {
    return A.sval64;
}
template <>
const float *sell_vals<float>(const DevCSR &A) {
    return A.sval32;
}

// Two chain steps in one launch on a box-stencil matrix (see PairPtrs for
// the arithmetic). A workgroup owns a TX x TY x TZ tile of grid points: it
// stages the first step's input on the tile and two points around it in
// LDS (zero outside the box, where the matrix has no entries), computes w1
// on the tile and one point around it into LDS, then the second step on the
// tile from w1. Every row's entries come from the pattern-coded copy: one
// byte per row naming its pattern, whose ND entries (diagonals in ascending
// offset order) sit in a table staged in LDS.
template <typename XT>
struct PairArgs {
    const XT *in;
    XT *out;
    XT *acc;
    const XT *vfin;
    typename Arith<XT>::T a01, a11, b01, b11, a02, a12, a22, b02, b12;
    int acc1, acc2, init, aux2;
    int gx, gy, gz;
    int ntx, nty, ntiles;
};

// Offset of diagonal d (ascending order) in a staged region of row length
// LX and plane size LX * LY.
template <int ND, int LX, int LY>
__device__ constexpr int box_off(int d) {
    if constexpr (ND == 7) {
        return d == 0 ? -LX * LY : d == 1 ? -LX : d == 2 ? -1 : d == 3 ? 0 : d == 4 ? 1 : d == 5 ? LX : LX * LY;
    } else {
        return d == 0 ? -LX : d == 1 ? -1 : d == 2 ? 0 : d == 3 ? 1 : LX;
    }
}

template <typename VT, typename XT, int ND, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_chain_pair(PairArgs<XT> a, const uint8_t *__restrict__ pbyte,
                                                    const VT *__restrict__ ptab, int nent, int remap) {
    using AT = typename Arith<XT>::T;
    static_assert(ND == 5 || ND == 7, "5- or 7-point box stencils");
    constexpr int HZ = ND == 7 ? 1 : 0;  // a 2-D box has one plane
    static_assert(HZ == 1 || TZ == 1, "one plane per 2-D tile");
    constexpr int SX = TX + 4, SY = TY + 4, SZ = TZ + 4 * HZ;  // staged input
    constexpr int WX = TX + 2, WY = TY + 2, WZ = TZ + 2 * HZ;  // w1
    constexpr int NS = SX * SY * SZ, NW = WX * WY * WZ, NT = TX * TY * TZ;
    static_assert(NT % 256 == 0, "tiles of whole 256-point rounds");
    constexpr int CS = (NS + 255) / 256, CW = (NW + 255) / 256, CT = NT / 256;
    __shared__ AT xs[NS];
    __shared__ AT ws[NW];
    __shared__ AT tab[kMaxPatEntries];
    const int tid = threadIdx.x;
    const int t = remap_tile(blockIdx.x, a.ntiles, remap);
    const int x0 = (t % a.ntx) * TX, y0 = ((t / a.ntx) % a.nty) * TY, z0 = (t / (a.ntx * a.nty)) * TZ;
    const int gx = a.gx, gy = a.gy, gz = a.gz, pxy = gx * gy;
    // every global load goes out before the first barrier: the staged
    // input, the patterns of the w1 points, and the tile's patterns and row
    // data
    AT v[CS];
#pragma unroll
    for (int k = 0; k < CS; ++k) {
        const int c = tid + k * 256;
        const int lx = c % SX, ly = (c / SX) % SY, lz = c / (SX * SY);
        const int px = x0 - 2 + lx, py = y0 - 2 + ly, pz = z0 - 2 * HZ + lz;
        const bool ok = c < NS && px >= 0 && px < gx && py >= 0 && py < gy && pz >= 0 && pz < gz;
        v[k] = ok ? (AT)ldx(a.in, px + gx * py + pxy * pz) : AT(0);
    }
    int cw[CW];
#pragma unroll
    for (int k = 0; k < CW; ++k) {
        const int c = tid + k * 256;
        const int lx = c % WX, ly = (c / WX) % WY, lz = c / (WX * WY);
        const int px = x0 - 1 + lx, py = y0 - 1 + ly, pz = z0 - HZ + lz;
        const bool ok = c < NW && px >= 0 && px < gx && py >= 0 && py < gy && pz >= 0 && pz < gz;
        cw[k] = ok ? (int)pbyte[px + gx * py + pxy * pz] : -1;
    }
    int ct[CT], rt[CT];
    AT pa[CT], pf[CT];
    const bool load_acc = a.acc && !a.init;
#pragma unroll
    for (int k = 0; k < CT; ++k) {
        const int c = tid + k * 256;
        const int px = x0 + c % TX, py = y0 + (c / TX) % TY, pz = z0 + c / (TX * TY);
        const bool ok = px < gx && py < gy && pz < gz;
        const int r = px + gx * py + pxy * pz;
        rt[k] = ok ? r : -1;
        ct[k] = ok ? (int)pbyte[r] : 0;
        pa[k] = ok && load_acc ? (AT)ldx(a.acc, r) : AT(0);
        pf[k] = ok && a.vfin ? (AT)ldx(a.vfin, r) : AT(0);
    }
    for (int i = tid; i < nent; i += 256) tab[i] = (AT)ptab[i];
#pragma unroll
    for (int k = 0; k < CS; ++k) {
        const int c = tid + k * 256;
        if (c < NS) xs[c] = v[k];
    }
    __syncthreads();
    // the first step on the tile and one point around it (zero outside the box)
#pragma unroll
    for (int k = 0; k < CW; ++k) {
        const int c = tid + k * 256;
        if (c < NW) {
            AT w = AT(0);
            if (cw[k] >= 0) {
                const int lx = c % WX, ly = (c / WX) % WY, lz = c / (WX * WY);
                const int q = (lx + 1) + SX * ((ly + 1) + SY * (lz + HZ));
                const AT *tp = tab + cw[k] * ND;
                AT sum = AT(0);
#pragma unroll
                for (int d = 0; d < ND; ++d) sum += tp[d] * xs[q + box_off<ND, SX, SY>(d)];
                w = a.a01 * sum + a.a11 * xs[q];
            }
            ws[c] = w;
        }
    }
    __syncthreads();
    // the second step on the tile
#pragma unroll
    for (int k = 0; k < CT; ++k) {
        if (rt[k] < 0) continue;
        const int c = tid + k * 256;
        const int lx = c % TX, ly = (c / TX) % TY, lz = c / (TX * TY);
        const int q = (lx + 1) + WX * ((ly + 1) + WY * (lz + HZ));
        const int qs = (lx + 2) + SX * ((ly + 2) + SY * (lz + 2 * HZ));
        const AT *tp = tab + ct[k] * ND;
        AT sum = AT(0);
#pragma unroll
        for (int d = 0; d < ND; ++d) sum += tp[d] * ws[q + box_off<ND, WX, WY>(d)];
        const AT w1 = ws[q], xin = xs[qs];
        AT w2 = a.a02 * sum + a.a12 * w1;
        if (a.aux2) w2 += a.a22 * xin;
        if (a.acc) {
            AT cacc = pa[k];
            if (a.acc1) cacc = cacc + a.b01 * xin + a.b11 * w1;
            if (a.acc2) cacc = cacc + a.b02 * w1 + a.b12 * w2;
            stx(a.acc, rt[k], cacc);
        }
        if (a.out) stx(a.out, rt[k], a.vfin ? pf[k] - w2 : w2);
    }
}

template <typename VT, typename XT, int ND, int TX, int TY, int TZ>
hipError_t pair_launch(const DevCSR &A, const VT *ptab, const PairPtrs &p, int remap, hipStream_t st) {
    using AT = typename Arith<XT>::T;
    PairArgs<XT> a;
    a.in = (const XT *)p.in;
    a.out = (XT *)p.out;
    a.acc = (XT *)p.acc;
    a.vfin = (const XT *)p.vfin;
    a.a01 = (AT)p.a01;
    a.a11 = (AT)p.a11;
    a.b01 = (AT)p.b01;
    a.b11 = (AT)p.b11;
    a.a02 = (AT)p.a02;
    a.a12 = (AT)p.a12;
    a.a22 = (AT)p.a22;
    a.aux2 = p.aux2;
    a.b02 = (AT)p.b02;
    a.b12 = (AT)p.b12;
    a.acc1 = p.acc1;
    a.acc2 = p.acc2;
    a.init = p.init;
    a.gx = A.box[0];
    a.gy = A.box[1];
    a.gz = A.box[2];
    a.ntx = (a.gx + TX - 1) / TX;
    a.nty = (a.gy + TY - 1) / TY;
    const long ntz = (a.gz + TZ - 1) / TZ;
    const long nt = (long)a.ntx * a.nty * ntz;
    if (nt == 0) return hipSuccess;
    if (nt >= (1L << 31)) return hipErrorInvalidValue;
    a.ntiles = (int)nt;
    hipLaunchKernelGGL((k_chain_pair<VT, XT, ND, TX, TY, TZ>), dim3((unsigned)nt), dim3(256), 0, st, a, A.pbyte, ptab,
                       A.npat * ND, remap);
    return hipGetLastError();
}

// Several chain steps per launch on a box stencil (see MarchPtrs). The grid
// is a stack of planes along the marching dimension (z in 3-D, y in 2-D): a
// plane is gx x gy points (gy = 1 in 2-D), P = gx gy apart. A workgroup
// owns a TX x TY tile of the plane (TX in 2-D) and the planes [m0, m1).
// Level l = 0 .. S holds w_l: level 0 the input, level S the output. Level
// l < S is kept on the tile and S - l points around it (a region of
// (TX + 2(S - l)) x (TY + 2(S - l)) points), zero outside the box, in a ring
// of three planes in LDS. At iteration j the workgroup stores input plane
// m0 - S + j (loaded during iteration j - 1) and then level l computes its
// plane m0 - S + j - l from the three newest planes of level l - 1 (and,
// for a conjugate pair's second step, level l - 2's plane, the step's aux).
// Level S writes plane m0 + j - 2S. Each level's region shrinks by one
// point per side, so every neighbour it reads exists in the level below;
// the first 2S iterations fill the rings.
//
// Row coefficients: KC (constant coefficients) when every row of the matrix
// is one interior row's stencil truncated at the box (the points outside
// the box hold zero in the rings, so the interior coefficients serve every
// row): the ND coefficients are that row's pattern, read once per
// workgroup. Otherwise each point's pattern id is loaded with its plane and
// staged in LDS, and its coefficients come from the pattern table.
template <typename XT>
struct MarchArgs {
    const XT *in;
    XT *out;
    const XT *vfin;
    typename Arith<XT>::T a0[kMarchMax], a1[kMarchMax], a2[kMarchMax];
    int aux;
    int gx, gy, gm;
    int ntx, nty, cz, ntiles;
    int pint;  // KC: the interior row's pattern
};

template <int ND, int S, int TX, int TY>
struct MarchGeom {
    static constexpr int rx(int l) { return TX + 2 * (S - l); }
    static constexpr int ry(int l) { return ND == 7 ? TY + 2 * (S - l) : 1; }
    static constexpr int size(int l) { return rx(l) * ry(l); }
    static constexpr int chunks(int l) { return (size(l) + 255) / 256; }
    // LDS ring of levels 0 .. S-1 (three planes each)
    static constexpr int base(int l) {
        int b = 0;
        for (int m = 0; m < l; ++m) b += 3 * size(m);
        return b;
    }
    // pattern ids of levels 1 .. S (one plane each)
    static constexpr int pbase(int l) {
        int b = 0;
        for (int m = 1; m < l; ++m) b += size(m);
        return b;
    }
    // per-thread registers of levels 1 .. S (one per chunk of 256 points)
    static constexpr int rbase(int l) {
        int b = 0;
        for (int m = 1; m < l; ++m) b += chunks(m);
        return b;
    }
};

// sum_d tab[d] x[d] over the stencil of point q of a level region with row
// length RX, in ascending diagonal order (the pattern table's order): the
// plane below (lo), the plane's own points (mid) and the plane above (hi)
template <typename AT, int ND, int RX>
__device__ __forceinline__ AT march_sum(const AT *tp, const AT *lo, const AT *mid, const AT *hi, int q) {
    AT s = AT(0);
    if constexpr (ND == 7) {
        s += tp[0] * lo[q];
        s += tp[1] * mid[q - RX];
        s += tp[2] * mid[q - 1];
        s += tp[3] * mid[q];
        s += tp[4] * mid[q + 1];
        s += tp[5] * mid[q + RX];
        s += tp[6] * hi[q];
    } else {
        s += tp[0] * lo[q];
        s += tp[1] * mid[q - 1];
        s += tp[2] * mid[q];
        s += tp[3] * mid[q + 1];
        s += tp[4] * hi[q];
    }
    return s;
}

// The per-thread, iteration-invariant part of a level's points: for chunk k
// (point c = thread + 256 k of the level's region) its index in the source
// region (the level below, one point wider per side), its index in the aux
// region (two points wider), and whether it lies in the plane's part of the
// box (x-y; the plane itself is checked per iteration).
template <int ND, int S, int TX, int TY>
struct MarchIdx {
    using G = MarchGeom<ND, S, TX, TY>;
    int q[G::rbase(S + 1)], qa[G::rbase(S + 1)];
    unsigned inb;  // bit rbase(l) + k
};

// Level L (1 <= L < S) of iteration j into its ring slot j % 3.
template <typename XT, int ND, int S, int TX, int TY, bool KC, int L>
__device__ __forceinline__ void march_level(const MarchArgs<XT> &a, typename Arith<XT>::T *ring,
                                            const typename Arith<XT>::T *tab, const int16_t *pat,
                                            const MarchIdx<ND, S, TX, TY> &ix, int j, int m0) {
    using AT = typename Arith<XT>::T;
    using G = MarchGeom<ND, S, TX, TY>;
    if constexpr (L < S) {
        if (j >= 2 * L) {
            constexpr int RXs = G::rx(L - 1), N = G::size(L), C = G::chunks(L), Ns = G::size(L - 1);
            const AT *src = ring + G::base(L - 1);
            const AT *lo = src + ((j + 1) % 3) * Ns, *mid = src + ((j + 2) % 3) * Ns, *hi = src + (j % 3) * Ns;
            AT *dst = ring + G::base(L) + (j % 3) * N;
            const int pm = m0 - S + j - L;
            const bool plane = pm >= 0 && pm < a.gm;
            const AT c0 = a.a0[L - 1], c1 = a.a1[L - 1], c2 = a.a2[L - 1];
            bool aux = false;
            const AT *ax = nullptr;
            if constexpr (L >= 2) {
                aux = (a.aux >> (L - 1)) & 1;
                ax = ring + G::base(L - 2) + ((j + 1) % 3) * G::size(L - 2);
            }
#pragma unroll
            for (int k = 0; k < C; ++k) {
                const int c = (int)threadIdx.x + k * 256;
                if (c < N) {
                    const int r = G::rbase(L) + k;
                    AT w = AT(0);
                    const AT *tp = tab;
                    bool live;
                    if constexpr (KC) {
                        live = plane && ((ix.inb >> r) & 1u);
                    } else {
                        const int id = pat[G::pbase(L) + c];
                        live = id >= 0;
                        tp = tab + id * ND;
                    }
                    if (live) {
                        const int q = ix.q[r];
                        w = c0 * march_sum<AT, ND, RXs>(tp, lo, mid, hi, q) + c1 * mid[q];
                        if (aux) w += c2 * ax[ix.qa[r]];
                    }
                    dst[c] = w;
                }
            }
            __syncthreads();
        }
        march_level<XT, ND, S, TX, TY, KC, L + 1>(a, ring, tab, pat, ix, j, m0);
    }
}

template <typename VT, typename XT, int ND, int S, int TX, int TY, bool KC, int D>
__global__ __launch_bounds__(256) void k_chain_march(MarchArgs<XT> a, const uint8_t *__restrict__ pbyte,
                                                     const VT *__restrict__ ptab, int nent, int remap) {
    using AT = typename Arith<XT>::T;
    using G = MarchGeom<ND, S, TX, TY>;
    static_assert(ND == 5 || ND == 7, "5- or 7-point box stencils");
    static_assert(S >= 2 && S <= kMarchMax, "2 to kMarchMax steps");
    static_assert(ND == 7 || TY == 1, "a 2-D tile is one line");
    static_assert(G::rbase(S + 1) <= 32, "validity bits of every level's chunks in one word");
    constexpr int N0 = G::size(0), C0 = G::chunks(0), RX0 = G::rx(0);
    constexpr int NO = G::size(S), CO = G::chunks(S);
    constexpr int RXl = G::rx(S - 1), Nl = G::size(S - 1);
    constexpr int NP = KC ? 1 : G::pbase(S + 1), CP = G::rbase(S + 1);
    __shared__ AT ring[G::base(S)];
    __shared__ AT tab[KC ? ND : kMaxPatEntries];
    __shared__ int16_t pats[2][NP];  // iteration j uses pats[j % 2] (the last level reads it after the last barrier)
    const int tid = threadIdx.x;
    const int t = remap_tile(blockIdx.x, a.ntiles, remap);
    const int x0 = (t % a.ntx) * TX, y0 = ((t / a.ntx) % a.nty) * TY, m0 = (t / (a.ntx * a.nty)) * a.cz;
    const int m1 = min(m0 + a.cz, a.gm);
    const int gx = a.gx, gy = a.gy, gm = a.gm;
    const long P = (long)gx * gy;
    const int nit = (m1 - m0) + 2 * S;
    if constexpr (KC) {
        if (tid < ND) tab[tid] = (AT)ptab[a.pint * ND + tid];
    } else {
        for (int i = tid; i < nent; i += 256) tab[i] = (AT)ptab[i];
    }
    // iteration-invariant indices of this thread's points
    MarchIdx<ND, S, TX, TY> ix;
    ix.inb = 0u;
    int off0[C0], offp[CP];
#pragma unroll
    for (int k = 0; k < C0; ++k) {
        const int c = tid + k * 256, lx = c % RX0, ly = c / RX0;
        const int px = x0 - S + lx, py = ND == 7 ? y0 - S + ly : 0;
        off0[k] = c < N0 && px >= 0 && px < gx && py >= 0 && py < gy ? px + gx * py : -1;
    }
#pragma unroll
    for (int l = 1; l <= S; ++l) {
        const int RX = G::rx(l), RXs = G::rx(l - 1), N = G::size(l);
#pragma unroll
        for (int k = 0; k < G::chunks(l); ++k) {
            const int c = tid + k * 256, lx = c % RX, ly = c / RX, r = G::rbase(l) + k;
            const int px = x0 - (S - l) + lx, py = ND == 7 ? y0 - (S - l) + ly : 0;
            const bool in = c < N && px >= 0 && px < gx && py >= 0 && py < gy;
            ix.q[r] = ND == 7 ? (lx + 1) + RXs * (ly + 1) : lx + 1;
            ix.qa[r] = l >= 2 ? (ND == 7 ? (lx + 2) + G::rx(l - 2) * (ly + 2) : lx + 2) : 0;
            ix.inb |= (in ? 1u : 0u) << r;
            offp[r] = in ? px + gx * py : -1;
        }
    }
    // What iteration j reads from global memory (the input plane, the
    // pattern ids of every level's plane and the final vector on the tile)
    // is loaded during iteration j - D, into a FIFO of D register sets: with
    // few workgroups per CU one plane in flight does not cover the latency.
    AT pre[D][C0], vf[D][CO];
    int pid[D][KC ? 1 : CP];
    auto prefetch = [&](int j, AT *pr, int *pi, AT *vv) {
        const int pm = m0 - S + j;
        const bool pl0 = j < nit && pm >= 0 && pm < gm;
#pragma unroll
        for (int k = 0; k < C0; ++k) pr[k] = pl0 && off0[k] >= 0 ? (AT)ldx(a.in, off0[k] + P * pm) : AT(0);
        if constexpr (!KC) {
#pragma unroll
            for (int l = 1; l <= S; ++l) {
                const int pml = pm - l;
                const bool pll = j < nit && pml >= 0 && pml < gm;
#pragma unroll
                for (int k = 0; k < G::chunks(l); ++k) {
                    const int r = G::rbase(l) + k;
                    pi[r] = pll && offp[r] >= 0 ? (int)pbyte[offp[r] + P * pml] : -1;
                }
            }
        }
        const int pmo = m0 + j - 2 * S;
        const bool plo = a.vfin && pmo >= m0 && pmo < m1;
#pragma unroll
        for (int k = 0; k < CO; ++k) {
            const int r = G::rbase(S) + k;
            vv[k] = plo && offp[r] >= 0 ? (AT)ldx(a.vfin, offp[r] + P * pmo) : AT(0);
        }
    };
#pragma unroll
    for (int d = 0; d < D; ++d) prefetch(d, pre[d], pid[d], vf[d]);
    for (int j = 0; j < nit; ++j) {
        // with two steps the last one reads level 0 as its aux: the slot
        // written next must not be overwritten before every wave read it
        if constexpr (S == 2) __syncthreads();
        AT *r0 = ring + (j % 3) * N0;
        int16_t *pat = pats[j % 2];
#pragma unroll
        for (int k = 0; k < C0; ++k) {
            const int c = tid + k * 256;
            if (c < N0) r0[c] = pre[0][k];
        }
        if constexpr (!KC) {
#pragma unroll
            for (int l = 1; l <= S; ++l) {
#pragma unroll
                for (int k = 0; k < G::chunks(l); ++k) {
                    const int c = tid + k * 256;
                    if (c < G::size(l)) pat[G::pbase(l) + c] = (int16_t)pid[0][G::rbase(l) + k];
                }
            }
        }
        AT vcur[CO];
#pragma unroll
        for (int k = 0; k < CO; ++k) vcur[k] = vf[0][k];
        // advance the FIFO and load what iteration j + D reads
#pragma unroll
        for (int d = 0; d + 1 < D; ++d) {
#pragma unroll
            for (int k = 0; k < C0; ++k) pre[d][k] = pre[d + 1][k];
            if constexpr (!KC) {
#pragma unroll
                for (int k = 0; k < CP; ++k) pid[d][k] = pid[d + 1][k];
            }
#pragma unroll
            for (int k = 0; k < CO; ++k) vf[d][k] = vf[d + 1][k];
        }
        if (j + D < nit) prefetch(j + D, pre[D - 1], pid[D - 1], vf[D - 1]);
        __syncthreads();
        march_level<XT, ND, S, TX, TY, KC, 1>(a, ring, tab, pat, ix, j, m0);
        if (j >= 2 * S) {
            // the last step on the tile: plane m0 + j - 2S, stored
            const int pm = m0 + j - 2 * S;
            const AT *src = ring + G::base(S - 1);
            const AT *lo = src + ((j + 1) % 3) * Nl, *mid = src + ((j + 2) % 3) * Nl, *hi = src + (j % 3) * Nl;
            const bool aux = (a.aux >> (S - 1)) & 1;
            const AT *ax = ring + G::base(S - 2) + ((j + 1) % 3) * G::size(S - 2);
            const AT c0 = a.a0[S - 1], c1 = a.a1[S - 1], c2 = a.a2[S - 1];
#pragma unroll
            for (int k = 0; k < CO; ++k) {
                const int c = tid + k * 256, r = G::rbase(S) + k;
                const AT *tp = tab;
                bool live;
                if constexpr (KC) {
                    live = (ix.inb >> r) & 1u;
                } else {
                    const int id = c < NO ? (int)pat[G::pbase(S) + c] : -1;
                    live = id >= 0;
                    tp = tab + id * ND;
                }
                if (live) {
                    const int q = ix.q[r];
                    AT w = c0 * march_sum<AT, ND, RXl>(tp, lo, mid, hi, q) + c1 * mid[q];
                    if (aux) w += c2 * ax[ix.qa[r]];
                    stx(a.out, offp[r] + P * pm, a.vfin ? vcur[k] - w : w);
                }
            }
        }
    }
}

// Two chain steps per launch on a constant-coefficient 7-point box stencil
// (DevCSR::box_pint) whose grid lines hold GX points: a workgroup owns TY x
// TZ whole grid lines (y x z). It stages the input on its lines and two lines
// around them in y and z (zero outside the box) in LDS, computes the first
// step on its lines and one line around them into LDS (zero on lines outside
// the box), then the second step on its lines, which it stores. The two
// steps are those of the pair kernel (PairPtrs), which include the marching
// kernel's two-step groups (MarchPtrs):
//     w1 = a01 (A in) + a11 in,   w2 = a02 (A w1) + a12 w1 [+ a22 in if aux2]
//     acc = (init ? 0 : acc) [+ b01 in + b11 w1 if acc1] [+ b02 w1 + b12 w2 if acc2]
//     out = vfin ? vfin - w2 : w2                          (if out)
// so a p chain's pair reads and writes its accumulator once, and w1 never
// leaves LDS. NTH threads; a lane owns 4 consecutive points of a line (GX / 4
// lanes per line): the line itself, the lines above and below in y and z are
// one 4-wide LDS access each, the two neighbours along the line single
// accesses. Products are summed in ascending diagonal order with the interior
// row's coefficients, as the other kernels do. There is no x halo and no
// per-point index arithmetic; the price is the two-line halo in y and z.
template <typename XT>
struct BoxtArgs {
    const XT *in;
    XT *out;
    XT *acc;
    const XT *vfin;
    typename Arith<XT>::T a01, a11, a02, a12, a22, b01, b11, b02, b12;
    int aux2, acc1, acc2, init;
    int gy, gz, nty, ntiles, pint;
};

template <typename VT, typename XT, int TY, int TZ, int GX, int NTH>
__global__ __launch_bounds__(NTH) void k_chain_boxt(BoxtArgs<XT> a, const VT *__restrict__ ptab, int remap) {
    using AT = typename Arith<XT>::T;
    typedef AT AV4 __attribute__((ext_vector_type(4)));
    static_assert(GX % 4 == 0 && NTH % (GX / 4) == 0, "whole lines of 4-point lanes in a workgroup");
    constexpr int LPL = GX / 4, LPP = NTH / LPL;  // lanes per line, lines per pass
    constexpr int RY0 = TY + 4, NL0 = RY0 * (TZ + 4);
    constexpr int RY1 = TY + 2, NL1 = RY1 * (TZ + 2);
    constexpr int NT = TY * TZ;
    constexpr int C0 = (NL0 + LPP - 1) / LPP, C1 = (NL1 + LPP - 1) / LPP, CT = (NT + LPP - 1) / LPP;
    __shared__ AV4 lev0[NL0 * LPL];
    __shared__ AV4 lev1[NL1 * LPL];
    const int tid = threadIdx.x, li = tid / LPL, lx = tid % LPL, x = 4 * lx;
    const int gy = a.gy, gz = a.gz;
    const int t = remap_tile(blockIdx.x, a.ntiles, remap);
    const int y0 = (t % a.nty) * TY, z0 = (t / a.nty) * TZ;
    const long P = (long)GX * gy;
    AT c[7];
#pragma unroll
    for (int d = 0; d < 7; ++d) c[d] = (AT)ptab[a.pint * 7 + d];
    // every global load before the first barrier: the staged input (clamped
    // to a point of the box, dropped outside it), the final vector and the
    // accumulator on the tile's lines
    AT pre[C0][4];
#pragma unroll
    for (int k = 0; k < C0; ++k) {
        const int L = min(li + k * LPP, NL0 - 1);
        const int y = y0 - 2 + L % RY0, z = z0 - 2 + L / RY0;
        const int yc = min(max(y, 0), gy - 1), zc = min(max(z, 0), gz - 1);
        ld4(a.in, zc * P + (long)yc * GX + x, pre[k]);
    }
    const bool load_acc = a.acc && !a.init;
    AT vf[CT][4], pa[CT][4];
#pragma unroll
    for (int k = 0; k < CT; ++k) {
        const int L = min(li + k * LPP, NT - 1);
        const int y = min(y0 + L % TY, gy - 1), z = min(z0 + L / TY, gz - 1);
        const long r = z * P + (long)y * GX + x;
#pragma unroll
        for (int i = 0; i < 4; ++i) vf[k][i] = pa[k][i] = AT(0);
        if (a.vfin) ld4(a.vfin, r, vf[k]);
        if (load_acc) ld4(a.acc, r, pa[k]);
    }
#pragma unroll
    for (int k = 0; k < C0; ++k) {
        const int L = li + k * LPP;
        const int y = y0 - 2 + L % RY0, z = z0 - 2 + L / RY0;
        const bool in = y >= 0 && y < gy && z >= 0 && z < gz;
        if (L < NL0) lev0[L * LPL + lx] = in ? AV4{pre[k][0], pre[k][1], pre[k][2], pre[k][3]} : AV4{0, 0, 0, 0};
    }
    __syncthreads();
    // one step on a line of an LDS region with RY lines per z slice
    auto step = [&](const AV4 *src, int line, int RY, AT a0, AT a1) -> AV4 {
        const AV4 cc = src[line * LPL + lx];
        const AV4 ym = src[(line - 1) * LPL + lx], yp = src[(line + 1) * LPL + lx];
        const AV4 zm = src[(line - RY) * LPL + lx], zp = src[(line + RY) * LPL + lx];
        const AT *sl = reinterpret_cast<const AT *>(src + line * LPL);
        const AT xl = x > 0 ? sl[max(x - 1, 0)] : AT(0);
        const AT xr = x + 4 < GX ? sl[min(x + 4, GX - 1)] : AT(0);
        const AT xv[6] = {xl, cc[0], cc[1], cc[2], cc[3], xr};
        AV4 w;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            AT s = AT(0);
            s += c[0] * zm[i];
            s += c[1] * ym[i];
            s += c[2] * xv[i];
            s += c[3] * xv[i + 1];
            s += c[4] * xv[i + 2];
            s += c[5] * yp[i];
            s += c[6] * zp[i];
            w[i] = a0 * s + a1 * xv[i + 1];
        }
        return w;
    };
    // the first step on the tile's lines and one line around them
#pragma unroll
    for (int k = 0; k < C1; ++k) {
        const int L = li + k * LPP;
        if (L < NL1) {
            const int ly = L % RY1, lz = L / RY1;
            const int y = y0 - 1 + ly, z = z0 - 1 + lz;
            AV4 w = AV4{0, 0, 0, 0};
            if (y >= 0 && y < gy && z >= 0 && z < gz) w = step(lev0, (ly + 1) + RY0 * (lz + 1), RY0, a.a01, a.a11);
            lev1[L * LPL + lx] = w;
        }
    }
    __syncthreads();
    // the second step on the tile's lines, its accumulator update, stored
#pragma unroll
    for (int k = 0; k < CT; ++k) {
        const int L = li + k * LPP;
        if (L < NT) {
            const int ly = L % TY, lz = L / TY;
            const int y = y0 + ly, z = z0 + lz;
            if (y < gy && z < gz) {
                const int q1 = (ly + 1) + RY1 * (lz + 1);
                AV4 w2 = step(lev1, q1, RY1, a.a02, a.a12);
                const AV4 w1 = lev1[q1 * LPL + lx];
                const AV4 xin = lev0[((ly + 2) + RY0 * (lz + 2)) * LPL + lx];
                const long r = z * P + (long)y * GX + x;
                if (a.aux2) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) w2[i] += a.a22 * xin[i];
                }
                if (a.acc) {
                    AT o[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        AT cacc = pa[k][i];
                        if (a.acc1) cacc = cacc + a.b01 * xin[i] + a.b11 * w1[i];
                        if (a.acc2) cacc = cacc + a.b02 * w1[i] + a.b12 * w2[i];
                        o[i] = cacc;
                    }
                    st4(a.acc, r, o);
                }
                if (a.out) {
                    AT o[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) o[i] = a.vfin ? vf[k][i] - w2[i] : w2[i];
                    st4(a.out, r, o);
                }
            }
        }
    }
}

template <typename VT, typename XT, int TY, int TZ, int GX, int NTH>
hipError_t boxt_launch(const DevCSR &A, const VT *ptab, BoxtArgs<XT> a, int remap, hipStream_t st) {
    a.gy = A.box[1];
    a.gz = A.box[2];
    a.nty = (a.gy + TY - 1) / TY;
    const long nt = (long)a.nty * ((a.gz + TZ - 1) / TZ);
    if (nt == 0) return hipSuccess;
    if (nt >= (1L << 31)) return hipErrorInvalidValue;
    a.ntiles = (int)nt;
    a.pint = A.box_pint;
    hipLaunchKernelGGL((k_chain_boxt<VT, XT, TY, TZ, GX, NTH>), dim3((unsigned)nt), dim3(NTH), 0, st, a, ptab,
                       remap);
    return hipGetLastError();
}

template <typename VT, typename XT, int ND, int S, int TX, int TY>
hipError_t march_launch(const DevCSR &A, const VT *ptab, const MarchPtrs &p, int cz, int remap, hipStream_t st) {
    using AT = typename Arith<XT>::T;
    MarchArgs<XT> a;
    a.in = (const XT *)p.in;
    a.out = (XT *)p.out;
    a.vfin = (const XT *)p.vfin;
    for (int k = 0; k < kMarchMax; ++k) {
        a.a0[k] = (AT)p.a0[k];
        a.a1[k] = (AT)p.a1[k];
        a.a2[k] = (AT)p.a2[k];
    }
    a.aux = p.aux;
    a.gx = A.box[0];
    a.gy = ND == 7 ? A.box[1] : 1;
    a.gm = ND == 7 ? A.box[2] : A.box[1];
    a.ntx = (a.gx + TX - 1) / TX;
    a.nty = (a.gy + TY - 1) / TY;
    a.cz = cz;
    const long nch = (a.gm + cz - 1) / cz;
    const long nt = (long)a.ntx * a.nty * nch;
    if (nt == 0) return hipSuccess;
    if (nt >= (1L << 31)) return hipErrorInvalidValue;
    a.ntiles = (int)nt;
    a.pint = A.box_pint;
    if (A.box_pint < 0)
        hipLaunchKernelGGL((k_chain_march<VT, XT, ND, S, TX, TY, false, 1>), dim3((unsigned)nt), dim3(256), 0, st, a,
                           A.pbyte, ptab, A.npat * ND, remap);
    else if (p.depth == 3)
        hipLaunchKernelGGL((k_chain_march<VT, XT, ND, S, TX, TY, true, 3>), dim3((unsigned)nt), dim3(256), 0, st, a,
                           A.pbyte, ptab, A.npat * ND, remap);
    else if (p.depth == 2)
        hipLaunchKernelGGL((k_chain_march<VT, XT, ND, S, TX, TY, true, 2>), dim3((unsigned)nt), dim3(256), 0, st, a,
                           A.pbyte, ptab, A.npat * ND, remap);
    else
        hipLaunchKernelGGL((k_chain_march<VT, XT, ND, S, TX, TY, true, 1>), dim3((unsigned)nt), dim3(256), 0, st, a,
                           A.pbyte, ptab, A.npat * ND, remap);
    return hipGetLastError();
}

template <typename VT, typename XT, int ND, int TX, int TY>
hipError_t march_dispatch(const DevCSR &A, const VT *ptab, const MarchPtrs &p, int cz, int remap, hipStream_t st) {
    switch (p.nsteps) {
        case 2:
            return march_launch<VT, XT, ND, 2, TX, TY>(A, ptab, p, cz, remap, st);
        case 3:
            return march_launch<VT, XT, ND, 3, TX, TY>(A, ptab, p, cz, remap, st);
        case 4:
            return march_launch<VT, XT, ND, 4, TX, TY>(A, ptab, p, cz, remap, st);
    }
    return hipErrorInvalidValue;
}

template <typename VT, typename XT>
ChainArgs<VT, XT> chain_args(const DevCSR &A, const VT *val, const StepPtrs &s) {
    using AT = typename Arith<XT>::T;
    ChainArgs<VT, XT> a;
    a.rowptr = A.rowptr;
    a.colind = A.colind;
    a.val = val;
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
    a.n = A.n;
    a.pin = nullptr;
    a.pout = nullptr;
    return a;
}

template <typename VT, typename XT, int LPR, int U>
hipError_t vec_launch(const ChainArgs<VT, XT> &a, int remap, hipStream_t st) {
    constexpr int RPB = 4 * (64 / LPR) * U;
    const int nb = (a.n + RPB - 1) / RPB;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_chain_vec<VT, XT, LPR, U>), dim3(nb), dim3(256), 0, st, a, nb, remap);
    return hipGetLastError();
}

template <typename XT>
constexpr int prec_of() {
    return sizeof(XT) == 8 ? 0 : (sizeof(XT) == 4 ? 1 : 2);
}

template <typename VT, typename XT, int LPR, int U, int K>
hipError_t vk_launch(const ChainArgs<VT, XT> &a, int remap, hipStream_t st) {
    constexpr int RPB = 4 * (64 / LPR) * U;
    const int nb = (a.n + RPB - 1) / RPB;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_chain_vk<VT, XT, LPR, U, K>), dim3(nb), dim3(256), 0, st, a, nb, remap);
    return hipGetLastError();
}

template <typename VT, typename XT>
hipError_t chain_launch(const DevCSR &A, const VT *val, const StepPtrs &s, int variant, int remap, hipStream_t st) {
    const ChainArgs<VT, XT> a = chain_args<VT, XT>(A, val, s);
    if (A.n == 0) return hipSuccess;
    if (!s.spmv) {
        hipLaunchKernelGGL((k_chain_elem<VT, XT>), dim3((A.n + 255) / 256), dim3(256), 0, st, a,
                           (const XT *)s.prod);
        return hipGetLastError();
    }
    switch (variant) {
        case CV_TILE8:
            hipLaunchKernelGGL((k_chain_tile<VT, XT, 8, 1>), dim3(A.ntile8), dim3(256), 0, st, a, A.tile8, A.ntile8,
                               remap);
            return hipGetLastError();
        case CV_TILE16:
            hipLaunchKernelGGL((k_chain_tile<VT, XT, 16, 2>), dim3(A.ntile16), dim3(256), 0, st, a, A.tile16,
                               A.ntile16, remap);
            return hipGetLastError();
        case CV_VEC1x4:
            return vec_launch<VT, XT, 1, 4>(a, remap, st);
        case CV_VEC4x4:
            return vec_launch<VT, XT, 4, 4>(a, remap, st);
        case CV_VEC8x2:
            return vec_launch<VT, XT, 8, 2>(a, remap, st);
        case CV_VEC8x4:
            return vec_launch<VT, XT, 8, 4>(a, remap, st);
        case CV_VEC16x2:
            return vec_launch<VT, XT, 16, 2>(a, remap, st);
        case CV_VEC16x4:
            return vec_launch<VT, XT, 16, 4>(a, remap, st);
        case CV_VEC32x2:
            return vec_launch<VT, XT, 32, 2>(a, remap, st);
        case CV_TILEV8:
            hipLaunchKernelGGL((k_chain_tilev<VT, XT, 8, 1>), dim3(A.ntile8), dim3(256), 0, st, a, A.tile8, A.ntile8,
                               remap, A.nnz);
            return hipGetLastError();
        case CV_TILEV16:
            hipLaunchKernelGGL((k_chain_tilev<VT, XT, 16, 2>), dim3(A.ntile16), dim3(256), 0, st, a, A.tile16,
                               A.ntile16, remap, A.nnz);
            return hipGetLastError();
        case CV_VK2x4x4:
            return vk_launch<VT, XT, 2, 4, 4>(a, remap, st);
        case CV_VK4x4x2:
            return vk_launch<VT, XT, 4, 4, 2>(a, remap, st);
        case CV_VK8x4x1:
            return vk_launch<VT, XT, 8, 4, 1>(a, remap, st);
        case CV_VK16x2x2:
            return vk_launch<VT, XT, 16, 2, 2>(a, remap, st);
        case CV_DIA:
        case CV_DIA4: {
            if (A.doff.nd <= 0) return hipErrorInvalidValue;
            const int rpt = variant == CV_DIA ? 2 : 1;
            const int nb = (int)((A.n + 256L * rpt - 1) / (256L * rpt));
            if (rpt == 2) {
                hipLaunchKernelGGL((k_chain_dia<VT, XT, 2, 8>), dim3(nb), dim3(256), 0, st, a, dia_vals<VT>(A), A.doff,
                                   nb, remap);
                return hipGetLastError();
            }
#define PP_DIA_ND(K)                                                                                              \
    case K:                                                                                                       \
        hipLaunchKernelGGL((k_chain_dia_nd<VT, XT, K>), dim3(nb), dim3(256), 0, st, a, dia_vals<VT>(A), A.doff, nb, \
                           remap);                                                                                \
        break;
            switch (A.doff.nd) {
                PP_DIA_ND(3)
                PP_DIA_ND(5)
                PP_DIA_ND(7)
                PP_DIA_ND(9)
                PP_DIA_ND(13)
                PP_DIA_ND(19)
                PP_DIA_ND(27)
                default:
                    hipLaunchKernelGGL((k_chain_dia<VT, XT, 1, 8>), dim3(nb), dim3(256), 0, st, a, dia_vals<VT>(A),
                                       A.doff, nb, remap);
            }
#undef PP_DIA_ND
            return hipGetLastError();
        }
        case CV_DIAC: {
            // 4 rows per lane (2 and 8 measured the same on the 128^3 stencil)
            if (A.doff.nd <= 0 || !A.dcode) return hipErrorInvalidValue;
            const int nb = (int)((A.n + 1023L) / 1024L);
#define PP_DIAC_ND(K)                                                                                              \
    case K:                                                                                                        \
        hipLaunchKernelGGL((k_chain_diac<VT, XT, K, 4>), dim3(nb), dim3(256), 0, st, a, A.dcode, diac_tab<VT>(A),    \
                           A.ntab, A.doff, nb, remap);                                                             \
        break;
            switch (A.doff.nd) {
                PP_DIAC_ND(1)
                PP_DIAC_ND(2)
                PP_DIAC_ND(3)
                PP_DIAC_ND(4)
                PP_DIAC_ND(5)
                PP_DIAC_ND(6)
                PP_DIAC_ND(7)
                PP_DIAC_ND(8)
                PP_DIAC_ND(9)
                PP_DIAC_ND(13)
                PP_DIAC_ND(19)
                PP_DIAC_ND(27)
                default:
                    return hipErrorInvalidValue;  // the coded copy is only built for these counts
            }
#undef PP_DIAC_ND
            return hipGetLastError();
        }
        case CV_DIAP: {
            const int nent = A.npat * A.doff.nd;
            if (A.doff.nd <= 0 || !A.pcode || nent <= 0 || nent > kMaxPatEntries) return hipErrorInvalidValue;
            const int nb = (int)((A.n + 1023L) / 1024L);
#define PP_DIAP_ND(K)                                                                                              \
    case K:                                                                                                        \
        hipLaunchKernelGGL((k_chain_diap<VT, XT, K>), dim3(nb), dim3(256), 0, st, a, A.pcode, diap_tab<VT>(A), nent, \
                           A.doff, nb, remap);                                                                     \
        break;
            switch (A.doff.nd) {
                PP_DIAP_ND(1)
                PP_DIAP_ND(2)
                PP_DIAP_ND(3)
                PP_DIAP_ND(4)
                PP_DIAP_ND(5)
                PP_DIAP_ND(6)
                PP_DIAP_ND(7)
                PP_DIAP_ND(8)
                PP_DIAP_ND(9)
                PP_DIAP_ND(13)
                PP_DIAP_ND(19)
                PP_DIAP_ND(27)
                default:
                    return hipErrorInvalidValue;  // built only with the value-coded copy
            }
#undef PP_DIAP_ND
            return hipGetLastError();
        }
        case CV_DIAPV: {
            const int nent = A.npat * A.doff.nd;
            if (A.doff.nd <= 0 || !A.pbyte || nent <= 0 || nent > kMaxPatEntries) return hipErrorInvalidValue;
            int omin = 0, omax = 0;
            for (int d = 0; d < A.doff.nd; ++d) {
                omin = std::min(omin, A.doff.off[d]);
                omax = std::max(omax, A.doff.off[d]);
            }
            const int nb = (int)((A.n + 1023L) / 1024L);
#define PP_DIAPV_ND(K)                                                                                             \
    case K:                                                                                                        \
        hipLaunchKernelGGL((k_chain_diapv<VT, XT, K>), dim3(nb), dim3(256), 0, st, a, A.pbyte, diap_tab<VT>(A),    \
                           nent, A.doff, omin, omax, nb, remap);                                                   \
        break;
            switch (A.doff.nd) {
                PP_DIAPV_ND(1)
                PP_DIAPV_ND(2)
                PP_DIAPV_ND(3)
                PP_DIAPV_ND(4)
                PP_DIAPV_ND(5)
                PP_DIAPV_ND(6)
                PP_DIAPV_ND(7)
                PP_DIAPV_ND(8)
                PP_DIAPV_ND(9)
                PP_DIAPV_ND(13)
                PP_DIAPV_ND(19)
                PP_DIAPV_ND(27)
                default:
                    return hipErrorInvalidValue;  // built only with the value-coded copy
            }
#undef PP_DIAPV_ND
            return hipGetLastError();
        }
        case CV_BOX: {
            if (!box_step_ok(A)) return hipErrorInvalidValue;
            const int nb = (int)((A.n + 1023L) / 1024L);
            if (A.box_nd == 7)
                hipLaunchKernelGGL((k_chain_box<VT, XT, 7>), dim3(nb), dim3(256), 0, st, a, diap_tab<VT>(A), A.box_pint,
                                   A.box[0], A.box[1], A.box[2], nb, remap);
            else
                hipLaunchKernelGGL((k_chain_box<VT, XT, 5>), dim3(nb), dim3(256), 0, st, a, diap_tab<VT>(A), A.box_pint,
                                   A.box[0], A.box[1], 1, nb, remap);
            return hipGetLastError();
        }
        case CV_SELLD:
        case CV_SELLD4: {
            if (A.nslices == 0 || !A.sdel) return hipErrorInvalidValue;
            const int spw = variant == CV_SELLD4 ? 4 : 1;
            const int nb = (A.nslices + 4 * spw - 1) / (4 * spw);
            if (spw == 1)
                hipLaunchKernelGGL((k_chain_sell<VT, XT, true, 1, int16_t>), dim3(nb), dim3(256), 0, st, a, A.sptr,
                                   A.sdel, sell_vals<VT>(A), A.nslices, nb, remap);
            else
                hipLaunchKernelGGL((k_chain_sell<VT, XT, true, 4, int16_t>), dim3(nb), dim3(256), 0, st, a, A.sptr,
                                   A.sdel, sell_vals<VT>(A), A.nslices, nb, remap);
            return hipGetLastError();
        }
        case CV_SELL:
        case CV_SELLT:
        case CV_SELL2:
        case CV_SELL4: {
            if (A.nslices == 0) return hipErrorInvalidValue;
            const int spw = variant == CV_SELL2 ? 2 : (variant == CV_SELL4 ? 4 : 1);
            const int nb = (A.nslices + 4 * spw - 1) / (4 * spw);
            if (variant == CV_SELL)
                hipLaunchKernelGGL((k_chain_sell<VT, XT, true, 1, int32_t>), dim3(nb), dim3(256), 0, st, a, A.sptr, A.scol,
                                   sell_vals<VT>(A), A.nslices, nb, remap);
            else if (variant == CV_SELLT)
                hipLaunchKernelGGL((k_chain_sell<VT, XT, false, 1, int32_t>), dim3(nb), dim3(256), 0, st, a, A.sptr, A.scol,
                                   sell_vals<VT>(A), A.nslices, nb, remap);
            else if (variant == CV_SELL2)
                hipLaunchKernelGGL((k_chain_sell<VT, XT, true, 2, int32_t>), dim3(nb), dim3(256), 0, st, a, A.sptr, A.scol,
                                   sell_vals<VT>(A), A.nslices, nb, remap);
            else
                hipLaunchKernelGGL((k_chain_sell<VT, XT, true, 4, int32_t>), dim3(nb), dim3(256), 0, st, a, A.sptr, A.scol,
                                   sell_vals<VT>(A), A.nslices, nb, remap);
            return hipGetLastError();
        }
        case CV_BAND2:
        case CV_BAND4: {
            // one launch per column band: at any time the gathers touch one
            // band of the input, which stays in the XCDs' L2
            using AT = typename Arith<XT>::T;
            const int c = variant == CV_BAND2 ? 0 : 1, K = A.bandK[c];
            if (K == 0 || !A.bpart) return hipErrorInvalidValue;
            for (int k = 0; k < K; ++k) {
                ChainArgs<VT, XT> ak = a;
                ak.rowptr = A.brow[c] + (size_t)k * (A.n + 1);
                ak.colind = A.bcol[c];
                ak.val = band_vals<VT>(A, c);
                ak.pin = k > 0 ? (const AT *)A.bpart : nullptr;
                ak.pout = k < K - 1 ? (AT *)A.bpart : nullptr;
                const int t0 = A.btoff[c][k], nt = A.btoff[c][k + 1] - t0;
                if (nt > 0)
                    hipLaunchKernelGGL((k_chain_tile<VT, XT, 8, 1, true>), dim3(nt), dim3(256), 0, st, ak,
                                       A.btile[c] + t0, nt, remap);
            }
            return hipGetLastError();
        }
        case CV_CSORT4:
            return cs_launch<VT, XT>(A, a, 4, remap, st);
        case CV_CSORT2:
            return cs_launch<VT, XT>(A, a, 2, remap, st);
        case CV_TILEB8: {
            const int p = prec_of<XT>();
            if (A.ntileB8[p] == 0) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_chain_tile<VT, XT, 8, 1>), dim3(A.ntileB8[p]), dim3(256), 0, st, a, A.tileB8[p],
                               A.ntileB8[p], remap);
            return hipGetLastError();
        }
        case CV_TILEB16: {
            const int p = prec_of<XT>();
            if (A.ntileB16[p] == 0) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_chain_tile<VT, XT, 16, 2>), dim3(A.ntileB16[p]), dim3(256), 0, st, a, A.tileB16[p],
                               A.ntileB16[p], remap);
            return hipGetLastError();
        }
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Gram-Schmidt pieces
// ---------------------------------------------------------------------------

// One chunk of KC Krylov columns for k_dots: all RPT * KC loads are issued
// before the first is used, then each column is reduced over the block.
template <typename XT, int KC>
__device__ __forceinline__ void dots_chunk(const XT *__restrict__ V, long ldv, int c0, const long *ii, const double *wv,
                                           double (*sm)[kDotCols], double *prow) {
    constexpr int RPT = kDotRows / 256;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double x[RPT][KC];
#pragma unroll
    for (int s = 0; s < RPT; ++s)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) x[s][kc] = (double)ldx(V, ii[s] + (long)(c0 + kc) * ldv);
    double acc[KC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        acc[kc] = 0.0;
#pragma unroll
        for (int s = 0; s < RPT; ++s) acc[kc] += x[s][kc] * wv[s];
        acc[kc] = wave_sum(acc[kc]);
    }
    if (lane == 0) {
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) sm[wave][kc] = acc[kc];
    }
    __syncthreads();
    if (tid < KC) prow[c0 + tid] = ((sm[0][tid] + sm[1][tid]) + sm[2][tid]) + sm[3][tid];
    __syncthreads();
}

// partial[b * ldp + c] = sum over the kDotRows rows of block b of V[i,c] w[i]
// (c < ncols). Columns go 8 at a time, then 4, 2, 1 for the remainder, so
// no load waits behind a column-count test. Rows past n read row n-1 and
// are weighted by zero.
template <typename XT>
__global__ __launch_bounds__(256) void k_dots(int n, const XT *V, long ldv, int ncols, const XT *w,
                                              double *partial, int ldp) {
    constexpr int RPT = kDotRows / 256;
    __shared__ double sm[4][kDotCols];
    const long base = (long)blockIdx.x * kDotRows;
    long ii[RPT];
    double wv[RPT];
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
        const long i = base + s * 256 + threadIdx.x;
        ii[s] = i < n ? i : (long)n - 1;
        const double t = (double)ldx(w, ii[s]);
        wv[s] = i < n ? t : 0.0;
    }
    double *prow = partial + (long)blockIdx.x * ldp;
    int c0 = 0;
    for (; c0 + 8 <= ncols; c0 += 8) dots_chunk<XT, 8>(V, ldv, c0, ii, wv, sm, prow);
    if (ncols - c0 >= 4) {
        dots_chunk<XT, 4>(V, ldv, c0, ii, wv, sm, prow);
        c0 += 4;
    }
    if (ncols - c0 >= 2) {
        dots_chunk<XT, 2>(V, ldv, c0, ii, wv, sm, prow);
        c0 += 2;
    }
    if (ncols - c0 >= 1) dots_chunk<XT, 1>(V, ldv, c0, ii, wv, sm, prow);
}

// sum over k < ncols of V[i,k] h[k] for one row: columns 8 at a time (then
// 4, 2, 1) with each chunk's loads issued together.
template <typename XT, int KC>
__device__ __forceinline__ void vh_chunk(const XT *__restrict__ V, long ldv, int k0, const double *__restrict__ h,
                                         long i, double *a) {
    double x[KC];
#pragma unroll
    for (int u = 0; u < KC; ++u) x[u] = (double)ldx(V, i + (long)(k0 + u) * ldv);
#pragma unroll
    for (int u = 0; u < KC; ++u) a[u] += x[u] * h[k0 + u];
}

template <typename XT>
__device__ __forceinline__ double vh_row(const XT *__restrict__ V, long ldv, int ncols, const double *__restrict__ h,
                                         long i) {
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int k0 = 0;
    for (; k0 + 8 <= ncols; k0 += 8) vh_chunk<XT, 8>(V, ldv, k0, h, i, a);
    if (ncols - k0 >= 4) {
        vh_chunk<XT, 4>(V, ldv, k0, h, i, a);
        k0 += 4;
    }
    if (ncols - k0 >= 2) {
        vh_chunk<XT, 2>(V, ldv, k0, h, i, a);
        k0 += 2;
    }
    if (ncols - k0 >= 1) vh_chunk<XT, 1>(V, ldv, k0, h, i, a);
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// ---------------------------------------------------------------------------
// Delayed Gram-Schmidt of the setup cycle: per Arnoldi step one pass of dot
// products (with the pending vector u and w = A u together) and one update
// pass (finishing v_j and forming the next pending vector), with the small
// coefficient algebra in one workgroup between them.
// ---------------------------------------------------------------------------

// One chunk of KC columns of k_dots_pair: sums V_c u and V_c w.
template <typename XT, int KC>
__device__ __forceinline__ void dots2_chunk(const XT *__restrict__ V, long ldv, int c0, int ncols, const long *ii,
                                            const double *uv, const double *wv, double (*sm)[2 * kDotCols],
                                            double *prow) {
    constexpr int RPT = kDotRows / 256;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double x[RPT][KC];
#pragma unroll
    for (int s = 0; s < RPT; ++s)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) x[s][kc] = (double)ldx(V, ii[s] + (long)(c0 + kc) * ldv);
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        double au = 0.0, aw = 0.0;
#pragma unroll
        for (int s = 0; s < RPT; ++s) {
            au += x[s][kc] * uv[s];
            aw += x[s][kc] * wv[s];
        }
        au = wave_sum(au);
        aw = wave_sum(aw);
        if (lane == 0) {
            sm[wave][kc] = au;
            sm[wave][KC + kc] = aw;
        }
    }
    __syncthreads();
    if (tid < 2 * KC) {
        const double t = ((sm[0][tid] + sm[1][tid]) + sm[2][tid]) + sm[3][tid];
        prow[tid < KC ? c0 + tid : ncols + c0 + (tid - KC)] = t;
    }
    __syncthreads();
}

// partial[b*ldp + c] = sum over block b of V_c u, partial[b*ldp + ncols + c]
// = sum of V_c w (c < ncols), partial[b*ldp + 2 ncols] = sum u u and
// [2 ncols + 1] = sum u w; kDotRows rows per block, columns 8 at a time.
template <typename XT>
__global__ __launch_bounds__(256) void k_dots_pair(int n, const XT *V, long ldv, int ncols, const XT *u, const XT *w,
                                                   double *partial, int ldp) {
    constexpr int RPT = kDotRows / 256;
    __shared__ double sm[4][2 * kDotCols];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long base = (long)blockIdx.x * kDotRows;
    long ii[RPT];
    double uv[RPT], wv[RPT];
    double suu = 0.0, suw = 0.0;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
        const long i = base + s * 256 + tid;
        ii[s] = i < n ? i : (long)n - 1;
        const double a = (double)ldx(u, ii[s]), b = (double)ldx(w, ii[s]);
        uv[s] = i < n ? a : 0.0;
        wv[s] = i < n ? b : 0.0;
        suu += uv[s] * uv[s];
        suw += uv[s] * wv[s];
    }
    double *prow = partial + (long)blockIdx.x * ldp;
    int c0 = 0;
    for (; c0 + 8 <= ncols; c0 += 8) dots2_chunk<XT, 8>(V, ldv, c0, ncols, ii, uv, wv, sm, prow);
    if (ncols - c0 >= 4) {
        dots2_chunk<XT, 4>(V, ldv, c0, ncols, ii, uv, wv, sm, prow);
        c0 += 4;
    }
    if (ncols - c0 >= 2) {
        dots2_chunk<XT, 2>(V, ldv, c0, ncols, ii, uv, wv, sm, prow);
        c0 += 2;
    }
    if (ncols - c0 >= 1) dots2_chunk<XT, 1>(V, ldv, c0, ncols, ii, uv, wv, sm, prow);
    suu = wave_sum(suu);
    suw = wave_sum(suw);
    if (lane == 0) {
        sm[wave][0] = suu;
        sm[wave][1] = suw;
    }
    __syncthreads();
    if (tid < 2) prow[2 * ncols + tid] = ((sm[0][tid] + sm[1][tid]) + sm[2][tid]) + sm[3][tid];
}

// The coefficient algebra of delayed step j (one workgroup). dd holds, after
// the reduction: a = V_j^T u (j values), b = V_j^T w (j), alpha = u^T u,
// beta = u^T w. pend holds the first-pass coefficients of H column j-1.
//   rho = sqrt(alpha - a^T a);  v_j = (u - V_j a) / rho
//   H[0:j, j-1] = pend + a,  H[j, j-1] = rho
// and, unless final, with y = Hbar_{(j+1) x j} a and A v_j = (w - V_{j+1} y)/rho:
//   c_k = (b_k - y_k)/rho (k < j),  c_j = ((beta - a^T b)/rho - y_j)/rho
//   g = y/rho + c, the next pending vector u' = w/rho - V_{j+1} g,
//   pend <- c (first-pass coefficients of column j), coef = {1/rho, g_j}.
// g is written to dd[2j+2 ...]. Sums run in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_dcgs_step(int j, double *dd, double *H, int ldh, double *pend, double *coef,
                                                   int final_step) {
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const double *a = dd, *b = dd + j;
    const double alpha = dd[2 * j], beta = dd[2 * j + 1];
    double saa = 0.0, sab = 0.0;
    for (int k = tid; k < j; k += 256) {
        saa += a[k] * a[k];
        sab += a[k] * b[k];
    }
    saa = block_sum256(saa, red);
    sab = block_sum256(sab, red);
    __shared__ double sh[2];
    if (tid == 0) {
        const double rho = sqrt(fmax(alpha - saa, 0.0));
        sh[0] = rho;
        sh[1] = rho > 0.0 ? 1.0 / rho : 0.0;
        if (j >= 1) H[j + (long)(j - 1) * ldh] = rho;
    }
    if (j >= 1)
        for (int k = tid; k < j; k += 256) H[k + (long)(j - 1) * ldh] = pend[k] + a[k];
    __syncthreads();
    if (final_step) return;
    const double inv = sh[1];
    double *g = dd + 2 * j + 2;
    // y_i = sum_k H[i,k] a_k over k < j (H upper Hessenberg: k >= i - 1);
    // the columns of H and a are staged in LDS first (all loads at once)
    // when they fit, so the sums below wait on LDS, not on memory
    constexpr int kStage = 64;
    __shared__ double hs[kStage * (kStage + 1)];
    __shared__ double as[kStage];
    const bool staged = j <= kStage;
    if (staged) {
        for (int q = tid; q < (j + 1) * j; q += 256) {
            const int i = q % (j + 1), k = q / (j + 1);
            hs[q] = H[i + (long)k * ldh];
        }
        for (int k = tid; k < j; k += 256) as[k] = a[k];
        __syncthreads();
    }
    for (int i = tid; i <= j; i += 256) {
        double y = 0.0;
        if (staged)
            for (int k = (i > 0 ? i - 1 : 0); k < j; ++k) y += hs[i + k * (j + 1)] * as[k];
        else
            for (int k = (i > 0 ? i - 1 : 0); k < j; ++k) y += H[i + (long)k * ldh] * a[k];
        const double c = i < j ? (b[i] - y) * inv : ((beta - sab) * inv - y) * inv;
        g[i] = y * inv + c;
        pend[i] = c;
    }
    __syncthreads();
    if (tid == 0) {
        coef[0] = inv;
        coef[1] = g[j];
    }
}

// The dot pass for a wide basis (ncols >= kDotsWideCols): workgroup (bx, c)
// sums the columns [8c, 8c + 8) over the row tiles bx, bx + nbx, ... of
// 256 rows, keeping per-lane sums across its tiles and reducing once at the
// end into partial row bx (same column layout as k_dots_pair, u^T u and
// u^T w from the workgroups with c = 0). Column indices past ncols are
// clamped and their sums dropped. Workgroup ids are ordered so that those
// on one XCD (id % 8) with consecutive id / 8 share their rows, which lets
// the re-reads of u and w hit that XCD's L2.
template <typename XT>
__global__ __launch_bounds__(256) void k_dots_pair_wide(int n, const XT *__restrict__ V, long ldv, int ncols,
                                                        const XT *__restrict__ u, const XT *__restrict__ w,
                                                        double *partial, int ldp, int nbx, int ngroups) {
    constexpr int KC = 8;
    __shared__ double sm[4][2 * KC + 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = (int)(blockIdx.x >> 3);
    const int grp = q % ngroups, bx = (q / ngroups) * 8 + (int)(blockIdx.x & 7);
    if (bx >= nbx) return;
    const int c0 = grp * KC;
    long cofs[KC];
    double au[KC], aw[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        cofs[k] = (long)min(c0 + k, ncols - 1) * ldv;
        au[k] = 0.0;
        aw[k] = 0.0;
    }
    double uu = 0.0, uw = 0.0;
#pragma unroll 2
    for (long b = (long)bx * 256; b < n; b += (long)nbx * 256) {
        const long i = b + tid;
        const long ic = i < n ? i : (long)n - 1;
        double x[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) x[k] = (double)__builtin_nontemporal_load(V + ic + cofs[k]);
        const double ut = (double)ldx(u, ic), wt = (double)ldx(w, ic);
        const double uv = i < n ? ut : 0.0, wv = i < n ? wt : 0.0;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            au[k] += x[k] * uv;
            aw[k] += x[k] * wv;
        }
        uu += uv * uv;
        uw += uv * wv;
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        au[k] = wave_sum(au[k]);
        aw[k] = wave_sum(aw[k]);
    }
    uu = wave_sum(uu);
    uw = wave_sum(uw);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            sm[wave][k] = au[k];
            sm[wave][KC + k] = aw[k];
        }
        sm[wave][2 * KC] = uu;
        sm[wave][2 * KC + 1] = uw;
    }
    __syncthreads();
    double *prow = partial + (long)bx * ldp;
    if (tid < 2 * KC + 2) {
        const double t = ((sm[0][tid] + sm[1][tid]) + sm[2][tid]) + sm[3][tid];
        if (tid < KC) {
            if (c0 + tid < ncols) prow[c0 + tid] = t;
        } else if (tid < 2 * KC) {
            if (c0 + tid - KC < ncols) prow[ncols + c0 + tid - KC] = t;
        } else if (grp == 0) {
            prow[2 * ncols + tid - 2 * KC] = t;
        }
    }
}

// The update pass of delayed step j: per row, s1 = sum_k V[i,k] a_k and
// s2 = sum_k V[i,k] g_k (k < j), then v = (u_i - s1) / rho into vout and
// u'_i = w_i / rho - s2 - v g_j into u (in place). coef = {1/rho, g_j}.
// RPT rows per lane (256 apart), the basis read KC columns at a time with
// all RPT * KC loads of a batch issued together (clamped column index, zero
// coefficient past ncols); NT: non-temporal loads of the basis.
template <typename XT, int RPT, int KC, bool NT>
__global__ __launch_bounds__(256) void k_update_pair(int n, const XT *__restrict__ V, long ldv, int ncols,
                                                     const double *__restrict__ a, const double *__restrict__ g,
                                                     const double *coef, XT *u, const XT *w, XT *vout) {
    const long base = (long)blockIdx.x * 256 * RPT + threadIdx.x;
    long ii[RPT];
    double s1[RPT], s2[RPT];
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
        const long i = base + s * 256;
        ii[s] = i < n ? i : (long)n - 1;
        s1[s] = 0.0;
        s2[s] = 0.0;
    }
    for (int k0 = 0; k0 < ncols; k0 += KC) {
        double x[RPT][KC], ak[KC], gk[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int c = min(k0 + k, ncols - 1);
            const bool in = k0 + k < ncols;
            ak[k] = in ? a[c] : 0.0;
            gk[k] = in ? g[c] : 0.0;
#pragma unroll
            for (int s = 0; s < RPT; ++s)
                x[s][k] = (double)(NT ? __builtin_nontemporal_load(V + ii[s] + (long)c * ldv)
                                      : V[ii[s] + (long)c * ldv]);
        }
#pragma unroll
        for (int s = 0; s < RPT; ++s)
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                s1[s] += x[s][k] * ak[k];
                s2[s] += x[s][k] * gk[k];
            }
    }
    const double inv = coef[0], gj = coef[1];
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
        const long i = base + s * 256;
        const double uo = (double)ldx(u, ii[s]), wo = (double)ldx(w, ii[s]);
        if (i < n) {
            const double v = (uo - s1[s]) * inv;
            stx(vout, i, (typename Arith<XT>::T)v);
            const double vs = stored_value(vout, v);
            stx(u, i, (typename Arith<XT>::T)(wo * inv - s2[s] - vs * gj));
        }
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
        const double vh = vh_row(V, ldv, ncols, h, i);
        const double wn = (double)ldx(w, i) - vh;
        stx(w, i, (typename Arith<XT>::T)wn);
        const double stored = stored_value(w, wn);
        sq = stored * stored;
    }
    if (norm_partial) {
        sq = block_sum256(sq, red);
        if (threadIdx.x == 0) norm_partial[blockIdx.x] = sq;
    }
}

// w <- w - V h and partial[b * ldp + k] = sum over the block's rows of
// V[i,k] * w_new[i]: the update of one Gram-Schmidt pass fused with the
// projection of the next, so V is read once. A row of V (ncols <= KMAX
// values) stays in registers between the two uses.
template <typename XT, int KMAX, int RPT>
__global__ __launch_bounds__(256) void k_update_dots(int n, const XT *V, long ldv, int ncols, const double *h, XT *w,
                                                     double *partial, int ldp) {
    using AT = typename Arith<XT>::T;
    __shared__ double hs[KMAX];
    __shared__ double sm[4][KMAX];
    __shared__ double sm2[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < KMAX) hs[tid] = tid < ncols ? h[tid] : 0.0;
    __syncthreads();
    AT acc[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) acc[k] = AT(0);
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const long i = ((long)blockIdx.x * RPT + q) * 256 + tid;
        if (i < n) {
            // columns past ncols re-read the last one (h is zero there and
            // their sums are dropped), so no load waits behind a test
            AT vr[KMAX];
#pragma unroll
            for (int k = 0; k < KMAX; ++k) vr[k] = (AT)ldx(V, i + (long)(k < ncols ? k : ncols - 1) * ldv);
            double wi = (double)ldx(w, i);
#pragma unroll
            for (int k = 0; k < KMAX; ++k) wi -= (double)vr[k] * hs[k];
            stx(w, i, (AT)wi);
            const double wst = stored_value(w, wi);
            sq += wst * wst;
            const AT ws = (AT)wst;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) acc[k] += vr[k] * ws;
        }
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const double t = wave_sum((double)acc[k]);
        if (lane == 0) sm[wave][k] = t;
    }
    sq = wave_sum(sq);
    if (lane == 0) sm2[wave] = sq;
    __syncthreads();
    if (tid < ncols) partial[(long)blockIdx.x * ldp + tid] = ((sm[0][tid] + sm[1][tid]) + sm[2][tid]) + sm[3][tid];
    if (tid == 0) partial[(long)blockIdx.x * ldp + ncols] = ((sm2[0] + sm2[1]) + sm2[2]) + sm2[3];
}

// After the fused pass: H[k] += h2[k] (k < ncols), and the norm of the final
// vector w'' = w' - V h2 from ||w''||^2 = ||w'||^2 - ||h2||^2 (h2[ncols] holds
// ||w'||^2; h2 is the small reorthogonalisation correction, so there is no
// cancellation). Writes H[ncols] = ||w''||, inv[0] = 1/||w''|| (0 if zero).
__global__ __launch_bounds__(256) void k_finish_col(int ncols, const double *h2, double *H, double *inv) {
    __shared__ double red[4];
    double s = 0.0;
    for (int k = threadIdx.x; k < ncols; k += 256) {
        s += h2[k] * h2[k];
        H[k] += h2[k];
    }
    s = block_sum256(s, red);
    if (threadIdx.x == 0) {
        const double nrm = sqrt(fmax(h2[ncols] - s, 0.0));
        H[ncols] = nrm;
        inv[0] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    }
}

// w <- (w - V h) * inv[0]: the last update of Gram-Schmidt fused with the
// normalisation.
template <typename XT>
__global__ __launch_bounds__(256) void k_update_scale(int n, const XT *V, long ldv, int ncols, const double *h, XT *w,
                                                      const double *inv) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double vh = vh_row(V, ldv, ncols, h, i);
    const double wn = ((double)ldx(w, i) - vh) * inv[0];
    stx(w, i, (typename Arith<XT>::T)wn);
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

// s[i] = 1 / a_ii (right Jacobi scaling); a row without a stored diagonal
// or with a_ii = 0 gets s[i] = 0 and sets *bad.
__global__ __launch_bounds__(256) void k_jacobi(int n, const int32_t *rowptr, const int32_t *colind,
                                                const double *val, double *s, int *bad) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double a = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e)
        if (colind[e] == i) a = val[e];
    s[i] = a != 0.0 ? 1.0 / a : 0.0;
    if (a == 0.0) *bad = 1;
}

// out[k] = val[k] * s[colind[k]]: the values of A diag(s)
__global__ __launch_bounds__(256) void k_scale_cols(int nnz, const int32_t *colind, const double *val,
                                                    const double *s, double *out) {
    const long k = (long)blockIdx.x * 256 + threadIdx.x;
    if (k < nnz) out[k] = val[k] * s[colind[k]];
}

// x[i] *= s[i]
// New values for the value- and pattern-coded copies, keeping their codes:
// the table entry of code c is the new value of its representative entry
// crep[c] (code 0 is zero), the pattern tables follow from their code
// tuples, and *flag is set when some entry differs from its code's new
// value (then the codes no longer describe the matrix).
__global__ __launch_bounds__(256) void k_recode_table(const double *val, const int32_t *crep, int ntab, double *tab64,
                                                      float *tab32, int *flag) {
    const int c = threadIdx.x;
    if (c == 0) *flag = 0;
    if (c < ntab) {
        const double t = (c == 0 || crep[c] < 0) ? 0.0 : val[crep[c]];
        tab64[c] = t;
        tab32[c] = (float)t;
    }
}

__global__ __launch_bounds__(256) void k_recode_check(long nnz, const double *val, const uint8_t *ecode,
                                                      const double *tab64, int *flag) {
    const long k = (long)blockIdx.x * 256 + threadIdx.x;
    if (k < nnz && !(val[k] == tab64[ecode[k]])) *flag = 1;
}

__global__ __launch_bounds__(256) void k_recode_patterns(int nent, const uint8_t *pcodes, const double *tab64,
                                                         double *ptab64, float *ptab32) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < nent) {
        const double t = tab64[pcodes[i]];
        ptab64[i] = t;
        ptab32[i] = (float)t;
    }
}

// x = M^{-1} x~ in place for a block-diagonal M^{-1}: one thread per block of
// bs rows (the last may be shorter), block k row-major with stride bs.
template <int BS>
__global__ __launch_bounds__(64) void k_block_apply(int n, int bs, const double *minv, double *x) {
    const long k = (long)blockIdx.x * 64 + threadIdx.x;
    const long r0 = k * bs;
    if (r0 >= n) return;
    const int m = (int)min((long)bs, (long)n - r0);
    double t[BS];
    for (int c = 0; c < m; ++c) t[c] = x[r0 + c];
    const double *b = minv + k * bs * bs;
    for (int r = 0; r < m; ++r) {
        double s = 0.0;
        for (int c = 0; c < m; ++c) s += b[r * bs + c] * t[c];
        x[r0 + r] = s;
    }
}

__global__ __launch_bounds__(256) void k_vmul(int n, double *x, const double *s) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] *= s[i];
}

__global__ __launch_bounds__(256) void k_val_to_f32(int nnz, const double *v, float *o) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < nnz) o[i] = (float)v[i];
}

__global__ __launch_bounds__(256) void k_sell_values(long npad, const int32_t *sperm, const double *val, double *s64,
                                                     float *s32) {
    const long k = (long)blockIdx.x * 256 + threadIdx.x;
    if (k < npad) {
        const int p = sperm[k];
        const double v = p >= 0 ? val[p] : 0.0;
        s64[k] = v;
        s32[k] = (float)v;
    }
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
    const int v = A.variant[prec], r = A.remap[prec];
    switch (prec) {
        case 0:
            return chain_launch<double, double>(A, A.val64, s, v, r, st);
        case 1:
            return chain_launch<float, float>(A, A.val32, s, v, r, st);
        case 2:
            return chain_launch<float, uint16_t>(A, A.val32, s, v, r, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_boxt_pair(const DevCSR &A, int prec, const PairPtrs &p, int remap, hipStream_t st);

hipError_t launch_chain_pair(const DevCSR &A, int prec, const PairPtrs &p, int remap, hipStream_t st) {
    if (p.shape == 1) return launch_boxt_pair(A, prec, p, remap, st);
    if (!A.pbyte || !p.in || (A.box_nd != 5 && A.box_nd != 7) || A.npat * A.box_nd > kMaxPatEntries ||
        (long)A.box[0] * A.box[1] * A.box[2] != A.n || (p.out && p.out == p.in) || (p.acc && p.acc == p.in))
        return hipErrorInvalidValue;
    switch (prec) {
        case 0:
            return A.box_nd == 7 ? pair_launch<double, double, 7, 32, 8, 4>(A, A.ptab64, p, remap, st)
                                 : pair_launch<double, double, 5, 64, 32, 1>(A, A.ptab64, p, remap, st);
        case 1:
            return A.box_nd == 7 ? pair_launch<float, float, 7, 32, 8, 8>(A, A.ptab32, p, remap, st)
                                 : pair_launch<float, float, 5, 64, 32, 1>(A, A.ptab32, p, remap, st);
    }
    return hipErrorInvalidValue;
}

// x-y tile (x tile in 2-D) of the marching kernel
constexpr int kMarchTX3 = 64, kMarchTY3 = 4, kMarchTX2 = 256;

__global__ __launch_bounds__(1024) void k_empty() {}

hipError_t launch_empty(long blocks, int threads, hipStream_t st) {
    hipLaunchKernelGGL(k_empty, dim3((unsigned)blocks), dim3(threads), 0, st);
    return hipGetLastError();
}

bool box_step_ok(const DevCSR &A) {
    return (A.box_nd == 5 || A.box_nd == 7) && A.box_pint >= 0 && A.pbyte && A.ptab64 && A.ptab32 && A.box[0] > 0 &&
           A.box[0] % 4 == 0 && (long)A.box[0] * A.box[1] * A.box[2] == A.n && A.box_pint < A.npat &&
           A.npat * A.box_nd <= kMaxPatEntries;
}

bool box_tile_ok(const DevCSR &A, int prec) {
    return box_step_ok(A) && A.box_nd == 7 && (prec == 0 || prec == 1) &&
           (A.box[0] == 64 || A.box[0] == 128 || A.box[0] == 256);
}

// tiles (y x z lines) and workgroup sizes of the whole-line kernel: the
// largest tiles whose two levels fit the LDS, with up to 1024 threads, so one
// workgroup per CU covers the 128^3 grid in one round (16 x 4 lines of 128
// points in FP32: 7.0 us per launch, against 8.8 us for 8 x 4 lines with 256
// threads and two workgroups per CU)
template <typename XT>
hipError_t boxt_dispatch(const DevCSR &A, int prec, const BoxtArgs<XT> &a, int remap, hipStream_t st);
template <>
hipError_t boxt_dispatch<float>(const DevCSR &A, int, const BoxtArgs<float> &a, int remap, hipStream_t st) {
    switch (A.box[0]) {
        case 64:
            return boxt_launch<float, float, 8, 8, 64, 256>(A, A.ptab32, a, remap, st);
        case 128:
            return boxt_launch<float, float, 16, 4, 128, 1024>(A, A.ptab32, a, remap, st);
        case 256:
            return boxt_launch<float, float, 8, 4, 256, 1024>(A, A.ptab32, a, remap, st);
    }
    return hipErrorInvalidValue;
}
template <>
hipError_t boxt_dispatch<double>(const DevCSR &A, int, const BoxtArgs<double> &a, int remap, hipStream_t st) {
    switch (A.box[0]) {
        case 64:
            return boxt_launch<double, double, 8, 4, 64, 256>(A, A.ptab64, a, remap, st);
        case 128:
            return boxt_launch<double, double, 8, 4, 128, 1024>(A, A.ptab64, a, remap, st);
        case 256:
            return boxt_launch<double, double, 4, 2, 256, 1024>(A, A.ptab64, a, remap, st);
    }
    return hipErrorInvalidValue;
}

template <typename XT>
BoxtArgs<XT> boxt_args(const PairPtrs &p) {
    using AT = typename Arith<XT>::T;
    BoxtArgs<XT> a;
    std::memset(&a, 0, sizeof(a));
    a.in = (const XT *)p.in;
    a.out = (XT *)p.out;
    a.acc = (XT *)p.acc;
    a.vfin = (const XT *)p.vfin;
    a.a01 = (AT)p.a01;
    a.a11 = (AT)p.a11;
    a.a02 = (AT)p.a02;
    a.a12 = (AT)p.a12;
    a.a22 = (AT)p.a22;
    a.b01 = (AT)p.b01;
    a.b11 = (AT)p.b11;
    a.b02 = (AT)p.b02;
    a.b12 = (AT)p.b12;
    a.aux2 = p.aux2;
    a.acc1 = p.acc1;
    a.acc2 = p.acc2;
    a.init = p.init;
    return a;
}

hipError_t launch_boxt_pair(const DevCSR &A, int prec, const PairPtrs &p, int remap, hipStream_t st) {
    if (!box_tile_ok(A, prec) || !p.in || (!p.out && !p.acc) || (p.out && (p.out == p.in || p.out == p.vfin)) ||
        (p.acc && (p.acc == p.in || p.acc == p.out)))
        return hipErrorInvalidValue;
    if (prec == 1) return boxt_dispatch<float>(A, prec, boxt_args<float>(p), remap, st);
    return boxt_dispatch<double>(A, prec, boxt_args<double>(p), remap, st);
}

hipError_t launch_boxt(const DevCSR &A, int prec, const MarchPtrs &m, int remap, hipStream_t st) {
    if (m.nsteps != 2 || (m.aux & 1) || !m.out) return hipErrorInvalidValue;
    PairPtrs p;
    std::memset(&p, 0, sizeof(p));
    p.in = m.in;
    p.out = m.out;
    p.vfin = m.vfin;
    p.a01 = m.a0[0];
    p.a11 = m.a1[0];
    p.a02 = m.a0[1];
    p.a12 = m.a1[1];
    p.a22 = m.a2[1];
    p.aux2 = (m.aux >> 1) & 1;
    return launch_boxt_pair(A, prec, p, remap, st);
}

hipError_t launch_chain_march(const DevCSR &A, int prec, const MarchPtrs &p, int cz, int remap, hipStream_t st) {
    if (p.shape == 1) return launch_boxt(A, prec, p, remap, st);
    if (!A.pbyte || !p.in || !p.out || (A.box_nd != 5 && A.box_nd != 7) || A.npat * A.box_nd > kMaxPatEntries ||
        (long)A.box[0] * A.box[1] * A.box[2] != A.n || p.out == p.in || p.out == p.vfin || p.nsteps < 2 ||
        p.nsteps > kMarchMax || (p.aux & 1) || cz < 1 || (A.box_nd == 5 && A.box[2] != 1))
        return hipErrorInvalidValue;
    switch (prec) {
        case 0:
            return A.box_nd == 7 ? march_dispatch<double, double, 7, kMarchTX3, kMarchTY3>(A, A.ptab64, p, cz, remap, st)
                                 : march_dispatch<double, double, 5, kMarchTX2, 1>(A, A.ptab64, p, cz, remap, st);
        case 1:
            return A.box_nd == 7 ? march_dispatch<float, float, 7, kMarchTX3, kMarchTY3>(A, A.ptab32, p, cz, remap, st)
                                 : march_dispatch<float, float, 5, kMarchTX2, 1>(A, A.ptab32, p, cz, remap, st);
    }
    return hipErrorInvalidValue;
}

int march_default_cz(const DevCSR &A, int target) {
    const int nd = A.box_nd;
    const long gx = A.box[0], gy = nd == 7 ? A.box[1] : 1, gm = nd == 7 ? A.box[2] : A.box[1];
    const long tiles = nd == 7 ? ((gx + kMarchTX3 - 1) / kMarchTX3) * ((gy + kMarchTY3 - 1) / kMarchTY3)
                               : (gx + kMarchTX2 - 1) / kMarchTX2;
    if (gm <= 0 || tiles <= 0) return 1;
    long cz = gm;
    while (cz > 4 && tiles * ((gm + cz - 1) / cz) < target) cz = (cz + 1) / 2;
    return (int)std::max(1L, cz);
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

template <typename XT>
hipError_t dots_pair_t(int n, const XT *V, long ldv, int ncols, const XT *u, const XT *w, double *partial, int ldp,
                       int max_rows, int *rows, hipStream_t st) {
    *rows = 0;
    if (n <= 0) return hipSuccess;
    // binary32 bases switch to the wide layout earlier (half the bytes per column)
    if (ncols < (sizeof(XT) == 4 ? kDotsWideCols / 2 : kDotsWideCols)) {
        const unsigned g = blocks_for(n, kDotRows);
        if ((int)g > max_rows) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_dots_pair<XT>, dim3(g), dim3(256), 0, st, n, V, ldv, ncols, u, w, partial, ldp);
        *rows = (int)g;
        return hipGetLastError();
    }
    const int nbx = std::min(kDotsWideRows, max_rows);
    if (nbx < 1) return hipErrorInvalidValue;
    const int ngroups = (ncols + 7) / 8;
    const unsigned nwg = 8u * (unsigned)ngroups * (unsigned)((nbx + 7) / 8);
    hipLaunchKernelGGL(k_dots_pair_wide<XT>, dim3(nwg), dim3(256), 0, st, n, V, ldv, ncols, u, w, partial, ldp,
                       nbx, ngroups);
    *rows = nbx;
    return hipGetLastError();
}

hipError_t launch_dots_pair(int prec, int n, const void *V, long ldv, int ncols, const void *u, const void *w,
                            double *partial, int ldp, int max_rows, int *rows, hipStream_t st) {
    if (prec == 0)
        return dots_pair_t<double>(n, (const double *)V, ldv, ncols, (const double *)u, (const double *)w, partial,
                                   ldp, max_rows, rows, st);
    if (prec == 1)
        return dots_pair_t<float>(n, (const float *)V, ldv, ncols, (const float *)u, (const float *)w, partial, ldp,
                                  max_rows, rows, st);
    return hipErrorInvalidValue;
}

hipError_t launch_dcgs_step(int j, double *dd, double *H, int ldh, double *pend, double *coef, int final_step,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_dcgs_step, dim3(1), dim3(256), 0, st, j, dd, H, ldh, pend, coef, final_step);
    return hipGetLastError();
}

template <typename XT>
hipError_t update_pair_t(int n, const XT *V, long ldv, int ncols, const double *a, const double *g,
                         const double *coef, XT *u, const XT *w, XT *vout, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    // narrow bases: 4 rows x 4 columns per batch, cached loads (the recent
    // columns are still in the MALL); wide: 8 rows x 2 columns, streaming
    if (ncols < kDotsWideCols)
        hipLaunchKernelGGL((k_update_pair<XT, 4, 4, false>), dim3(blocks_for(n, 1024)), dim3(256), 0, st, n, V,
                           ldv, ncols, a, g, coef, u, w, vout);
    else
        hipLaunchKernelGGL((k_update_pair<XT, 8, 2, true>), dim3(blocks_for(n, 2048)), dim3(256), 0, st, n, V,
                           ldv, ncols, a, g, coef, u, w, vout);
    return hipGetLastError();
}

hipError_t launch_update_pair(int prec, int n, const void *V, long ldv, int ncols, const double *a, const double *g,
                              const double *coef, void *u, const void *w, void *vout, hipStream_t st) {
    if (prec == 0)
        return update_pair_t<double>(n, (const double *)V, ldv, ncols, a, g, coef, (double *)u, (const double *)w,
                                     (double *)vout, st);
    if (prec == 1)
        return update_pair_t<float>(n, (const float *)V, ldv, ncols, a, g, coef, (float *)u, (const float *)w,
                                    (float *)vout, st);
    return hipErrorInvalidValue;
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

hipError_t launch_jacobi(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double *s, int *bad,
                         hipStream_t st) {
    const unsigned g = blocks_for(n, 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_jacobi, dim3(g), dim3(256), 0, st, n, rowptr, colind, val, s, bad);
    return hipGetLastError();
}

hipError_t launch_scale_cols(int nnz, const int32_t *colind, const double *val, const double *s, double *out,
                             hipStream_t st) {
    const unsigned g = blocks_for(nnz, 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_cols, dim3(g), dim3(256), 0, st, nnz, colind, val, s, out);
    return hipGetLastError();
}

hipError_t launch_recode(long nnz, const double *val, const uint8_t *ecode, const int32_t *crep, int ntab,
                         double *tab64, float *tab32, int nent, const uint8_t *pcodes, double *ptab64, float *ptab32,
                         int *flag, hipStream_t st) {
    if (ntab < 1 || ntab > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_recode_table, dim3(1), dim3(256), 0, st, val, crep, ntab, tab64, tab32, flag);
    if (nnz > 0)
        hipLaunchKernelGGL(k_recode_check, dim3(blocks_for(nnz, 256)), dim3(256), 0, st, nnz, val, ecode, tab64, flag);
    if (nent > 0 && pcodes)
        hipLaunchKernelGGL(k_recode_patterns, dim3(blocks_for(nent, 256)), dim3(256), 0, st, nent, pcodes, tab64,
                           ptab64, ptab32);
    return hipGetLastError();
}

hipError_t launch_block_apply(int n, int bs, const double *minv, double *x, hipStream_t st) {
    if (bs < 1 || bs > kMaxRightBlock) return hipErrorInvalidValue;
    const long nb = ((long)n + bs - 1) / bs;
    const unsigned g = (unsigned)((nb + 63) / 64);
    if (g == 0) return hipSuccess;
    if (bs <= 8)
        hipLaunchKernelGGL(k_block_apply<8>, dim3(g), dim3(64), 0, st, n, bs, minv, x);
    else if (bs <= 16)
        hipLaunchKernelGGL(k_block_apply<16>, dim3(g), dim3(64), 0, st, n, bs, minv, x);
    else
        hipLaunchKernelGGL(k_block_apply<kMaxRightBlock>, dim3(g), dim3(64), 0, st, n, bs, minv, x);
    return hipGetLastError();
}

hipError_t launch_vmul(int n, double *x, const double *s, hipStream_t st) {
    const unsigned g = blocks_for(n, 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_vmul, dim3(g), dim3(256), 0, st, n, x, s);
    return hipGetLastError();
}

hipError_t launch_val_to_f32(int nnz, const double *val64, float *val32, hipStream_t st) {
    const unsigned g = blocks_for(nnz, 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_val_to_f32, dim3(g), dim3(256), 0, st, nnz, val64, val32);
    return hipGetLastError();
}

hipError_t launch_sell_values(long npad, const int32_t *sperm, const double *val, double *sval64, float *sval32,
                              hipStream_t st) {
    const unsigned g = blocks_for(npad, 256);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sell_values, dim3(g), dim3(256), 0, st, npad, sperm, val, sval64, sval32);
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

constexpr int kUdRows = 4;  // rows per thread of k_update_dots

int update_dots_blocks(int n) { return (int)blocks_for(n, 256 * kUdRows); }

int update_dots_max_cols(int prec) { return prec == 0 ? 48 : 64; }

template <typename XT>
static hipError_t ud_launch(int n, const XT *V, long ldv, int ncols, const double *h, XT *w, double *partial, int ldp,
                            hipStream_t st, int prec) {
    const unsigned g = blocks_for(n, 256 * kUdRows);
    if (g == 0 || ncols == 0) return hipSuccess;
#define PP_UD(K)                                                                                             \
    hipLaunchKernelGGL((k_update_dots<XT, K, kUdRows>), dim3(g), dim3(256), 0, st, n, V, ldv, ncols, h, w, partial, \
                       ldp)
    if (ncols <= 4)
        PP_UD(4);
    else if (ncols <= 8)
        PP_UD(8);
    else if (ncols <= 16)
        PP_UD(16);
    else if (ncols <= 24)
        PP_UD(24);
    else if (ncols <= 32)
        PP_UD(32);
    else if (ncols <= 40)
        PP_UD(40);
    else if (ncols <= 48)
        PP_UD(48);
    else if (prec != 0 && ncols <= 64)
        PP_UD(64);
#undef PP_UD
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_update_dots(int prec, int n, const void *V, long ldv, int ncols, const double *h, void *w,
                              double *partial, int ldp, hipStream_t st) {
    switch (prec) {
        case 0:
            return ud_launch<double>(n, (const double *)V, ldv, ncols, h, (double *)w, partial, ldp, st, prec);
        case 1:
            return ud_launch<float>(n, (const float *)V, ldv, ncols, h, (float *)w, partial, ldp, st, prec);
        case 2:
            return ud_launch<uint16_t>(n, (const uint16_t *)V, ldv, ncols, h, (uint16_t *)w, partial, ldp, st, prec);
    }
    return hipErrorInvalidValue;
}

template <typename VT, typename XT>
static hipError_t persist_launch(const DevCSR &A, const VT *val, void *const bufs[5], const PStep *steps, int nsteps,
                                 unsigned long long *bar, unsigned long long bar_base, int *err, int grid, int remap,
                                 hipStream_t st) {
    PArgs<VT, XT> p;
    p.rowptr = A.rowptr;
    p.colind = A.colind;
    p.val = val;
    p.tiles = A.tileP;
    p.ntiles = A.ntileP;
    p.n = A.n;
    for (int i = 0; i < 5; ++i) p.bufs[i] = (XT *)bufs[i];
    p.steps = steps;
    p.nsteps = nsteps;
    p.remap = remap;
    p.bar = bar;
    p.bar_base = bar_base;
    p.err = err;
    void *args[] = {&p};
    return hipLaunchCooperativeKernel((const void *)k_chain_persist<VT, XT, 8>, dim3(grid), dim3(256), args, 0, st);
}

hipError_t launch_chain_persist(const DevCSR &A, int prec, void *const bufs[5], const PStep *steps, int nsteps,
                                unsigned long long *bar, unsigned long long bar_base, int *err, int grid, int remap,
                                hipStream_t st) {
    if (nsteps <= 0) return hipSuccess;
    switch (prec) {
        case 0:
            return persist_launch<double, double>(A, A.val64, bufs, steps, nsteps, bar, bar_base, err, grid, remap, st);
        case 1:
            return persist_launch<float, float>(A, A.val32, bufs, steps, nsteps, bar, bar_base, err, grid, remap, st);
        case 2:
            return persist_launch<float, uint16_t>(A, A.val32, bufs, steps, nsteps, bar, bar_base, err, grid, remap,
                                                   st);
    }
    return hipErrorInvalidValue;
}

template <typename VT, typename XT>
static hipError_t tile_occ(int ept, int *per) {
    if (ept == 8) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, (const void *)k_chain_tile<VT, XT, 8, 1>, 256, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, (const void *)k_chain_tile<VT, XT, 16, 2>, 256, 0);
}

hipError_t tile_slots(int prec, int ept, int *slots) {
    int dev = 0, ncu = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (prec == 0)
        e = tile_occ<double, double>(ept, &per);
    else if (prec == 1)
        e = tile_occ<float, float>(ept, &per);
    else
        e = tile_occ<float, uint16_t>(ept, &per);
    if (e != hipSuccess) return e;
    *slots = per * ncu;
    return hipSuccess;
}

hipError_t persist_max_grid(int prec, int *grid) {
    int dev = 0, ncu = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    switch (prec) {
        case 0:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_chain_persist<double, double, 8>, 256,
                                                             0);
            break;
        case 1:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_chain_persist<float, float, 8>, 256,
                                                             0);
            break;
        default:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_chain_persist<float, uint16_t, 8>,
                                                             256, 0);
    }
    if (e != hipSuccess) return e;
    *grid = per * ncu;
    return hipSuccess;
}

hipError_t launch_finish_col(int ncols, const double *h2, double *H, double *inv, hipStream_t st) {
    hipLaunchKernelGGL(k_finish_col, dim3(1), dim3(256), 0, st, ncols, h2, H, inv);
    return hipGetLastError();
}

hipError_t launch_update_scale(int prec, int n, const void *V, long ldv, int ncols, const double *h, void *w,
                               const double *inv, hipStream_t st) {
    const unsigned g = blocks_for(n, 256);
    if (g == 0) return hipSuccess;
    switch (prec) {
        case 0:
            hipLaunchKernelGGL(k_update_scale<double>, dim3(g), dim3(256), 0, st, n, (const double *)V, ldv, ncols, h,
                               (double *)w, inv);
            break;
        case 1:
            hipLaunchKernelGGL(k_update_scale<float>, dim3(g), dim3(256), 0, st, n, (const float *)V, ldv, ncols, h,
                               (float *)w, inv);
            break;
        case 2:
            hipLaunchKernelGGL(k_update_scale<uint16_t>, dim3(g), dim3(256), 0, st, n, (const uint16_t *)V, ldv, ncols,
                               h, (uint16_t *)w, inv);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

void build_tiles(const int32_t *rp, int n, int row_cap, int nnz_cap, std::vector<int4> &out) {
    out.clear();
    int r = 0;
    while (r < n) {
        const int start = r;
        long nz = 0;
        while (r < n && r - start < row_cap) {
            const long rn = (long)rp[r + 1] - rp[r];
            if (r > start && nz + rn > nnz_cap) break;
            nz += rn;
            ++r;
            if (rn > nnz_cap) break;  // a long row stays alone
        }
        out.push_back(make_int4(start, r, rp[start], rp[r]));
    }
}

const char *chain_variant_name(int v) {
    static const char *names[CV_COUNT] = {"tile8x1", "tile16x2", "vec1x4",  "vec4x4",    "vec8x2",
                                          "vec8x4",  "vec16x2",  "vec16x4", "vec32x2",   "tilev8x1",
                                          "tilev16x2", "vk2x4x4", "vk4x4x2", "vk8x4x1", "vk16x2x2", "persist8",
                                          "tileb8x1", "tileb16x2", "sell64", "sell64t", "sell64x2", "sell64x4", "sell64d16", "sell64d16x4",
                                              "dia2",   "dia1", "diac", "diap", "tile8b2", "tile8b4", "diapv", "box",
                                          "csort4", "csort2"};
    return (v >= 0 && v < CV_COUNT) ? names[v] : "?";
}

}  // namespace ppg
