// Batched kernels: many independent systems (a block-diagonal matrix) with
// R right-hand sides each, advanced in lockstep so that every step of the
// polynomial chain and of Gram-Schmidt is one launch for the whole batch.
//
// * The chain reads the batch's sliced-ELL copy once per step for all R
//   right-hand sides (interleaved vectors: the gather of one entry fetches
//   R consecutive values). Each slice belongs to one system and reads that
//   system's step descriptor (its own polynomial). Workgroups are remapped
//   so that consecutive slices run on one XCD: a row's neighbours a grid
//   line away are then in that XCD's L2, not fetched again by another.
// * Gram-Schmidt works on system-aligned row blocks; per-block partial sums
//   are reduced per system in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batched.h"
#include "devutil.h"

namespace ppg {
namespace {

// The R interleaved values of row i (elements i*R .. i*R + R - 1) move as
// one vector access; every buffer is aligned to R elements (workspace
// columns are multiples of 64 elements apart and the caller's b and x are
// checked on entry).
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(uint16_t v) { return __uint_as_float(((uint32_t)v) << 16); }
__device__ __forceinline__ double narrow(const double *, double v) { return v; }
__device__ __forceinline__ float narrow(const float *, float v) { return v; }
__device__ __forceinline__ uint16_t narrow(const uint16_t *, float v) { return f32_to_bf16(v); }

template <typename XT, int R>
__device__ __forceinline__ void ldr(const XT *__restrict__ p, long i, typename Arith<XT>::T *o) {
    if constexpr (R == 1) {
        o[0] = widen(p[i]);
    } else {
        typedef XT VecT __attribute__((ext_vector_type(R)));
        const VecT t = *reinterpret_cast<const VecT *>(p + i * R);
#pragma unroll
        for (int r = 0; r < R; ++r) o[r] = widen(t[r]);
    }
}

template <typename XT, int R>
__device__ __forceinline__ void str(XT *__restrict__ p, long i, const typename Arith<XT>::T *v) {
    if constexpr (R == 1) {
        p[i] = narrow(p, v[0]);
    } else {
        typedef XT VecT __attribute__((ext_vector_type(R)));
        VecT t;
#pragma unroll
        for (int r = 0; r < R; ++r) t[r] = narrow(p, v[r]);
        *reinterpret_cast<VecT *>(p + i * R) = t;
    }
}

template <typename VT, typename XT>
struct BChainArgs {
    const int4 *slice;
    const int32_t *sptr;
    const int32_t *scol;
    const VT *sval;
    int nslices;
    const int *active;
    const PStep *desc;
    int K;
    int k;
    XT *bufs[5];
};

// Buffers of one chain step for a row. The loads of the row's update go out
// before the product's gathers are used; an absent vector (a uniform
// property of the step) is not read and holds zeros.
template <typename XT>
struct BRow {
    const XT *in, *aux, *fin, *accr;
    XT *out, *acc;
};

template <typename VT, typename XT>
__device__ __forceinline__ BRow<XT> brow_ptrs(const BChainArgs<VT, XT> &a, const PStep &st) {
    BRow<XT> p;
    p.in = a.bufs[st.in];
    p.aux = st.aux >= 0 ? a.bufs[st.aux] : p.in;
    p.fin = st.fin ? a.bufs[0] : p.in;
    p.out = st.out >= 0 ? a.bufs[st.out] : nullptr;
    p.acc = st.acc >= 0 ? a.bufs[st.acc] : nullptr;
    p.accr = (st.acc >= 0 && !st.acc_init) ? p.acc : p.in;
    return p;
}

template <typename XT, int R>
struct BRowIn {
    typename Arith<XT>::T xin[R], aux[R], acc[R], fin[R];
};

template <typename XT, int R>
__device__ __forceinline__ void brow_load(const BRow<XT> &p, const PStep &st, long i, BRowIn<XT, R> &t) {
    using AT = typename Arith<XT>::T;
#pragma unroll
    for (int r = 0; r < R; ++r) t.aux[r] = t.acc[r] = t.fin[r] = AT(0);
    ldr<XT, R>(p.in, i, t.xin);
    if (st.aux >= 0) ldr<XT, R>(p.aux, i, t.aux);
    if (st.acc >= 0 && !st.acc_init) ldr<XT, R>(p.accr, i, t.acc);
    if (st.fin) ldr<XT, R>(p.fin, i, t.fin);
}

// The chain update of one row after its sparse product s (R right-hand
// sides): w = a0 s + a1 in (+ a2 aux), then acc and out as in k_chain.
template <typename XT, int R>
__device__ __forceinline__ void bchain_finish(const PStep &st, const BRow<XT> &p, const BRowIn<XT, R> &t, long row,
                                              const typename Arith<XT>::T *s) {
    using AT = typename Arith<XT>::T;
    const AT a0 = (AT)st.a0, a1 = (AT)st.a1, a2 = (AT)st.a2, b0 = (AT)st.b0, b1 = (AT)st.b1;
    const bool has_aux = st.aux >= 0, zero_acc = st.acc_init != 0, fin = st.fin != 0;
    AT wv[R], o[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const AT w = a0 * s[r] + a1 * t.xin[r];
        const AT wa = w + a2 * t.aux[r];
        wv[r] = has_aux ? wa : w;
    }
    if (p.acc) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const AT c = zero_acc ? AT(0) : t.acc[r];
            o[r] = c + b0 * t.xin[r] + b1 * wv[r];
        }
        str<XT, R>(p.acc, row, o);
    }
    if (p.out) {
#pragma unroll
        for (int r = 0; r < R; ++r) o[r] = fin ? t.fin[r] - wv[r] : wv[r];
        str<XT, R>(p.out, row, o);
    }
}

// The wave's slice index. It is the same on every lane; readfirstlane says
// so to the compiler, so the slice, its step descriptor and the buffer
// pointers come through scalar loads.
__device__ __forceinline__ int bslice_index(int remap) {
    return remap_tile(blockIdx.x, gridDim.x, remap) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// The step descriptor and the active flag of system sys, all fields read
// before the first is tested: the empty asm takes every field as an input,
// so the compiler issues all their scalar loads together and waits once.
template <typename VT, typename XT>
__device__ __forceinline__ PStep bstep(const BChainArgs<VT, XT> &a, int sys, bool &skip) {
    const int on = a.active[sys];
    const PStep st = a.desc[(long)sys * a.K + a.k];
    asm volatile("" ::"s"(on), "s"(st.spmv), "s"(st.in), "s"(st.aux), "s"(st.out), "s"(st.acc), "s"(st.acc_init),
                 "s"(st.fin), "s"(st.a0), "s"(st.a1), "s"(st.a2), "s"(st.b0), "s"(st.b1));
    skip = !on || st.spmv < 0;  // a converged system, or its program is shorter
    return st;
}

template <typename VT, typename XT, int R>
__global__ __launch_bounds__(256) void k_bchain(BChainArgs<VT, XT> a, int remap) {
    using AT = typename Arith<XT>::T;
    constexpr int U = 8;
    const int w = bslice_index(remap);
    if (w >= a.nslices) return;
    const int lane = threadIdx.x & 63;
    const int4 si = a.slice[w];
    bool skip;
    const PStep st = bstep(a, si.z, skip);
    if (skip) return;
    const long row = (long)si.x + lane;
    const long rc = (long)si.x + min(lane, si.y - 1);
    const BRow<XT> p = brow_ptrs(a, st);
    BRowIn<XT, R> t;
    brow_load<XT, R>(p, st, rc, t);
    AT s[R];
#pragma unroll
    for (int r = 0; r < R; ++r) s[r] = AT(0);
    if (st.spmv) {
        const int o0 = a.sptr[w];
        const int width = (a.sptr[w + 1] - o0) >> 6;
        // positions past the slice width re-read its last entry and are
        // dropped by a select, so every load of a block of U is issued
        // before the first is used
        for (int k0 = 0; k0 < width; k0 += U) {
            int c[U];
            VT v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int o = o0 + min(k0 + u, width - 1) * 64 + lane;
                c[u] = __builtin_nontemporal_load(a.scol + o);
                v[u] = __builtin_nontemporal_load(a.sval + o);
            }
            AT xv[U][R];
#pragma unroll
            for (int u = 0; u < U; ++u) ldr<XT, R>(p.in, c[u], xv[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const AT q = (AT)v[u] * xv[u][r];
                    s[r] += (k0 + u < width) ? q : AT(0);
                }
        }
    }
    if (lane >= si.y) return;
    bchain_finish<XT, R>(st, p, t, row, s);
}

// The same step on the pattern-coded copy: a wave takes SPW consecutive
// 64-row slices (one row of each per lane); row i of system sys sums
// ptab[ptoff[sys] + bpat[i] ND + d] x[i + poff[sys ND + d]] over its ND
// diagonals. Columns are clamped into the system's rows (a diagonal that
// leaves the system has a zero entry there) and rows past the slice read its
// last row, so all loads go out unconditionally, those of the SPW rows
// together.
template <typename VT, typename XT, int R, int ND, int SPW>
__global__ __launch_bounds__(256) void k_bchain_pat(BChainArgs<VT, XT> a, const uint8_t *__restrict__ bpat,
                                                    const int32_t *__restrict__ poff,
                                                    const int32_t *__restrict__ ptoff,
                                                    const int32_t *__restrict__ sysoff, const VT *__restrict__ ptab,
                                                    int remap) {
    using AT = typename Arith<XT>::T;
    const int w0 = bslice_index(remap) * SPW;
    if (w0 >= a.nslices) return;
    const int lane = threadIdx.x & 63;
    int4 si[SPW];
    int rc[SPW], code[SPW], lo[SPW], hi[SPW], toff[SPW], po[SPW][ND];
    // what depends on the slices alone goes out first: the rows' pattern
    // bytes and the systems' offsets, beside the step descriptors
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
        si[q] = a.slice[min(w0 + q, a.nslices - 1)];
        const int sys = si[q].z;
        rc[q] = si[q].x + min(lane, si[q].y - 1);
        code[q] = bpat[rc[q]];
        lo[q] = sysoff[sys];
        hi[q] = sysoff[sys + 1] - 1;
        toff[q] = ptoff[sys];
#pragma unroll
        for (int d = 0; d < ND; ++d) po[q][d] = poff[sys * ND + d];
    }
    bool skip[SPW];
    PStep st[SPW];
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
        st[q] = bstep(a, si[q].z, skip[q]);
        skip[q] = skip[q] || w0 + q >= a.nslices;
    }
    BRow<XT> p[SPW];
    BRowIn<XT, R> t[SPW];
    AT xv[SPW][ND][R];
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
        if (skip[q]) continue;
        p[q] = brow_ptrs(a, st[q]);
        brow_load<XT, R>(p[q], st[q], rc[q], t[q]);
        if (st[q].spmv) {
#pragma unroll
            for (int d = 0; d < ND; ++d) ldr<XT, R>(p[q].in, min(max(rc[q] + po[q][d], lo[q]), hi[q]), xv[q][d]);
        }
    }
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
        if (skip[q]) continue;
        AT s[R];
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] = AT(0);
        if (st[q].spmv) {
            const VT *tb = ptab + toff[q] + code[q] * ND;
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                const AT v = (AT)tb[d];
#pragma unroll
                for (int r = 0; r < R; ++r) s[r] += v * xv[q][d][r];
            }
        }
        if (lane < si[q].y) bchain_finish<XT, R>(st[q], p[q], t[q], (long)si[q].x + lane, s);
    }
}

// The same step on constant-coefficient 5-point stencils (every system's
// rows are its interior row's stencil truncated at its own gx_s x gy_s grid):
// no per-row matrix data. A wave takes SPW consecutive 64-row slices (a slice
// lies in one system); the system's line length gx_s, its interior pattern
// (ptab[ptoff[sys] + pint[sys] 5 + d], d over the offsets -gx_s, -1, 0, +1,
// +gx_s) come through uniform loads, and a neighbour outside the system's
// grid counts as zero, which is what its truncated row holds. The terms are
// summed in the pattern-coded kernel's order. The rows above and below are
// loaded (an index outside the grid is clamped to the row itself and dropped
// by a select); the neighbours along the line are the adjacent lanes' own
// inputs (a slice is 64 consecutive rows of one system, cut from its first
// row, so only a full slice's end lanes need rows of another wave).
template <typename VT, typename XT, int R, int SPW>
__global__ __launch_bounds__(256) void k_bchain_box(BChainArgs<VT, XT> a, const int32_t *__restrict__ bgx,
                                                    const int32_t *__restrict__ bpint,
                                                    const int32_t *__restrict__ ptoff,
                                                    const int32_t *__restrict__ sysoff, const VT *__restrict__ ptab,
                                                    int remap) {
    using AT = typename Arith<XT>::T;
    constexpr int ND = 5;
    const int w0 = bslice_index(remap) * SPW;
    if (w0 >= a.nslices) return;
    const int lane = threadIdx.x & 63;
    int4 si[SPW];
    int rc[SPW], gx[SPW], nb[SPW];
    bool in[SPW][ND];
    const VT *tb[SPW];
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
        si[q] = a.slice[min(w0 + q, a.nslices - 1)];
        const int sys = si[q].z;
        rc[q] = si[q].x + min(lane, si[q].y - 1);
        const int base = sysoff[sys], ns = sysoff[sys + 1] - base;
        gx[q] = bgx[sys];
        tb[q] = ptab + ptoff[sys] + bpint[sys] * ND;
        const int loc = rc[q] - base, y = loc / gx[q], x = loc - y * gx[q], gy = ns / gx[q];
        in[q][0] = y > 0;
        in[q][1] = x > 0;
        in[q][2] = true;
        in[q][3] = x + 1 < gx[q];
        in[q][4] = y + 1 < gy;
        nb[q] = base;
    }
    bool skip[SPW];
    PStep st[SPW];
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
        st[q] = bstep(a, si[q].z, skip[q]);
        skip[q] = skip[q] || w0 + q >= a.nslices;
    }
    BRow<XT> p[SPW];
    BRowIn<XT, R> t[SPW];
    AT xv[SPW][ND][R];
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
        if (skip[q]) continue;
        p[q] = brow_ptrs(a, st[q]);
        brow_load<XT, R>(p[q], st[q], rc[q], t[q]);
        if (st[q].spmv) {
            // the rows above and below in the grid; the row's own input and
            // its neighbours along the line come from this lane's and the
            // adjacent lanes' input (rows rc - 1 and rc + 1), except at the
            // wave's two ends, which load theirs
            ldr<XT, R>(p[q].in, in[q][0] ? rc[q] - gx[q] : rc[q], xv[q][0]);
            ldr<XT, R>(p[q].in, in[q][4] ? rc[q] + gx[q] : rc[q], xv[q][4]);
            // the end lanes' loads go out with the others, one instruction
            // for both
            AT e[R] = {};
            const bool lo = lane == 0;
            if (lo || lane == 63)
                ldr<XT, R>(p[q].in, lo ? (in[q][1] ? rc[q] - 1 : rc[q]) : (in[q][3] ? rc[q] + 1 : rc[q]), e);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                xv[q][2][r] = t[q].xin[r];
                const AT up = __shfl_up(t[q].xin[r], 1), dn = __shfl_down(t[q].xin[r], 1);
                xv[q][1][r] = lo ? e[r] : up;
                xv[q][3][r] = lane == 63 ? e[r] : dn;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
        if (skip[q]) continue;
        AT s[R];
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] = AT(0);
        if (st[q].spmv) {
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                const AT v = (AT)tb[q][d];
#pragma unroll
                for (int r = 0; r < R; ++r) s[r] += v * (in[q][d] ? xv[q][d][r] : AT(0));
            }
        }
        if (lane < si[q].y) bchain_finish<XT, R>(st[q], p[q], t[q], (long)si[q].x + lane, s);
    }
}

// One chunk of KC Krylov columns of k_bdots for R interleaved right-hand
// sides: all loads of the chunk are issued before the first is used; each
// wave leaves its sums in sm[wave][(c - g0) R + r], g0 the column group's
// first column (no barrier here).
template <typename XT, int R, int KC>
__device__ __forceinline__ void bdots_chunk(const XT *__restrict__ V, long ldv, int c0, int g0, const long *ii,
                                            const double (*wv)[R], double (*sm)[64]) {
    constexpr int RPT = kBatchBlockRows / 256;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    typename Arith<XT>::T x[RPT][KC][R];
#pragma unroll
    for (int s = 0; s < RPT; ++s)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) ldr<XT, R>(V + (long)(c0 + kc) * ldv, ii[s], x[s][kc]);
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < RPT; ++s) acc += (double)x[s][kc][r] * wv[s][r];
            acc = wave_sum(acc);
            if (lane == 0) sm[wave][(c0 - g0 + kc) * R + r] = acc;
        }
}

// Gram-Schmidt projections of one system-aligned block (<= kBatchBlockRows
// rows, 4 per thread): partial[b*ldp + c*R + r] = sum over the block of
// V_c[i*R+r] w[i*R+r]. Columns go 8/R at a time, then smaller chunks for the
// remainder; rows past the block read its last row with weight zero. The
// waves meet once per group of 64/R columns, when the group's sums are
// combined (wave 0 + 1 + 2 + 3, in that order) and written.
template <typename XT, int R>
__global__ __launch_bounds__(256) void k_bdots(const int4 *block, const int *active, const XT *V, long ldv, int ncols,
                                               const XT *w, double *partial, int ldp) {
    constexpr int RPT = kBatchBlockRows / 256;
    constexpr int KC = 8 / R;
    constexpr int GW = 64 / R;  // a multiple of KC
    __shared__ double sm[4][64];
    const int4 bi = block[blockIdx.x];
    if (active && !active[bi.z]) return;
    const long r1 = (long)bi.x + bi.y;
    long ii[RPT];
    double wv[RPT][R];
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
        const long i = (long)bi.x + s * 256 + threadIdx.x;
        ii[s] = i < r1 ? i : r1 - 1;
        typename Arith<XT>::T t[R];
        ldr<XT, R>(w, ii[s], t);
#pragma unroll
        for (int r = 0; r < R; ++r) wv[s][r] = i < r1 ? (double)t[r] : 0.0;
    }
    double *prow = partial + (long)blockIdx.x * ldp;
    const int tid = threadIdx.x;
    for (int g0 = 0; g0 < ncols; g0 += GW) {
        const int g1 = min(ncols, g0 + GW);
        int c0 = g0;
        for (; c0 + KC <= g1; c0 += KC) bdots_chunk<XT, R, KC>(V, ldv, c0, g0, ii, wv, sm);
        if (KC >= 8 && g1 - c0 >= 4) {
            bdots_chunk<XT, R, (KC >= 8 ? 4 : 1)>(V, ldv, c0, g0, ii, wv, sm);
            c0 += 4;
        }
        if (KC >= 4 && g1 - c0 >= 2) {
            bdots_chunk<XT, R, (KC >= 4 ? 2 : 1)>(V, ldv, c0, g0, ii, wv, sm);
            c0 += 2;
        }
        if (KC >= 2 && g1 - c0 >= 1) bdots_chunk<XT, R, 1>(V, ldv, c0, g0, ii, wv, sm);
        __syncthreads();
        if (tid < (g1 - g0) * R) prow[(long)g0 * R + tid] = ((sm[0][tid] + sm[1][tid]) + sm[2][tid]) + sm[3][tid];
        __syncthreads();
    }
}

// ---- delayed Gram-Schmidt of the cycle (two basis sweeps per step) -------
//
// Step j of pair p works on its pending vector u (the new column once
// orthogonalised, not yet normalised) and w = phi(A) u:
//  dot pass:   V_c^T u and V_c^T w (c < j), u^T u and u^T w per pair;
//  coefficient step (per pair): rho = sqrt(u^T u - ||V^T u||^2) completes
//    column j-1 of the Hessenberg matrix, and the first-pass coefficients
//    of the next column follow from A V = V H (the setup's scheme, per pair);
//  update pass: v_j = (u - V a) / rho (column j), and the next pending vector
//    u' = w / rho - V g - v_j g_j, both from one read of V.

// One chunk of KC columns of k_bdots2: the chunk's loads go out together,
// then per column and rhs the sums against u and w; wave sums land in
// sm[wave][2 ((c - g0) R + r) + {0, 1}].
template <typename XT, int R, int KC>
__device__ __forceinline__ void bdots2_chunk(const XT *__restrict__ V, long ldv, int c0, int g0, const long *ii,
                                             const double (*uv)[R], const double (*wv)[R], double (*sm)[64]) {
    constexpr int RPT = kBatchBlockRows / 256;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    typename Arith<XT>::T x[RPT][KC][R];
#pragma unroll
    for (int s = 0; s < RPT; ++s)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) ldr<XT, R>(V + (long)(c0 + kc) * ldv, ii[s], x[s][kc]);
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double au = 0.0, aw = 0.0;
#pragma unroll
            for (int s = 0; s < RPT; ++s) {
                au += (double)x[s][kc][r] * uv[s][r];
                aw += (double)x[s][kc][r] * wv[s][r];
            }
            au = wave_sum(au);
            aw = wave_sum(aw);
            if (lane == 0) {
                sm[wave][2 * ((c0 - g0 + kc) * R + r)] = au;
                sm[wave][2 * ((c0 - g0 + kc) * R + r) + 1] = aw;
            }
        }
}

// The dot pass of the delayed scheme for one system-aligned block:
// partial[b*ldp + c*R + r] = sum V_c u, partial[b*ldp + (ncols + c)*R + r] =
// sum V_c w (c < ncols), partial[b*ldp + 2 ncols R + r] = sum u u and
// [(2 ncols + 1) R + r] = sum u w. Columns in groups of 32/R (the waves meet
// once per group); rows past the block read its last row with weight zero.
template <typename XT, int R>
__global__ __launch_bounds__(256) void k_bdots2(const int4 *block, const int *active, const XT *V, long ldv, int ncols,
                                                const XT *u, const XT *w, double *partial, int ldp) {
    constexpr int RPT = kBatchBlockRows / 256;
    constexpr int KC = 8 / R > 4 ? 4 : 8 / R;
    constexpr int GW = 32 / R;  // a multiple of KC
    __shared__ double sm[4][64];
    const int4 bi = block[blockIdx.x];
    if (active && !active[bi.z]) return;
    const long r1 = (long)bi.x + bi.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    long ii[RPT];
    double uv[RPT][R], wv[RPT][R], suu[R], suw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) suu[r] = suw[r] = 0.0;
#pragma unroll
    for (int s = 0; s < RPT; ++s) {
        const long i = (long)bi.x + s * 256 + tid;
        ii[s] = i < r1 ? i : r1 - 1;
        typename Arith<XT>::T tu[R], tw[R];
        ldr<XT, R>(u, ii[s], tu);
        ldr<XT, R>(w, ii[s], tw);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uv[s][r] = i < r1 ? (double)tu[r] : 0.0;
            wv[s][r] = i < r1 ? (double)tw[r] : 0.0;
            suu[r] += uv[s][r] * uv[s][r];
            suw[r] += uv[s][r] * wv[s][r];
        }
    }
    double *prow = partial + (long)blockIdx.x * ldp;
    for (int g0 = 0; g0 < ncols; g0 += GW) {
        const int g1 = min(ncols, g0 + GW);
        int c0 = g0;
        for (; c0 + KC <= g1; c0 += KC) bdots2_chunk<XT, R, KC>(V, ldv, c0, g0, ii, uv, wv, sm);
        for (; c0 < g1; ++c0) bdots2_chunk<XT, R, 1>(V, ldv, c0, g0, ii, uv, wv, sm);
        __syncthreads();
        const int nv = (g1 - g0) * R;
        if (tid < 2 * nv) {
            const double t = ((sm[0][tid] + sm[1][tid]) + sm[2][tid]) + sm[3][tid];
            const int q = tid >> 1, c = g0 + q / R, r = q % R;
            prow[((tid & 1) ? ncols + c : c) * R + r] = t;
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double a = wave_sum(suu[r]), b = wave_sum(suw[r]);
        if (lane == 0) {
            sm[wave][2 * r] = a;
            sm[wave][2 * r + 1] = b;
        }
    }
    __syncthreads();
    if (tid < 2 * R) {
        const double t = ((sm[0][tid] + sm[1][tid]) + sm[2][tid]) + sm[3][tid];
        prow[(2 * ncols + (tid & 1)) * R + (tid >> 1)] = t;
    }
}

// The coefficient step of the delayed scheme, one wave per pair p = s R + r
// (systems with no running pair skipped). dd: the dot pass reduced per system
// (layout of k_bdots2, row s at dd + s*ldd). Completes column j-1 of the
// pair's Hessenberg matrix Hf (column c at Hf + p*ldhp + c*ldc, rows 0..c+1)
// from the pending coefficients pend and rho; then, unless final_step, the
// next pending coefficients: with y_i = sum_k H[i,k] a_k (k < j),
// c_i = (b_i - y_i) / rho (i < j), c_j = ((beta - a.b) / rho - y_j) / rho,
// g_i = y_i / rho + c_i; pend = c, g = g, coef[2p] = 1/rho, coef[2p+1] = g_j.
__global__ __launch_bounds__(64) void k_bdcgs_step(int j, int R, const double *dd, int ldd, double *Hf, long ldhp,
                                                   int ldc, double *pend, double *g, double *coef, int final_step,
                                                   const int *active) {
    const int p = blockIdx.x, s = p / R, r = p % R;
    if (active && !active[s]) return;
    const int lane = threadIdx.x;
    const double *ds = dd + (long)s * ldd;
    const double alpha = ds[2 * j * R + r], beta = ds[(2 * j + 1) * R + r];
    double saa = 0.0, sab = 0.0;
    for (int k = lane; k < j; k += 64) {
        const double a = ds[k * R + r], b = ds[(j + k) * R + r];
        saa += a * a;
        sab += a * b;
    }
    saa = wave_sum(saa);
    sab = wave_sum(sab);
    const double rho = sqrt(fmax(alpha - saa, 0.0));
    const double inv = rho > 0.0 ? 1.0 / rho : 0.0;
    double *H = Hf + (long)p * ldhp;
    double *pp = pend + (long)p * ldc, *gg = g + (long)p * ldc;
    if (j >= 1) {
        for (int k = lane; k < j; k += 64) H[(long)(j - 1) * ldc + k] = pp[k] + ds[k * R + r];
        if (lane == 0) H[(long)(j - 1) * ldc + j] = rho;
    }
    __syncthreads();
    if (final_step) {
        if (lane == 0) {
            coef[2 * p] = inv;
            coef[2 * p + 1] = 0.0;
        }
        return;
    }
    for (int i = lane; i <= j; i += 64) {
        double y = 0.0;
        for (int k = (i > 0 ? i - 1 : 0); k < j; ++k) y += H[(long)k * ldc + i] * ds[k * R + r];
        const double c = i < j ? (ds[(j + i) * R + r] - y) * inv : ((beta - sab) * inv - y) * inv;
        gg[i] = y * inv + c;
        pp[i] = c;
    }
    __syncthreads();
    if (lane == 0) {
        coef[2 * p] = inv;
        coef[2 * p + 1] = gg[j];
    }
}

// The update pass of the delayed scheme for one system-aligned block: per
// element (row i, rhs r of pair p), s1 = sum_k V_k a_k and s2 = sum_k V_k g_k
// (k < ncols; a from dd, g per pair), then v = (u - s1) / rho into vout and
// u = w / rho - s2 - v g_j (in place). Coefficients staged in LDS; at most
// kBDcgsMaxCols columns.
constexpr int kBDcgsMaxCols = 128;
template <typename XT, int R>
__global__ __launch_bounds__(256) void k_bupdate2(const int4 *block, const int *active, const XT *V, long ldv, int ncols,
                                                  const double *dd, int ldd, const double *g, int ldc,
                                                  const double *coef, XT *u, const XT *w, XT *vout) {
    constexpr int KC = 8 / R > 4 ? 4 : 8 / R;
    __shared__ double as[kBDcgsMaxCols * R], gs[kBDcgsMaxCols * R], cs[2 * R];
    const int4 bi = block[blockIdx.x];
    if (active && !active[bi.z]) return;
    const int tid = threadIdx.x;
    for (int t = tid; t < ncols * R; t += 256) {
        as[t] = dd[(long)bi.z * ldd + t];  // a_k of rhs r at k R + r
        const int k = t / R, r = t % R;
        gs[t] = g[((long)bi.z * R + r) * ldc + k];
    }
    if (tid < 2 * R) cs[tid] = coef[(long)bi.z * R * 2 + tid];
    __syncthreads();
    const long r0 = bi.x, r1 = (long)bi.x + bi.y;
    for (long i = r0 + tid; i < r1; i += 256) {
        double s1[R], s2[R];
#pragma unroll
        for (int r = 0; r < R; ++r) s1[r] = s2[r] = 0.0;
        int c0 = 0;
        for (; c0 + KC <= ncols; c0 += KC) {
            typename Arith<XT>::T x[KC][R];
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) ldr<XT, R>(V + (long)(c0 + kc) * ldv, i, x[kc]);
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    s1[r] += (double)x[kc][r] * as[(c0 + kc) * R + r];
                    s2[r] += (double)x[kc][r] * gs[(c0 + kc) * R + r];
                }
        }
        for (; c0 < ncols; ++c0) {
            typename Arith<XT>::T x[R];
            ldr<XT, R>(V + (long)c0 * ldv, i, x);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                s1[r] += (double)x[r] * as[c0 * R + r];
                s2[r] += (double)x[r] * gs[c0 * R + r];
            }
        }
        typename Arith<XT>::T uo[R], wo[R], vo[R], un[R];
        ldr<XT, R>(u, i, uo);
        ldr<XT, R>(w, i, wo);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double inv = cs[2 * r], gj = cs[2 * r + 1];
            const double v = ((double)uo[r] - s1[r]) * inv;
            vo[r] = (typename Arith<XT>::T)v;
            const double vs = stored_value(vout, v);
            un[r] = (typename Arith<XT>::T)((double)wo[r] * inv - s2[r] - vs * gj);
        }
        str<XT, R>(vout, i, vo);
        str<XT, R>(u, i, un);
    }
}

// sum over c < ncols of V_c[i*R+r] h[c*R+r] for one row and every r, with
// columns taken KC at a time (all loads of a chunk issued together); KC = 1
// covers the remainder.
template <typename XT, int R>
__device__ __forceinline__ void bvh_row(const XT *__restrict__ V, long ldv, int ncols, const double *__restrict__ hs,
                                        long i, double *acc) {
    constexpr int KC = 16 / R;
    int c0 = 0;
    for (; c0 + KC <= ncols; c0 += KC) {
        typename Arith<XT>::T x[KC][R];
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) ldr<XT, R>(V + (long)(c0 + kc) * ldv, i, x[kc]);
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += (double)x[kc][r] * hs[(c0 + kc) * R + r];
    }
    for (; c0 < ncols; ++c0) {
        typename Arith<XT>::T x[R];
        ldr<XT, R>(V + (long)c0 * ldv, i, x);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += (double)x[r] * hs[c0 * R + r];
    }
}

__global__ __launch_bounds__(256) void k_bred(const int32_t *boff, int R, const double *partial, int ldp, int nt,
                                              double *h, int ldh, double *H, long pstride, int hmode) {
    const int s = blockIdx.x;
    const int b0 = boff[s], b1 = boff[s + 1];
    for (int t = threadIdx.x; t < nt; t += 256) {
        double acc = 0.0;
        for (int b = b0; b < b1; ++b) acc += partial[(long)b * ldp + t];
        if (h) h[(long)s * ldh + t] = acc;
        if (H) {
            double *dst = H + ((long)s * R + t % R) * pstride + t / R;
            if (hmode == 1)
                *dst = acc;
            else if (hmode == 2)
                *dst += acc;
        }
    }
}

template <typename XT, int R>
__global__ __launch_bounds__(256) void k_bupdate(const int4 *block, const int *active, const XT *V, long ldv, int ncols,
                                                 const double *h, int ldh, XT *w, double *npart,
                                                 const double *scale) {
    __shared__ double red[4][R];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int4 bi = block[blockIdx.x];
    if (active && !active[bi.z]) return;
    const long r0 = bi.x, r1 = (long)bi.x + bi.y;
    const double *hs = h + (long)bi.z * ldh;
    double sq[R];
#pragma unroll
    for (int r = 0; r < R; ++r) sq[r] = 0.0;
    for (long i = r0 + tid; i < r1; i += 256) {
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        bvh_row<XT, R>(V, ldv, ncols, hs, i, acc);
        typename Arith<XT>::T wr[R];
        ldr<XT, R>(w, i, wr);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double wn = (double)wr[r] - acc[r];
            if (scale) wn *= scale[(long)bi.z * R + r];
            wr[r] = (typename Arith<XT>::T)wn;
            const double stv = stored_value(w, wn);
            sq[r] += stv * stv;
        }
        str<XT, R>(w, i, wr);
    }
    if (!npart) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double t = wave_sum(sq[r]);
        if (lane == 0) red[wave][r] = t;
    }
    __syncthreads();
    if (tid < R) npart[(long)blockIdx.x * R + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// Fused pass of batched CGS2 (up to KMAX columns): each thread owns the
// elements e = i*R + r of its block with a fixed right-hand side r, keeps
// the element's KMAX basis values in registers, forms w' = w - V h1 (h1 of
// pair (sys, r)) and adds up V^T w' and ||w'||^2 per r:
// partial[b*ldp + k*R + r] for k < ncols, partial[b*ldp + ncols*R + r].
// Columns past ncols re-read the last one with a zero coefficient and
// their sums are dropped.
template <typename XT, int KMAX, int R>
__global__ __launch_bounds__(256) void k_bupdate_dots(const int4 *block, const int *active, const XT *V, long ldv,
                                                      int ncols, const double *h, int ldh, XT *w, double *partial,
                                                      int ldp) {
    using AT = typename Arith<XT>::T;
    __shared__ double hs[KMAX * R];
    __shared__ double sm[4][KMAX * R + R];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int4 bi = block[blockIdx.x];
    if (active && !active[bi.z]) return;
    for (int t = tid; t < KMAX * R; t += 256) hs[t] = t < ncols * R ? h[(long)bi.z * ldh + t] : 0.0;
    __syncthreads();
    const int r = tid % R;
    const long e0 = (long)bi.x * R, e1 = ((long)bi.x + bi.y) * R;
    AT acc[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) acc[k] = AT(0);
    double sq = 0.0;
    for (long e = e0 + tid; e < e1; e += 256) {
        AT vr[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) vr[k] = (AT)ldx(V, e + (long)(k < ncols ? k : ncols - 1) * ldv);
        double wi = (double)ldx(w, e);
#pragma unroll
        for (int k = 0; k < KMAX; ++k) wi -= (double)vr[k] * hs[k * R + r];
        stx(w, e, (AT)wi);
        const double wst = stored_value(w, wi);
        sq += wst * wst;
        const AT ws = (AT)wst;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) acc[k] += vr[k] * ws;
    }
    // sums over the lanes of one r (lanes r, r + R, ...), then over waves
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        double t = (double)acc[k];
#pragma unroll
        for (int off = 32; off >= R; off >>= 1) t += __shfl_xor(t, off, 64);
        if (lane < R) sm[wave][k * R + lane] = t;
    }
#pragma unroll
    for (int off = 32; off >= R; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if (lane < R) sm[wave][KMAX * R + lane] = sq;
    __syncthreads();
    double *prow = partial + (long)blockIdx.x * ldp;
    for (int t = tid; t < ncols * R; t += 256) prow[t] = ((sm[0][t] + sm[1][t]) + sm[2][t]) + sm[3][t];
    if (tid < R) {
        const int t = KMAX * R + tid;
        prow[ncols * R + tid] = ((sm[0][t] + sm[1][t]) + sm[2][t]) + sm[3][t];
    }
}

// After the fused pass, per pair p = s*R + r: H[p][k] += h2[s][k*R + r]
// (k < ncols), and the norm of w'' = w' - V h2 from ||w'||^2 - ||h2||^2
// (h2[s][ncols*R + r] holds ||w'||^2): H[p][ncols] = ||w''||,
// inv[p] = 1/||w''|| (0 if zero).
__global__ __launch_bounds__(64) void k_bfinish(int nsys, int R, int ncols, const double *h2, int ldh, double *H,
                                                long pstride, double *inv) {
    const int p = blockIdx.x * 64 + threadIdx.x;
    if (p >= nsys * R) return;
    const int s = p / R, r = p % R;
    const double *hp = h2 + (long)s * ldh;
    double *Hp = H + (long)p * pstride;
    double ss = 0.0;
    for (int k = 0; k < ncols; ++k) {
        const double c = hp[k * R + r];
        Hp[k] += c;
        ss += c * c;
    }
    const double nrm = sqrt(fmax(hp[ncols * R + r] - ss, 0.0));
    Hp[ncols] = nrm;
    inv[p] = nrm > 0.0 ? 1.0 / nrm : 0.0;
}

__global__ __launch_bounds__(64) void k_bnorm(const int32_t *boff, int nsys, int R, const double *npart, double *H,
                                              long pstride, double *inv) {
    const int p = blockIdx.x * 64 + threadIdx.x;
    if (p >= nsys * R) return;
    const int s = p / R, r = p % R;
    double acc = 0.0;
    for (int b = boff[s]; b < boff[s + 1]; ++b) acc += npart[(long)b * R + r];
    const double nrm = sqrt(acc);
    if (H) H[(long)p * pstride] = nrm;
    inv[p] = nrm > 0.0 ? 1.0 / nrm : 0.0;
}

template <typename TI, typename TO, int R>
__global__ __launch_bounds__(256) void k_bscale(const int4 *block, const int *active, const TI *in, const double *scale,
                                                TO *out) {
    const int4 bi = block[blockIdx.x];
    if (active && !active[bi.z]) return;
    const long r0 = bi.x, r1 = (long)bi.x + bi.y;
    for (long i = r0 + threadIdx.x; i < r1; i += 256) {
        typename Arith<TI>::T v[R];
        typename Arith<TO>::T o[R];
        ldr<TI, R>(in, i, v);
#pragma unroll
        for (int r = 0; r < R; ++r) o[r] = (typename Arith<TO>::T)((double)v[r] * scale[(long)bi.z * R + r]);
        str<TO, R>(out, i, o);
    }
}

// out = V z per pair over that pair's own kp[p] columns (columns past a
// pair's last step may hold stale values of other cycles and are not read)
template <typename XT, int R>
__global__ __launch_bounds__(256) void k_bcombine(const int4 *block, const XT *V, long ldv, const int *kp,
                                                  const double *z, int ldz, XT *out) {
    const int4 bi = block[blockIdx.x];
    const long r0 = bi.x, r1 = (long)bi.x + bi.y;
    int kr[R], kmax = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        kr[r] = kp[(long)bi.z * R + r];
        kmax = kr[r] > kmax ? kr[r] : kmax;
    }
    const double *zs = z + (long)bi.z * R * ldz;
    constexpr int KC = 16 / R;
    for (long i = r0 + threadIdx.x; i < r1; i += 256) {
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        // columns j >= kr[r] of pair r are dropped by a select (they may hold
        // stale values of other cycles), so a chunk's loads go out together
        for (int j0 = 0; j0 < kmax; j0 += KC) {
            typename Arith<XT>::T x[KC][R];
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) ldr<XT, R>(V + (long)min(j0 + kc, kmax - 1) * ldv, i, x[kc]);
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int j = j0 + kc;
                    const double t = (double)x[kc][r] * zs[(long)r * ldz + min(j, kmax - 1)];
                    acc[r] += j < kr[r] ? t : 0.0;
                }
        }
        typename Arith<XT>::T o[R];
#pragma unroll
        for (int r = 0; r < R; ++r) o[r] = (typename Arith<XT>::T)acc[r];
        str<XT, R>(out, i, o);
    }
}

// ---- dispatch helpers -----------------------------------------------------

template <typename VT, typename XT, int R, int SPW>
hipError_t bchain_box_t(const BatchSell &S, const BChainArgs<VT, XT> &a, const VT *ptab, hipStream_t st) {
    const unsigned g = (unsigned)((S.nslices + 4 * SPW - 1) / (4 * SPW));
    hipLaunchKernelGGL((k_bchain_box<VT, XT, R, SPW>), dim3(g), dim3(256), 0, st, a, S.bgx, S.bpint, S.ptoff,
                       S.sysoff, ptab, S.remap);
    return hipGetLastError();
}

template <typename VT, typename XT, int R, int SPW>
hipError_t bchain_pat_t(const BatchSell &S, const BChainArgs<VT, XT> &a, const VT *ptab, hipStream_t st) {
    const unsigned g = (unsigned)((S.nslices + 4 * SPW - 1) / (4 * SPW));
#define PP_BPAT_ND(K)                                                                                             \
    case K:                                                                                                       \
        hipLaunchKernelGGL((k_bchain_pat<VT, XT, R, K, SPW>), dim3(g), dim3(256), 0, st, a, S.bpat, S.poff,      \
                           S.ptoff, S.sysoff, ptab, S.remap);                                                     \
        break;
    switch (S.pnd) {
        PP_BPAT_ND(3)
        PP_BPAT_ND(5)
        PP_BPAT_ND(7)
        PP_BPAT_ND(9)
        PP_BPAT_ND(13)
        PP_BPAT_ND(19)
        PP_BPAT_ND(27)
        default:
            return hipErrorInvalidValue;  // the copy is built only for these counts
    }
#undef PP_BPAT_ND
    return hipGetLastError();
}

template <typename VT, typename XT>
hipError_t bchain_t(const BatchSell &S, const VT *sval, const VT *ptab, int R, const PStep *desc, int K, int k,
                    void *const bufs[5], hipStream_t st) {
    if (!S.active) return hipErrorInvalidValue;  // the kernels read the flags unconditionally
    BChainArgs<VT, XT> a;
    a.slice = S.slice;
    a.sptr = S.sptr;
    a.scol = S.scol;
    a.sval = sval;
    a.nslices = S.nslices;
    a.active = S.active;
    a.desc = desc;
    a.K = K;
    a.k = k;
    for (int i = 0; i < 5; ++i) a.bufs[i] = (XT *)bufs[i];
    const unsigned g = (unsigned)((S.nslices + 3) / 4);
    if (g == 0) return hipSuccess;
    if (S.bgx) {
        if (!S.bpint || !S.ptoff || !S.sysoff || !ptab) return hipErrorInvalidValue;
        const bool two = S.spw == 2;
        switch (R) {
            case 1:
                return two ? bchain_box_t<VT, XT, 1, 2>(S, a, ptab, st) : bchain_box_t<VT, XT, 1, 1>(S, a, ptab, st);
            case 2:
                return two ? bchain_box_t<VT, XT, 2, 2>(S, a, ptab, st) : bchain_box_t<VT, XT, 2, 1>(S, a, ptab, st);
            case 4:
                return two ? bchain_box_t<VT, XT, 4, 2>(S, a, ptab, st) : bchain_box_t<VT, XT, 4, 1>(S, a, ptab, st);
            default:
                return hipErrorInvalidValue;
        }
    }
    if (S.bpat) {
        const bool two = S.spw == 2;
        switch (R) {
            case 1:
                return two ? bchain_pat_t<VT, XT, 1, 2>(S, a, ptab, st) : bchain_pat_t<VT, XT, 1, 1>(S, a, ptab, st);
            case 2:
                return two ? bchain_pat_t<VT, XT, 2, 2>(S, a, ptab, st) : bchain_pat_t<VT, XT, 2, 1>(S, a, ptab, st);
            case 4:
                return two ? bchain_pat_t<VT, XT, 4, 2>(S, a, ptab, st) : bchain_pat_t<VT, XT, 4, 1>(S, a, ptab, st);
            default:
                return hipErrorInvalidValue;
        }
    }
    switch (R) {
        case 1:
            hipLaunchKernelGGL((k_bchain<VT, XT, 1>), dim3(g), dim3(256), 0, st, a, S.remap);
            break;
        case 2:
            hipLaunchKernelGGL((k_bchain<VT, XT, 2>), dim3(g), dim3(256), 0, st, a, S.remap);
            break;
        case 4:
            hipLaunchKernelGGL((k_bchain<VT, XT, 4>), dim3(g), dim3(256), 0, st, a, S.remap);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename XT>
hipError_t bdots_t(const BatchBlocks &B, int R, const XT *V, long ldv, int ncols, const XT *w, double *partial, int ldp,
                   hipStream_t st) {
    if (B.nblocks == 0 || ncols == 0) return hipSuccess;
    switch (R) {
        case 1:
            hipLaunchKernelGGL((k_bdots<XT, 1>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols, w, partial,
                               ldp);
            break;
        case 2:
            hipLaunchKernelGGL((k_bdots<XT, 2>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols, w, partial,
                               ldp);
            break;
        case 4:
            hipLaunchKernelGGL((k_bdots<XT, 4>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols, w, partial,
                               ldp);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename XT>
hipError_t bupdate_t(const BatchBlocks &B, int R, const XT *V, long ldv, int ncols, const double *h, int ldh, XT *w,
                     double *npart, const double *scale, hipStream_t st) {
    if (B.nblocks == 0) return hipSuccess;
    switch (R) {
        case 1:
            hipLaunchKernelGGL((k_bupdate<XT, 1>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols, h, ldh, w,
                               npart, scale);
            break;
        case 2:
            hipLaunchKernelGGL((k_bupdate<XT, 2>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols, h, ldh, w,
                               npart, scale);
            break;
        case 4:
            hipLaunchKernelGGL((k_bupdate<XT, 4>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols, h, ldh, w,
                               npart, scale);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename XT, int R>
hipError_t bupdate_dots_r(const BatchBlocks &B, const XT *V, long ldv, int ncols, const double *h, int ldh, XT *w,
                          double *partial, int ldp, hipStream_t st) {
#define PP_BUD(K)                                                                                                  \
    if (ncols <= K) {                                                                                              \
        hipLaunchKernelGGL((k_bupdate_dots<XT, K, R>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, \
                           ncols, h, ldh, w, partial, ldp);                                                        \
        return hipGetLastError();                                                                                  \
    }
    PP_BUD(8)
    PP_BUD(16)
    PP_BUD(24)
    PP_BUD(32)
    PP_BUD(40)
    PP_BUD(48)
    if constexpr (sizeof(XT) < 8) {
        PP_BUD(64)
    }
#undef PP_BUD
    return hipErrorInvalidValue;
}

template <typename XT>
hipError_t bupdate_dots_t(const BatchBlocks &B, int R, const XT *V, long ldv, int ncols, const double *h, int ldh,
                          XT *w, double *partial, int ldp, hipStream_t st) {
    if (B.nblocks == 0 || ncols < 1) return hipSuccess;
    switch (R) {
        case 1:
            return bupdate_dots_r<XT, 1>(B, V, ldv, ncols, h, ldh, w, partial, ldp, st);
        case 2:
            return bupdate_dots_r<XT, 2>(B, V, ldv, ncols, h, ldh, w, partial, ldp, st);
        case 4:
            return bupdate_dots_r<XT, 4>(B, V, ldv, ncols, h, ldh, w, partial, ldp, st);
    }
    return hipErrorInvalidValue;
}

template <typename TI, typename TO>
hipError_t bscale_t(const BatchBlocks &B, int R, const TI *in, const double *scale, TO *out, hipStream_t st) {
    if (B.nblocks == 0) return hipSuccess;
    switch (R) {
        case 1:
            hipLaunchKernelGGL((k_bscale<TI, TO, 1>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, in, scale, out);
            break;
        case 2:
            hipLaunchKernelGGL((k_bscale<TI, TO, 2>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, in, scale, out);
            break;
        case 4:
            hipLaunchKernelGGL((k_bscale<TI, TO, 4>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, in, scale, out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TI>
hipError_t bscale_in(const BatchBlocks &B, int prec_out, int R, const TI *in, const double *scale, void *out,
                     hipStream_t st) {
    switch (prec_out) {
        case 0:
            return bscale_t<TI, double>(B, R, in, scale, (double *)out, st);
        case 1:
            return bscale_t<TI, float>(B, R, in, scale, (float *)out, st);
        case 2:
            return bscale_t<TI, uint16_t>(B, R, in, scale, (uint16_t *)out, st);
    }
    return hipErrorInvalidValue;
}

template <typename XT>
hipError_t bcombine_t(const BatchBlocks &B, int R, const XT *V, long ldv, const int *k, const double *z, int ldz, XT *out,
                      hipStream_t st) {
    if (B.nblocks == 0) return hipSuccess;
    switch (R) {
        case 1:
            hipLaunchKernelGGL((k_bcombine<XT, 1>), dim3(B.nblocks), dim3(256), 0, st, B.block, V, ldv, k, z, ldz, out);
            break;
        case 2:
            hipLaunchKernelGGL((k_bcombine<XT, 2>), dim3(B.nblocks), dim3(256), 0, st, B.block, V, ldv, k, z, ldz, out);
            break;
        case 4:
            hipLaunchKernelGGL((k_bcombine<XT, 4>), dim3(B.nblocks), dim3(256), 0, st, B.block, V, ldv, k, z, ldz, out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bchain(const BatchSell &S, int prec, int R, const PStep *desc, int K, int k, void *const bufs[5],
                         hipStream_t st) {
    switch (prec) {
        case 0:
            return bchain_t<double, double>(S, S.sval64, S.ptab64, R, desc, K, k, bufs, st);
        case 1:
            return bchain_t<float, float>(S, S.sval32, S.ptab32, R, desc, K, k, bufs, st);
        case 2:
            return bchain_t<float, uint16_t>(S, S.sval32, S.ptab32, R, desc, K, k, bufs, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_bdots(const BatchBlocks &B, int prec, int R, const void *V, long ldv, int ncols, const void *w,
                        double *partial, int ldp, hipStream_t st) {
    switch (prec) {
        case 0:
            return bdots_t<double>(B, R, (const double *)V, ldv, ncols, (const double *)w, partial, ldp, st);
        case 1:
            return bdots_t<float>(B, R, (const float *)V, ldv, ncols, (const float *)w, partial, ldp, st);
        case 2:
            return bdots_t<uint16_t>(B, R, (const uint16_t *)V, ldv, ncols, (const uint16_t *)w, partial, ldp, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_bred(const BatchBlocks &B, int R, const double *partial, int ldp, int nt, double *h, int ldh,
                       double *H, long pstride, int hmode, hipStream_t st) {
    if (B.nsys == 0 || nt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bred, dim3(B.nsys), dim3(256), 0, st, B.boff, R, partial, ldp, nt, h, ldh, H, pstride, hmode);
    return hipGetLastError();
}

hipError_t launch_bupdate(const BatchBlocks &B, int prec, int R, const void *V, long ldv, int ncols, const double *h,
                          int ldh, void *w, double *npart, const double *scale, hipStream_t st) {
    switch (prec) {
        case 0:
            return bupdate_t<double>(B, R, (const double *)V, ldv, ncols, h, ldh, (double *)w, npart, scale, st);
        case 1:
            return bupdate_t<float>(B, R, (const float *)V, ldv, ncols, h, ldh, (float *)w, npart, scale, st);
        case 2:
            return bupdate_t<uint16_t>(B, R, (const uint16_t *)V, ldv, ncols, h, ldh, (uint16_t *)w, npart, scale, st);
    }
    return hipErrorInvalidValue;
}

int bupdate_dots_max_cols(int prec) { return prec == 0 ? 48 : 64; }

hipError_t launch_bupdate_dots(const BatchBlocks &B, int prec, int R, const void *V, long ldv, int ncols,
                               const double *h, int ldh, void *w, double *partial, int ldp, hipStream_t st) {
    switch (prec) {
        case 0:
            return bupdate_dots_t<double>(B, R, (const double *)V, ldv, ncols, h, ldh, (double *)w, partial, ldp, st);
        case 1:
            return bupdate_dots_t<float>(B, R, (const float *)V, ldv, ncols, h, ldh, (float *)w, partial, ldp, st);
        case 2:
            return bupdate_dots_t<uint16_t>(B, R, (const uint16_t *)V, ldv, ncols, h, ldh, (uint16_t *)w, partial, ldp,
                                            st);
    }
    return hipErrorInvalidValue;
}

template <typename XT>
hipError_t bdots2_t(const BatchBlocks &B, int R, const XT *V, long ldv, int ncols, const XT *u, const XT *w,
                    double *partial, int ldp, hipStream_t st) {
    if (B.nblocks == 0) return hipSuccess;
    switch (R) {
        case 1:
            hipLaunchKernelGGL((k_bdots2<XT, 1>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols, u,
                               w, partial, ldp);
            break;
        case 2:
            hipLaunchKernelGGL((k_bdots2<XT, 2>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols, u,
                               w, partial, ldp);
            break;
        case 4:
            hipLaunchKernelGGL((k_bdots2<XT, 4>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols, u,
                               w, partial, ldp);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename XT>
hipError_t bupdate2_t(const BatchBlocks &B, int R, const XT *V, long ldv, int ncols, const double *dd, int ldd,
                      const double *g, int ldc, const double *coef, XT *u, const XT *w, XT *vout, hipStream_t st) {
    if (B.nblocks == 0) return hipSuccess;
    switch (R) {
        case 1:
            hipLaunchKernelGGL((k_bupdate2<XT, 1>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols,
                               dd, ldd, g, ldc, coef, u, w, vout);
            break;
        case 2:
            hipLaunchKernelGGL((k_bupdate2<XT, 2>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols,
                               dd, ldd, g, ldc, coef, u, w, vout);
            break;
        case 4:
            hipLaunchKernelGGL((k_bupdate2<XT, 4>), dim3(B.nblocks), dim3(256), 0, st, B.block, B.active, V, ldv, ncols,
                               dd, ldd, g, ldc, coef, u, w, vout);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bdots2(const BatchBlocks &B, int prec, int R, const void *V, long ldv, int ncols, const void *u,
                         const void *w, double *partial, int ldp, hipStream_t st) {
    switch (prec) {
        case 0:
            return bdots2_t<double>(B, R, (const double *)V, ldv, ncols, (const double *)u, (const double *)w, partial,
                                    ldp, st);
        case 1:
            return bdots2_t<float>(B, R, (const float *)V, ldv, ncols, (const float *)u, (const float *)w, partial, ldp,
                                   st);
        case 2:
            return bdots2_t<uint16_t>(B, R, (const uint16_t *)V, ldv, ncols, (const uint16_t *)u,
                                      (const uint16_t *)w, partial, ldp, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_bdcgs_step(const BatchBlocks &B, int R, int j, const double *dd, int ldd, double *Hf, long ldhp,
                             int ldc, double *pend, double *g, double *coef, int final_step, hipStream_t st) {
    const int np = B.nsys * R;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bdcgs_step, dim3(np), dim3(64), 0, st, j, R, dd, ldd, Hf, ldhp, ldc, pend, g, coef, final_step,
                       B.active);
    return hipGetLastError();
}

hipError_t launch_bupdate2(const BatchBlocks &B, int prec, int R, const void *V, long ldv, int ncols, const double *dd,
                           int ldd, const double *g, int ldc, const double *coef, void *u, const void *w, void *vout,
                           hipStream_t st) {
    if (ncols > kBDcgsMaxCols) return hipErrorInvalidValue;
    switch (prec) {
        case 0:
            return bupdate2_t<double>(B, R, (const double *)V, ldv, ncols, dd, ldd, g, ldc, coef, (double *)u,
                                      (const double *)w, (double *)vout, st);
        case 1:
            return bupdate2_t<float>(B, R, (const float *)V, ldv, ncols, dd, ldd, g, ldc, coef, (float *)u,
                                     (const float *)w, (float *)vout, st);
        case 2:
            return bupdate2_t<uint16_t>(B, R, (const uint16_t *)V, ldv, ncols, dd, ldd, g, ldc, coef, (uint16_t *)u,
                                        (const uint16_t *)w, (uint16_t *)vout, st);
    }
    return hipErrorInvalidValue;
}

int bdcgs_max_cols() { return kBDcgsMaxCols; }

hipError_t launch_bfinish(const BatchBlocks &B, int R, int ncols, const double *h2, int ldh, double *H, long pstride,
                          double *inv, hipStream_t st) {
    const int np = B.nsys * R;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bfinish, dim3((np + 63) / 64), dim3(64), 0, st, B.nsys, R, ncols, h2, ldh, H, pstride, inv);
    return hipGetLastError();
}

hipError_t launch_bnorm(const BatchBlocks &B, int R, const double *npart, double *H, long pstride, double *inv,
                        hipStream_t st) {
    const int np = B.nsys * R;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bnorm, dim3((np + 63) / 64), dim3(64), 0, st, B.boff, B.nsys, R, npart, H, pstride, inv);
    return hipGetLastError();
}

hipError_t launch_bscale(const BatchBlocks &B, int prec_in, int prec_out, int R, const void *in, const double *scale,
                         void *out, hipStream_t st) {
    switch (prec_in) {
        case 0:
            return bscale_in<double>(B, prec_out, R, (const double *)in, scale, out, st);
        case 1:
            return bscale_in<float>(B, prec_out, R, (const float *)in, scale, out, st);
        case 2:
            return bscale_in<uint16_t>(B, prec_out, R, (const uint16_t *)in, scale, out, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_bcombine(const BatchBlocks &B, int prec, int R, const void *V, long ldv, const int *k,
                           const double *z, int ldz, void *out, hipStream_t st) {
    switch (prec) {
        case 0:
            return bcombine_t<double>(B, R, (const double *)V, ldv, k, z, ldz, (double *)out, st);
        case 1:
            return bcombine_t<float>(B, R, (const float *)V, ldv, k, z, ldz, (float *)out, st);
        case 2:
            return bcombine_t<uint16_t>(B, R, (const uint16_t *)V, ldv, k, z, ldz, (uint16_t *)out, st);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Givens least squares of every pair, on the device: one thread per system
// runs its R pairs in order. The arithmetic is the host's GivensLS step for
// step (multiply-adds not contracted), so a cycle decides exactly as the
// host would.
// ---------------------------------------------------------------------------
namespace {

__global__ __launch_bounds__(256) void k_bgivens_init(BGivens G, const double *beta) {
    const int s = (int)(blockIdx.x * 256 + threadIdx.x);
    if (s >= G.nsys) return;
    int a = 0;
    for (int r = 0; r < G.R; ++r) {
        const int p = s * G.R + r;
        G.g[(size_t)p * (G.m + 1)] = beta[p];
        G.fro2[p] = 0.0;
        G.k[p] = 0;
        G.steps[p] = 0;
        a |= G.run[p];
    }
    G.act[s] = a;
}

__global__ __launch_bounds__(256) void k_bgivens_step(BGivens G, int j, const double *Hc, int ldh, double tol_brk) {
#pragma clang fp contract(off)
    const int s = (int)(blockIdx.x * 256 + threadIdx.x);
    if (s >= G.nsys) return;
    const int m = G.m, ld = m + 1;
    int a = 0;
    for (int r = 0; r < G.R; ++r) {
        const int p = s * G.R + r;
        if (!G.run[p]) continue;
        const double *h = Hc + (size_t)p * ldh;
        G.steps[p] += 1;
        bool finite = true;
        double f = G.fro2[p];
        for (int i = 0; i <= j + 1; ++i) {
            finite = finite && isfinite(h[i]);
            f += h[i] * h[i];
        }
        G.fro2[p] = f;
        if (!finite) {
            G.run[p] = 0;
            continue;
        }
        double *col = G.Rm + (size_t)p * ld * m + (size_t)j * ld;
        double *c = G.c + (size_t)p * m, *sn = G.s + (size_t)p * m, *g = G.g + (size_t)p * ld;
        for (int i = 0; i <= j + 1; ++i) col[i] = h[i];
        for (int i = 0; i < j; ++i) {
            const double t1 = c[i] * col[i] + sn[i] * col[i + 1];
            const double t2 = -sn[i] * col[i] + c[i] * col[i + 1];
            col[i] = t1;
            col[i + 1] = t2;
        }
        const double x = col[j], y = col[j + 1];
        double cj, sj;
        if (y == 0.0) {
            cj = 1.0;
            sj = 0.0;
        } else if (fabs(y) > fabs(x)) {
            const double tau = x / y;
            sj = 1.0 / sqrt(1.0 + tau * tau);
            cj = sj * tau;
        } else {
            const double tau = y / x;
            cj = 1.0 / sqrt(1.0 + tau * tau);
            sj = cj * tau;
        }
        c[j] = cj;
        sn[j] = sj;
        col[j] = cj * x + sj * y;
        col[j + 1] = 0.0;
        g[j + 1] = -sj * g[j];
        g[j] = cj * g[j];
        G.k[p] = j + 1;
        const double sc = fabs(g[j + 1]);
        G.sc[p] = sc;
        if (h[j + 1] <= tol_brk * sqrt(f) || sc <= G.target[p])
            G.run[p] = 0;
        else
            a = 1;
    }
    G.act[s] = a;
}

__global__ __launch_bounds__(256) void k_bgivens_solve(BGivens G, double *z, int ldz) {
#pragma clang fp contract(off)
    const int p = (int)(blockIdx.x * 256 + threadIdx.x);
    if (p >= G.nsys * G.R) return;
    const int k = G.k[p], ld = G.m + 1;
    const double *Rm = G.Rm + (size_t)p * ld * G.m, *g = G.g + (size_t)p * ld;
    double *zp = z + (size_t)p * ldz;
    for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int q = i + 1; q < k; ++q) t -= Rm[(size_t)i + (size_t)q * ld] * zp[q];
        zp[i] = t / Rm[(size_t)i + (size_t)i * ld];
    }
}

// flag[0] = 1 if some system still has a running pair, else 0 (one workgroup)
__global__ __launch_bounds__(256) void k_bany(const int *act, int nsys, int *flag) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int a = 0;
    for (int s = (int)threadIdx.x; s < nsys; s += 256) a |= act[s];
    if (a) any = 1;
    __syncthreads();
    if (threadIdx.x == 0) flag[0] = any;
}

}  // namespace

hipError_t launch_bany(const int *act, int nsys, int *flag, hipStream_t st) {
    hipLaunchKernelGGL(k_bany, dim3(1), dim3(256), 0, st, act, nsys, flag);
    return hipGetLastError();
}

hipError_t launch_bgivens_init(const BGivens &G, const double *beta, hipStream_t st) {
    if (G.nsys <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bgivens_init, dim3((G.nsys + 255) / 256), dim3(256), 0, st, G, beta);
    return hipGetLastError();
}

hipError_t launch_bgivens_step(const BGivens &G, int j, const double *Hc, int ldh, double tol_brk, hipStream_t st) {
    if (G.nsys <= 0) return hipSuccess;
    if (j < 0 || j >= G.m || ldh < j + 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bgivens_step, dim3((G.nsys + 255) / 256), dim3(256), 0, st, G, j, Hc, ldh, tol_brk);
    return hipGetLastError();
}

hipError_t launch_bgivens_solve(const BGivens &G, double *z, int ldz, hipStream_t st) {
    const int P = G.nsys * G.R;
    if (P <= 0) return hipSuccess;
    if (ldz < G.m) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bgivens_solve, dim3((P + 255) / 256), dim3(256), 0, st, G, z, ldz);
    return hipGetLastError();
}

}  // namespace ppg
