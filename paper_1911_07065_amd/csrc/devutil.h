// Device helpers shared by the kernel files (internal): element access for
// double / float / bfloat16-bits storage, reductions, XCD-aware order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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

// A double's sum over the wave, valid in every lane: within each row of 16
// lanes by DPP moves (a VALU operation per half: lane ^ 1 and lane ^ 2
// through quad permutations, then rotations by 4 and 8 lanes), then across
// the four rows by two lane exchanges. Fixed order, so repeated sums are
// identical.
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_double<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_double<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_double<0x124>(v);  // row_ror 4
    v += dpp_double<0x128>(v);  // row_ror 8
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
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


}  // namespace
}  // namespace ppg
