// Device helpers shared by the kernel files: complex arithmetic on native
// 2-vectors, streaming loads/stores, bit insertion, fixed-order reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "qv_internal.h"

namespace qv {

template <typename T> struct RealOf;
template <> struct RealOf<d2> { using type = double; };
template <> struct RealOf<f2> { using type = float; };

constexpr int kThreads = 256;

// ------------------------------------------------------------- helpers ---

template <typename T>
__device__ __forceinline__ T cmul(T a, T b)
{
    T r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// u0 * x + u1 * y
template <typename T>
__device__ __forceinline__ T cmul2(T u0, T x, T u1, T y)
{
    T r;
    r.x = u0.x * x.x - u0.y * x.y + u1.x * y.x - u1.y * y.y;
    r.y = u0.x * x.y + u0.y * x.x + u1.x * y.y + u1.y * y.x;
    return r;
}

// u0 x0 + u1 x1 + u2 x2 + u3 x3 as one multiply-add chain per component
// (a row of a 4x4 update)
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__device__ __forceinline__ T cdot4(T u0, T x0, T u1, T x1, T u2, T x2, T u3, T x3)
{
    T r;
    r.x = u0.x * x0.x;
    r.y = u0.x * x0.y;
    r.x = fma_(-u0.y, x0.y, r.x);
    r.y = fma_(u0.y, x0.x, r.y);
    r.x = fma_(u1.x, x1.x, r.x);
    r.y = fma_(u1.x, x1.y, r.y);
    r.x = fma_(-u1.y, x1.y, r.x);
    r.y = fma_(u1.y, x1.x, r.y);
    r.x = fma_(u2.x, x2.x, r.x);
    r.y = fma_(u2.x, x2.y, r.y);
    r.x = fma_(-u2.y, x2.y, r.x);
    r.y = fma_(u2.y, x2.x, r.y);
    r.x = fma_(u3.x, x3.x, r.x);
    r.y = fma_(u3.x, x3.y, r.y);
    r.x = fma_(-u3.y, x3.y, r.x);
    r.y = fma_(u3.y, x3.x, r.y);
    return r;
}

template <typename T>
__device__ __forceinline__ T ld_nt(const T* p)
{
    return __builtin_nontemporal_load(p);
}

template <typename T>
__device__ __forceinline__ void st_nt(T* p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// Insert a zero bit at each position of pos[0..cnt) (ascending final
// positions) into v.
struct Ins {
    int cnt;
    int pos[5];
};

__device__ __forceinline__ uint64_t insert_zeros(uint64_t v, const Ins& ins)
{
#pragma unroll
    for (int j = 0; j < 5; j++) {
        if (j < ins.cnt) {
            const int p = ins.pos[j];
            const uint64_t lo = v & ((1ull << p) - 1);
            v = ((v >> p) << (p + 1)) | lo;
        }
    }
    return v;
}

inline Ins make_ins(uint64_t mask)
{
    Ins r{};
    r.cnt = 0;
    for (int q = 0; q < 64 && mask; q++) {
        if (mask & (1ull << q)) {
            r.pos[r.cnt++] = q;
            mask &= ~(1ull << q);
        }
    }
    return r;
}

template <typename T>
inline T to_dev(cd v)
{
    T r;
    r.x = (typename RealOf<T>::type)v.real();
    r.y = (typename RealOf<T>::type)v.imag();
    return r;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Cross-lane move of a double with a DPP pattern; lanes of rows left out by
// ROW_MASK get 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, ROW_MASK, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes of a wave in a fixed order, returned to every lane
// (uniform). Every lane must be active. Pairs, quads, half-rows and rows
// combine through DPP lane patterns, then row sums move across rows with the
// row broadcasts; lane 63 ends with the total.
__device__ __forceinline__ double wave_total(double v)
{
    v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_move<0x140, 0xF>(v);  // row_mirror
    v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0x8>(v);  // row_bcast:31 into row 3
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, 63);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide sum in a fixed order (waves reduced by shuffles, then wave 0
// adds the per-wave results in index order). Result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) t += red[i];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double block_max(double v, double* red)
{
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) t = fmax(t, red[i]);
    __syncthreads();
    return t;
}


}  // namespace qv
