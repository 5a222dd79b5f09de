// Wavefront (64 lanes) and workgroup primitives for gfx950.
#pragma once

#include "internal.h"

namespace spg {

// Device memory named through a pointer read from memory (a problem's arrays)
// is reached with flat instructions unless the type says it is global. Flat
// loads and stores also count against the LDS wait counter, so every LDS read
// after them waits for them to complete; through a gmem pointer they are
// global memory instructions, and LDS work overlaps the gathers in flight.
template <typename T>
using gmem = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ gmem<T> *to_gmem(T *p) {
    return (gmem<T> *)p;
}

// two consecutive ints at 4-byte alignment (a column pointer and the next one)
typedef int int2a __attribute__((ext_vector_type(2), aligned(4)));

// p[i] and p[i + 1] in one 8-byte load; the caller keeps i + 1 inside the array
__device__ __forceinline__ int2a load_pair(const int32_t *p, long long i) {
    return *(const gmem<const int2a> *)((const gmem<const int32_t> *)p + i);
}

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ unsigned long long ballot(bool p) {
    return __builtin_amdgcn_ballot_w64(p);
}

// lanes below this one
__device__ __forceinline__ unsigned long long mask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ int popc64(unsigned long long x) { return __builtin_popcountll(x); }

// value of lane `src` (any lane pattern) through the LDS crossbar
__device__ __forceinline__ int shfl_idx(int v, int src) {
    return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

// XOR butterfly exchange inside the wavefront. Distances 1 and 2 stay in a
// quad (DPP quad_perm), 4..16 use ds_swizzle's bit-mask mode inside 32-lane
// halves, 32 crosses halves through ds_bpermute.
template <int J>
__device__ __forceinline__ int shfl_xor_c(int v) {
    if constexpr (J == 1) {
        // quad_perm [1,0,3,2]
        return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
    } else if constexpr (J == 2) {
        // quad_perm [2,3,0,1]
        return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
    } else if constexpr (J >= 4 && J <= 16) {
        // bit-mask mode: and_mask = 0x1f, or_mask = 0, xor_mask = J
        return __builtin_amdgcn_ds_swizzle(v, (J << 10) | 0x1F);
    } else {
        return __builtin_amdgcn_ds_bpermute((lane_id() ^ J) << 2, v);
    }
}

template <int J>
__device__ __forceinline__ unsigned long long shfl_xor_c64(unsigned long long v) {
    int lo = (int)(unsigned)v, hi = (int)(unsigned)(v >> 32);
    lo = shfl_xor_c<J>(lo);
    hi = shfl_xor_c<J>(hi);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

__device__ __forceinline__ int shfl_up1_or(int v, int d, int fill) {
    int l = lane_id();
    int t = __builtin_amdgcn_ds_bpermute((l - d) << 2, v);
    return l >= d ? t : fill;
}

// inclusive prefix sum over the wavefront
__device__ __forceinline__ int wave_incl_scan(int v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) v += shfl_up1_or(v, d, 0);
    return v;
}

__device__ __forceinline__ int wave_bcast(int v, int src) { return shfl_idx(v, src); }

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __builtin_amdgcn_ds_bpermute((lane_id() ^ d) << 2, v);
    return v;
}

// Exclusive prefix sum over a workgroup of kBlock threads. `tmp` holds
// kBlock / 64 + 1 ints of LDS. Returns the exclusive prefix; `total` gets the
// workgroup sum. Contains barriers: every thread must call it.
__device__ __forceinline__ int block_excl_scan(int v, int *tmp, int &total) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    int inc = wave_incl_scan(v);
    if (l == 63) tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int i = 0; i < kBlock / 64; ++i) {
            int x = tmp[i];
            tmp[i] = run;
            run += x;
        }
        tmp[kBlock / 64] = run;
    }
    __syncthreads();
    int ex = tmp[w] + inc - v;
    total = tmp[kBlock / 64];
    __syncthreads();
    return ex;
}

// Exclusive prefix over a workgroup of T threads; `tmp` holds T / 64 + 1 ints
// of LDS; `total` gets the workgroup sum. Contains barriers: every thread must
// call it.
template <int T>
__device__ __forceinline__ int wg_excl_scan(int v, int *tmp, int &total) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    int inc = wave_incl_scan(v);
    if (l == 63) tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int i = 0; i < T / 64; ++i) {
            int x = tmp[i];
            tmp[i] = run;
            run += x;
        }
        tmp[T / 64] = run;
    }
    __syncthreads();
    int ex = tmp[w] + inc - v;
    total = tmp[T / 64];
    __syncthreads();
    return ex;
}

// Largest index i in [0, n) with a[i] <= x, for non-decreasing a with a[0] <= x.
__device__ __forceinline__ int last_le(const int *a, int n, int x) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int ceil_log2(int x) {  // x >= 1
    return x <= 1 ? 0 : 32 - __builtin_clz((unsigned)(x - 1));
}

}  // namespace spg
