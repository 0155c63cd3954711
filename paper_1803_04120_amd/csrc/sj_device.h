// Wave64 / workgroup helpers for gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sj {

__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x & 63u); }

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T y = __shfl_up(v, off, 64);
        if (lane >= off) v += y;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const T y = __shfl_xor(v, off, 64);
        v = y > v ? y : v;
    }
    return v;
}

// Exclusive prefix of one value per thread over a workgroup of kThreads
// (multiple of 64). *total receives the workgroup sum. `lds` holds
// kThreads/64 values. Contains two barriers; every thread must call it.
template <typename T, int kThreads>
__device__ __forceinline__ T block_exclusive_scan(T v, T *total, T *lds) {
    const int lane = lane_id();
    const int wave = static_cast<int>(threadIdx.x >> 6);
    const T incl = wave_inclusive_scan(v);
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        const T x = lds[w];
        if (w < wave) before += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

// Sorts one 64-entry row per 16-lane group (4 rows per wave): lane l of a
// group holds entries e = 16 k + l in v[k], k = 0..3. Bitonic network: stages
// with a partner distance of 16 or more exchange registers within the lane,
// shorter ones exchange with lane l ^ j of the same group. Every lane of the
// wave must take part.
// The value x of lane (lane ^ m). Partners inside the lane's 16-lane row
// are DPP moves, plain VALU operations: quad permutations for m = 1, 2, 3,
// the 8- and 16-lane mirrors for m = 7, 15, and for m = 4, 8 the row shift
// towards the partner (by 4 or 8 lanes up or down). Any other m goes
// through the LDS crossbar. Every lane of the wave must take part; m is a
// constant after unrolling.
__device__ __forceinline__ uint32_t lane_xor(uint32_t x, int m) {
    const int xi = static_cast<int>(x);
    const uint32_t lane = static_cast<uint32_t>(lane_id());
    switch (m) {
        case 1: return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(xi, 0xB1, 0xF, 0xF, true));  // [1,0,3,2]
        case 2: return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(xi, 0x4E, 0xF, 0xF, true));  // [2,3,0,1]
        case 3: return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(xi, 0x1B, 0xF, 0xF, true));  // [3,2,1,0]
        case 4: {
            const int up = __builtin_amdgcn_mov_dpp(xi, 0x104, 0xF, 0xF, true);  // row_shl:4, lane + 4
            const int dn = __builtin_amdgcn_mov_dpp(xi, 0x114, 0xF, 0xF, true);  // row_shr:4, lane - 4
            return static_cast<uint32_t>((lane & 4u) ? dn : up);
        }
        case 7: return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(xi, 0x141, 0xF, 0xF, true));  // half mirror
        case 8: {
            const int up = __builtin_amdgcn_mov_dpp(xi, 0x108, 0xF, 0xF, true);  // row_shl:8, lane + 8
            const int dn = __builtin_amdgcn_mov_dpp(xi, 0x118, 0xF, 0xF, true);  // row_shr:8, lane - 8
            return static_cast<uint32_t>((lane & 8u) ? dn : up);
        }
        case 15: return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(xi, 0x140, 0xF, 0xF, true));  // mirror
        default: return static_cast<uint32_t>(__shfl_xor(xi, m, 64));
    }
}

__device__ __forceinline__ void group16_bitonic64(uint32_t (&v)[4]) {
    const uint32_t l = static_cast<uint32_t>(lane_id()) & 15u;
#pragma unroll
    for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= 16) {
                const int jr = j >> 4;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int kp = k ^ jr;
                    if (kp > k) {
                        const uint32_t e = static_cast<uint32_t>(k) * 16 + l;
                        const bool asc = (e & static_cast<uint32_t>(kk)) == 0;
                        const uint32_t a = v[k], b = v[kp];
                        const uint32_t mn = a < b ? a : b, mx = a < b ? b : a;
                        v[k] = asc ? mn : mx;
                        v[kp] = asc ? mx : mn;
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t p = lane_xor(v[k], j);
                    const uint32_t e = static_cast<uint32_t>(k) * 16 + l;
                    const bool asc = (e & static_cast<uint32_t>(kk)) == 0;
                    const bool lower = (l & static_cast<uint32_t>(j)) == 0;
                    const uint32_t mn = v[k] < p ? v[k] : p, mx = v[k] < p ? p : v[k];
                    v[k] = (lower == asc) ? mn : mx;
                }
            }
        }
    }
}

// Sorts the first W of N values held in registers ascending with a fully
// unrolled bitonic network (W a power of two; all register indices are
// compile-time constants). The stages of the N-wide network up to width W,
// restricted to the first W entries, leave those sorted ascending.
template <int W, int N>
__device__ __forceinline__ void register_bitonic_first(uint32_t (&v)[N]) {
    static_assert(W <= N && (W & (W - 1)) == 0, "sort width");
#pragma unroll
    for (int k = 2; k <= W; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < W; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const uint32_t a = v[i], b = v[l];
                    const uint32_t mn = a < b ? a : b, mx = a < b ? b : a;
                    if ((i & k) == 0) {
                        v[i] = mn;
                        v[l] = mx;
                    } else {
                        v[i] = mx;
                        v[l] = mn;
                    }
                }
            }
        }
    }
}

template <int N>
__device__ __forceinline__ void register_bitonic(uint32_t (&v)[N]) {
    register_bitonic_first<N, N>(v);
}

// Counters that many workgroups add to are spread over kCounterSlots
// addresses, one 128-byte line apart, so the additions do not serialise on a
// single L2 line; the host sums the slots.
constexpr int kCounterSlots = 256;
constexpr int kCounterStride = 16;  // u64 per slot (128 bytes)

// Adds a per-lane value to counter slot (block % slots): wave sum, then one
// atomic per wave. Every lane of the wave must call it.
__device__ __forceinline__ void add_counter(unsigned long long *slots, uint32_t v) {
    const unsigned long long s = wave_sum<unsigned long long>(v);
    if (lane_id() == 0 && s)
        atomicAdd(slots + static_cast<size_t>(blockIdx.x % kCounterSlots) * kCounterStride, s);
}

}  // namespace sj
