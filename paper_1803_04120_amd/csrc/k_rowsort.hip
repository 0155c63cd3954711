// Result rows to sorted (i, j) pairs.
//
// After the fill pass every result row i (all j within eps of point i)
// occupies its own contiguous segment, in candidate order. Sorting each
// segment by j and writing (i, j) gives the key/value result sorted by key
// and value (Section IV-E sorts the key/value pairs after the kernel), and
// because rows are laid out in order of i the whole result is sorted by
// (i, j) without any global sort.
//
// Rows are sorted by size class:
//   <= 64     one wave, one element per lane, bitonic network over lanes
//   <= 1024   one wave, bitonic network in the wave's LDS slot
//   <= 16384  one workgroup, bitonic network in 64 KiB of LDS
//   larger    one workgroup, bitonic network in global memory, using the
//             row's own output segment (twice the row's size) as scratch
// j values within a row are distinct, so no stability is needed.
#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kWaveCap = 1024;
constexpr uint32_t kBlockCap = 16384;
constexpr uint32_t kPad = 0xffffffffu;

__device__ __forceinline__ uint32_t next_pow2(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// One compare-exchange step of the bitonic network over N elements
// (pair index q in [0, N/2)).
__device__ __forceinline__ void bitonic_pair(uint32_t q, uint32_t j, uint32_t k, uint32_t &lo,
                                             uint32_t &hi, bool &asc) {
    lo = 2 * j * (q / j) + (q % j);
    hi = lo + j;
    asc = (lo & k) == 0;
}

__device__ __forceinline__ void write_pairs(uint2 *__restrict__ out, uint64_t at, uint32_t row,
                                            uint32_t j) {
    out[at] = make_uint2(row, j);
}

__global__ __launch_bounds__(kThreads) void k_rowsort_small(const uint64_t *__restrict__ off,
                                                             uint64_t i0, uint64_t i1,
                                                             uint64_t base,
                                                             const uint32_t *__restrict__ out_j,
                                                             uint2 *__restrict__ pairs,
                                                             uint32_t *__restrict__ big_list,
                                                             uint32_t *__restrict__ big_count) {
    __shared__ uint32_t slot[kWaves][kWaveCap];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const uint64_t row = i0 + static_cast<uint64_t>(blockIdx.x) * kWaves + wave;
    if (row >= i1) return;
    const uint64_t s = off[row] - base;
    const uint32_t len = static_cast<uint32_t>(off[row + 1] - off[row]);
    if (len <= 64) {
        uint32_t v = lane < static_cast<int>(len) ? out_j[s + lane] : kPad;
#pragma unroll
        for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                const uint32_t p = __shfl_xor(v, j, 64);
                const bool up = (lane & k) == 0;
                const bool lower = (lane & j) == 0;
                const uint32_t mn = v < p ? v : p, mx = v < p ? p : v;
                v = (lower == up) ? mn : mx;
            }
        }
        if (lane < static_cast<int>(len)) write_pairs(pairs, s + lane, static_cast<uint32_t>(row), v);
        return;
    }
    if (len <= kWaveCap) {
        volatile uint32_t *sh = slot[wave];
        const uint32_t N = next_pow2(len);
        for (uint32_t e = lane; e < N; e += 64) sh[e] = e < len ? out_j[s + e] : kPad;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t k = 2; k <= N; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t q = lane; q < N / 2; q += 64) {
                    uint32_t lo, hi;
                    bool asc;
                    bitonic_pair(q, j, k, lo, hi, asc);
                    const uint32_t a = sh[lo], b = sh[hi];
                    if ((a > b) == asc) {
                        sh[lo] = b;
                        sh[hi] = a;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        for (uint32_t e = lane; e < len; e += 64) write_pairs(pairs, s + e, static_cast<uint32_t>(row), sh[e]);
        return;
    }
    if (lane == 0) {
        const uint32_t at = atomicAdd(big_count, 1u);
        big_list[at] = static_cast<uint32_t>(row - i0);
    }
}

__global__ __launch_bounds__(kThreads) void k_rowsort_big(const uint64_t *__restrict__ off,
                                                           uint64_t i0, uint64_t base,
                                                           uint32_t *__restrict__ out_j,
                                                           uint2 *__restrict__ pairs,
                                                           const uint32_t *__restrict__ big_list,
                                                           const uint32_t *__restrict__ big_count) {
    __shared__ uint32_t sh[kBlockCap];
    const uint32_t nbig = *big_count;
    for (uint32_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const uint64_t row = i0 + big_list[b];
        const uint64_t s = off[row] - base;
        const uint32_t len = static_cast<uint32_t>(off[row + 1] - off[row]);
        const uint32_t N = next_pow2(len);
        if (N <= kBlockCap) {
            for (uint32_t e = threadIdx.x; e < N; e += kThreads) sh[e] = e < len ? out_j[s + e] : kPad;
            __syncthreads();
            for (uint32_t k = 2; k <= N; k <<= 1) {
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    for (uint32_t q = threadIdx.x; q < N / 2; q += kThreads) {
                        uint32_t lo, hi;
                        bool asc;
                        bitonic_pair(q, j, k, lo, hi, asc);
                        const uint32_t a = sh[lo], c = sh[hi];
                        if ((a > c) == asc) {
                            sh[lo] = c;
                            sh[hi] = a;
                        }
                    }
                    __syncthreads();
                }
            }
            for (uint32_t e = threadIdx.x; e < len; e += kThreads)
                write_pairs(pairs, s + e, static_cast<uint32_t>(row), sh[e]);
            __syncthreads();
            continue;
        }
        // Global-memory network; the row's pair segment (2 * len words >= N)
        // is the scratch array.
        uint32_t *T = reinterpret_cast<uint32_t *>(pairs + s);
        for (uint32_t e = threadIdx.x; e < N; e += kThreads) T[e] = e < len ? out_j[s + e] : kPad;
        __threadfence();
        __syncthreads();
        for (uint32_t k = 2; k <= N; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t q = threadIdx.x; q < N / 2; q += kThreads) {
                    uint32_t lo, hi;
                    bool asc;
                    bitonic_pair(q, j, k, lo, hi, asc);
                    const uint32_t a = T[lo], c = T[hi];
                    if ((a > c) == asc) {
                        T[lo] = c;
                        T[hi] = a;
                    }
                }
                __threadfence();
                __syncthreads();
            }
        }
        for (uint32_t e = threadIdx.x; e < len; e += kThreads) out_j[s + e] = T[e];
        __threadfence();
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < len; e += kThreads)
            write_pairs(pairs, s + e, static_cast<uint32_t>(row), out_j[s + e]);
        __syncthreads();
    }
}

__global__ void k_zero1(uint32_t *p) {
    if (threadIdx.x == 0) *p = 0;
}

}  // namespace

void launch_rowsort(const uint64_t *off, uint64_t i0, uint64_t i1, uint64_t base, uint32_t *out_j,
                    uint32_t *pairs, uint32_t *big_list, uint32_t *big_count, hipStream_t s) {
    if (i1 <= i0) return;
    const uint64_t rows = i1 - i0;
    k_zero1<<<1, 64, 0, s>>>(big_count);
    SJ_LAUNCH_CHECK();
    const uint64_t nb = (rows + kWaves - 1) / kWaves;
    if (nb > 0x7fffffffULL) throw Error(SJ_EINVAL, "row sort: too many rows");
    uint2 *p2 = reinterpret_cast<uint2 *>(pairs);
    {
        KTimer kt_("rowsort_small", s);
        k_rowsort_small<<<static_cast<unsigned>(nb), kThreads, 0, s>>>(off, i0, i1, base, out_j, p2,
                                                                       big_list, big_count);
        SJ_LAUNCH_CHECK();
    }
    {
        KTimer kt_("rowsort_big", s);
        k_rowsort_big<<<512, kThreads, 0, s>>>(off, i0, base, out_j, p2, big_list, big_count);
        SJ_LAUNCH_CHECK();
    }
}

}  // namespace sj
