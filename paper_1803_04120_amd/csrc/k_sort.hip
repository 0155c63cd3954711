// Stable LSD radix sort of (cell id, point id) pairs: builds the point map A
// of Section IV-C (points ordered by linearised cell id, ties by point id).
//
// Passes over digits of RB = 8 or 9 bits (9 when it saves a pass):
//   upsweep   - per-tile digit histogram (LDS atomics), digit-major table;
//   scan      - exclusive scan of the table (digit-major, tile-minor) gives
//               each (digit, tile) its first output slot;
//   downsweep - per tile, a stable rank of every key within its digit using
//               wave64 ballots (RB ballots give the lanes with an equal
//               digit), per-wave running counts in LDS, and a block prefix;
//               keys are staged in LDS in digit order so the global writes of
//               one digit run are contiguous.
#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = 8;                 // per lane
constexpr int kTile = kThreads * kItems;  // 2048 keys per workgroup

template <typename K, int RB>
__global__ __launch_bounds__(kThreads) void k_upsweep(const K *__restrict__ keys, size_t n,
                                                       int shift, uint32_t *__restrict__ hist,
                                                       uint32_t ntiles) {
    constexpr int R = 1 << RB;
    __shared__ uint32_t h[kWaves][R];
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kWaves * R; i += kThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const size_t base = static_cast<size_t>(blockIdx.x) * kTile;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const size_t i = base + static_cast<size_t>(k) * kThreads + threadIdx.x;
        if (i < n) {
            const uint32_t dgt = static_cast<uint32_t>(keys[i] >> shift) & (R - 1);
            atomicAdd(&h[wave][dgt], 1u);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < R; t += kThreads) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += h[w][t];
        hist[static_cast<size_t>(t) * ntiles + blockIdx.x] = s;
    }
}

template <typename K, int RB>
__global__ __launch_bounds__(kThreads) void k_downsweep(const K *__restrict__ kin,
                                                         const uint32_t *__restrict__ vin,
                                                         K *__restrict__ kout,
                                                         uint32_t *__restrict__ vout, size_t n,
                                                         int shift,
                                                         const uint32_t *__restrict__ hist_scan,
                                                         uint32_t ntiles) {
    constexpr int R = 1 << RB;
    constexpr int kPerThread = R / kThreads;  // digits per thread in the block prefix
    __shared__ uint32_t wcnt[kWaves][R];
    __shared__ uint32_t doff[R];
    __shared__ uint32_t gbase[R];
    __shared__ uint32_t lds_scan[kWaves];
    __shared__ K skey[kTile];
    __shared__ uint32_t sval[kTile];

    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    for (int i = threadIdx.x; i < kWaves * R; i += kThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    const size_t base = static_cast<size_t>(blockIdx.x) * kTile;
    const uint32_t count =
        static_cast<uint32_t>((n - base) < static_cast<size_t>(kTile) ? (n - base) : kTile);

    K key[kItems];
    uint32_t val[kItems];
    uint32_t rank[kItems];
    uint32_t dig[kItems];
    volatile uint32_t *my_cnt = wcnt[wave];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t local = static_cast<uint32_t>(wave * (kItems * 64) + k * 64 + lane);
        const bool valid = local < count;
        key[k] = valid ? kin[base + local] : K(0);
        val[k] = valid ? vin[base + local] : 0u;
        const uint32_t dg = static_cast<uint32_t>(key[k] >> shift) & (R - 1);
        dig[k] = dg;
        uint64_t m = ballot(valid);
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t bb = ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t below = mbcnt(m);
        const uint32_t same = static_cast<uint32_t>(__popcll(m));
        uint32_t pre = 0;
        if (valid) pre = my_cnt[dg];
        rank[k] = pre + below;
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) my_cnt[dg] = pre + same;
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // wave prefixes per digit, block digit offsets, global bases; thread t
    // owns digits [t * kPerThread, (t + 1) * kPerThread)
    {
        uint32_t tot_d[kPerThread];
        uint32_t mine = 0;
#pragma unroll
        for (int q = 0; q < kPerThread; ++q) {
            const int t = threadIdx.x * kPerThread + q;
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wcnt[w][t];
                wcnt[w][t] = run;
                run += c;
            }
            tot_d[q] = run;
            mine += run;
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_scan<uint32_t, kThreads>(mine, &tot, lds_scan);
#pragma unroll
        for (int q = 0; q < kPerThread; ++q) {
            const int t = threadIdx.x * kPerThread + q;
            doff[t] = ex;
            ex += tot_d[q];
            gbase[t] = hist_scan[static_cast<size_t>(t) * ntiles + blockIdx.x];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t local = static_cast<uint32_t>(wave * (kItems * 64) + k * 64 + lane);
        if (local < count) {
            const uint32_t pos = doff[dig[k]] + wcnt[wave][dig[k]] + rank[k];
            skey[pos] = key[k];
            sval[pos] = val[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t i = static_cast<uint32_t>(k * kThreads + threadIdx.x);
        if (i < count) {
            const K kk = skey[i];
            const uint32_t dg = static_cast<uint32_t>(kk >> shift) & (R - 1);
            const size_t o = static_cast<size_t>(gbase[dg]) + (i - doff[dg]);
            kout[o] = kk;
            vout[o] = sval[i];
        }
    }
}

template <typename K, int RB>
void radix_pass(const K *kin, const uint32_t *vin, K *kout, uint32_t *vout, size_t n, int shift,
                uint32_t *hist, uint32_t ntiles, hipStream_t s) {
    {
        KTimer kt_("radix_upsweep", s);
        k_upsweep<K, RB><<<ntiles, kThreads, 0, s>>>(kin, n, shift, hist, ntiles);
        SJ_LAUNCH_CHECK();
    }
    scan_exclusive_u32(hist, hist, static_cast<size_t>(1u << RB) * ntiles, s);
    {
        KTimer kt_("radix_downsweep", s);
        k_downsweep<K, RB><<<ntiles, kThreads, 0, s>>>(kin, vin, kout, vout, n, shift, hist, ntiles);
        SJ_LAUNCH_CHECK();
    }
}

// Digit width for `bits` significant bits: 9-bit digits when they save a
// pass over 8-bit ones (17 or 18 bits), else 8. Wider digits were measured
// slower: a 10- or 11-bit downsweep holds 40-70 KiB of LDS per workgroup and
// runs at 2-3 waves per SIMD, and its digit table scan grows with the radix.
int digit_bits(int bits) {
    return (bits > 16 && bits <= 18) ? 9 : 8;
}

template <typename K>
bool radix_sort_impl(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, size_t n,
                     int bits, hipStream_t s) {
    if (n <= 1 || bits <= 0) return false;
    if (n >= 0xffffffffULL) throw Error(SJ_EINVAL, "radix sort: too many keys");
    const uint32_t ntiles = static_cast<uint32_t>((n + kTile - 1) / kTile);
    const int rb = digit_bits(bits);
    DevBuf<uint32_t> hist((static_cast<size_t>(1) << rb) * ntiles);
    K *src_k = keys, *dst_k = keys_alt;
    uint32_t *src_v = vals, *dst_v = vals_alt;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += rb) {
        switch (rb) {
            case 8: radix_pass<K, 8>(src_k, src_v, dst_k, dst_v, n, shift, hist.ptr, ntiles, s); break;
            case 9: radix_pass<K, 9>(src_k, src_v, dst_k, dst_v, n, shift, hist.ptr, ntiles, s); break;
            default: throw Error(SJ_EINVAL, "radix sort: digit width");
        }
        std::swap(src_k, dst_k);
        std::swap(src_v, dst_v);
        ++passes;
    }
    return (passes & 1) != 0;
}

}  // namespace

bool radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                    size_t n, int bits, hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n, bits, s);
}

bool radix_sort_u32(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                    size_t n, int bits, hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, s);
}

}  // namespace sj
