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
//   <= 32     one lane per row: the row is loaded into 16 or 32 registers
//             (16 when no row is longer) and sorted by a fully unrolled
//             bitonic network (static register indices, v_min/v_max only)
//   <= 64     16 lanes per row, 4 registers each, bitonic network over
//             registers and 16-lane shuffles (queued rows only)
//   <= 1024   one wave per row, bitonic network in the wave's LDS slot
//   <= 16384  one workgroup per row, bitonic network in 64 KiB of LDS
//   larger    one workgroup per row, bitonic network in global memory, using
//             the row's own output segment (twice the row's size) as scratch
// No kernel appends rows to a shared queue (a queue counter is one address
// that every producer hits). The 33..64 class is found by scanning the row
// offsets (64 rows per wave and ballot). Rows longer than 64 are listed in
// row order by a stream compaction (a scan of the long-row flags) and the
// wave and workgroup kernels walk that list, so the long rows of a dense
// cluster -- adjacent in cell order -- spread over all waves.
//
// Row r's neighbour ids are read from out_j[in_off[r] - in_base, +len) and
// its pairs are written at pairs[out_off[id] - out_base, +len) with
// id = perm ? perm[r] : r0 + r. A whole result is filled in cell order (the
// rows of one wave's points are adjacent, so the fill writes and these reads
// are contiguous) and scattered to the rows' places in order of i here;
// batches are filled directly in order of i (in_off = out_off).
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

struct RowMap {
    const uint64_t *in_off;
    uint64_t in_base;
    const uint64_t *out_off;
    uint64_t out_base;
    const uint32_t *perm;
    uint64_t r0;
    uint64_t rows;
};

struct RowRef {
    uint64_t in, out;
    uint32_t len, id;
};

__device__ __forceinline__ RowRef row_ref(const RowMap &m, uint64_t r) {
    RowRef x;
    x.in = m.in_off[r] - m.in_base;
    x.len = static_cast<uint32_t>(m.in_off[r + 1] - m.in_off[r]);
    const uint64_t id = m.perm ? m.perm[r] : m.r0 + r;
    x.id = static_cast<uint32_t>(id);
    x.out = m.out_off[id] - m.out_base;
    return x;
}

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

template <int N>
__global__ __launch_bounds__(kThreads) void k_rowsort_lane(RowMap m, const uint32_t *__restrict__ out_j,
                                                            uint2 *__restrict__ pairs) {
    const uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r >= m.rows) return;
    const uint32_t len = static_cast<uint32_t>(m.in_off[r + 1] - m.in_off[r]);
    if (len > static_cast<uint32_t>(N)) return;  // a longer-row kernel sorts it
    const RowRef x = row_ref(m, r);
    uint32_t v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = static_cast<uint32_t>(k) < x.len ? out_j[x.in + k] : kPad;
    register_bitonic<N>(v);
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (static_cast<uint32_t>(k) < x.len) pairs[x.out + k] = make_uint2(x.id, v[k]);
}

// Rows of 64 consecutive row indices per wave: the mask of those whose
// length lies in (lo, hi]. Uniform across the wave.
__device__ __forceinline__ uint64_t class_mask(const RowMap &m, uint64_t base, uint32_t lo, uint32_t hi) {
    const uint64_t r = base + static_cast<uint64_t>(lane_id());
    uint32_t len = 0;
    if (r < m.rows) len = static_cast<uint32_t>(m.in_off[r + 1] - m.in_off[r]);
    return ballot(len > lo && len <= hi);
}

// Rows of up to 64 entries, 16 lanes per row (4 rows per wave): lane l holds
// elements e = 16 k + l, k = 0..3; bitonic stages with a partner distance of
// 16 or more exchange registers within the lane, shorter ones exchange with
// lane l ^ j of the same 16-lane group. Each row is read and written by 16
// consecutive lanes at consecutive addresses.
__global__ __launch_bounds__(kThreads) void k_rowsort_group16(RowMap m, const uint32_t *__restrict__ out_j,
                                                               uint2 *__restrict__ pairs, uint32_t lo) {
    const uint32_t l = threadIdx.x & 15u;
    const uint32_t grp = (threadIdx.x >> 4) & 3u;  // 16-lane group within the wave
    const uint64_t waves = static_cast<uint64_t>(gridDim.x) * kWaves;
    for (uint64_t base = (blockIdx.x * static_cast<uint64_t>(kWaves) + (threadIdx.x >> 6)) * 64; base < m.rows;
         base += waves * 64) {
    uint64_t mask = class_mask(m, base, lo, 64);
    // four rows of the class per pass, one per 16-lane group; the loop is
    // uniform across the wave, so every group takes part in every shuffle
    while (mask) {
    uint64_t take = mask;
    int pick = -1;
#pragma unroll
    for (uint32_t g = 0; g < 4; ++g) {
        if (take) {
            const int b0 = __builtin_ctzll(take);
            if (g == grp) pick = b0;
            take &= take - 1;
        }
    }
    mask = take;
    const bool mine = pick >= 0;
    RowRef x{0, 0, 0, 0};
    if (mine) x = row_ref(m, base + static_cast<uint64_t>(pick));
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t e = static_cast<uint32_t>(k) * 16 + l;
        v[k] = (mine && e < x.len) ? out_j[x.in + e] : kPad;
    }
    group16_bitonic64(v);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t e = static_cast<uint32_t>(k) * 16 + l;
        if (mine && e < x.len) pairs[x.out + e] = make_uint2(x.id, v[k]);
    }
    }
    }
}

// list[pos[r]] = r for every row longer than 64 entries
__global__ __launch_bounds__(kThreads) void k_compact_long(const uint64_t *__restrict__ off, uint64_t rows,
                                                           const uint32_t *__restrict__ pos,
                                                           uint32_t *__restrict__ list) {
    const uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r < rows && off[r + 1] - off[r] > 64) list[pos[r]] = static_cast<uint32_t>(r);
}

__global__ __launch_bounds__(kThreads) void k_rowsort_wave(RowMap m,
                                                            const uint32_t *__restrict__ out_j,
                                                            uint2 *__restrict__ pairs,
                                                            const uint32_t *__restrict__ list,
                                                            const uint32_t *__restrict__ count) {
    __shared__ uint32_t slot[kWaves][kWaveCap];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    volatile uint32_t *sh = slot[wave];
    const uint32_t nlong = *count;
    for (uint32_t w = blockIdx.x * kWaves + wave; w < nlong; w += gridDim.x * kWaves) {
        const RowRef x = row_ref(m, list[w]);
        if (x.len > kWaveCap) continue;  // the workgroup kernel's
        const uint32_t len = x.len;
        const uint32_t N = next_pow2(len);
        for (uint32_t e = lane; e < N; e += 64) sh[e] = e < len ? out_j[x.in + e] : kPad;
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
        for (uint32_t e = lane; e < len; e += 64) pairs[x.out + e] = make_uint2(x.id, sh[e]);
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ __launch_bounds__(kThreads) void k_rowsort_big(RowMap m,
                                                           uint32_t *__restrict__ out_j,
                                                           uint2 *__restrict__ pairs,
                                                           const uint32_t *__restrict__ list,
                                                           const uint32_t *__restrict__ count) {
    __shared__ uint32_t sh[kBlockCap];
    const uint32_t nlong = *count;
    for (uint32_t b = blockIdx.x; b < nlong; b += gridDim.x) {
        const RowRef x = row_ref(m, list[b]);
        if (x.len <= kWaveCap) continue;  // the wave kernel's
        const uint64_t s = x.in, so = x.out;
        const uint32_t len = x.len;
        const uint32_t N = next_pow2(len);
        const uint32_t r32 = x.id;
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
            for (uint32_t e = threadIdx.x; e < len; e += kThreads) pairs[so + e] = make_uint2(r32, sh[e]);
            __syncthreads();
            continue;
        }
        // Global-memory network; the row's pair segment (2 * len words >= N)
        // is the scratch array.
        uint32_t *T = reinterpret_cast<uint32_t *>(pairs + so);
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
        for (uint32_t e = threadIdx.x; e < len; e += kThreads) pairs[so + e] = make_uint2(r32, out_j[s + e]);
        __syncthreads();
    }
}

template <int N>
void launch_lane(const RowMap &m, const uint32_t *out_j, uint2 *pairs, hipStream_t s) {
    const uint64_t nb = (m.rows + kThreads - 1) / kThreads;
    KTimer kt_("rowsort_lane", s);
    k_rowsort_lane<N><<<static_cast<unsigned>(nb), kThreads, 0, s>>>(m, out_j, pairs);
    SJ_LAUNCH_CHECK();
}

// Rows longer than `sorted` (already sorted by the lane kernel or the fill).
void rowsort_long(const RowMap &m, uint32_t *out_j, uint2 *p2, uint32_t max_len, uint32_t sorted,
                  hipStream_t s) {
    const uint64_t chunks64 = (m.rows + 63) / 64;
    const unsigned grid = static_cast<unsigned>(std::min<uint64_t>((chunks64 + kWaves - 1) / kWaves, 8192));
    if (max_len > sorted && sorted < 64) {
        KTimer kt_("rowsort_group16", s);
        k_rowsort_group16<<<grid, kThreads, 0, s>>>(m, out_j, p2, sorted);
        SJ_LAUNCH_CHECK();
    }
    if (max_len <= 64) return;
    // rows longer than 64, in row order
    DevBuf<uint32_t> pos(m.rows + 1), list(m.rows);
    scan_long_rows_exclusive(m.in_off, 64, pos.ptr, m.rows, s);
    k_compact_long<<<static_cast<unsigned>((m.rows + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        m.in_off, m.rows, pos.ptr, list.ptr);
    SJ_LAUNCH_CHECK();
    const uint32_t *count = pos.ptr + m.rows;
    {
        KTimer kt_("rowsort_wave", s);
        const unsigned gw = static_cast<unsigned>(std::min<uint64_t>((m.rows + kWaves - 1) / kWaves, 8192));
        k_rowsort_wave<<<gw, kThreads, 0, s>>>(m, out_j, p2, list.ptr, count);
        SJ_LAUNCH_CHECK();
    }
    if (max_len > kWaveCap) {
        KTimer kt_("rowsort_big", s);
        const unsigned gb = static_cast<unsigned>(std::min<uint64_t>(m.rows, 1024));
        k_rowsort_big<<<gb, kThreads, 0, s>>>(m, out_j, p2, list.ptr, count);
        SJ_LAUNCH_CHECK();
    }
}

void rowsort(const RowMap &m, uint32_t *out_j, uint32_t *pairs, uint32_t max_len, hipStream_t s) {
    if (m.rows == 0) return;
    if (m.rows > 0x7fffffffULL) throw Error(SJ_EINVAL, "row sort: too many rows");
    uint2 *p2 = reinterpret_cast<uint2 *>(pairs);
    if (max_len <= 16)
        launch_lane<16>(m, out_j, p2, s);
    else
        launch_lane<32>(m, out_j, p2, s);
    rowsort_long(m, out_j, p2, max_len, max_len <= 16 ? 16 : 32, s);
}

}  // namespace

void launch_rowsort(const uint64_t *off, uint64_t i0, uint64_t i1, uint64_t base, uint32_t *out_j,
                    uint32_t *pairs, uint32_t max_len, hipStream_t s) {
    if (i1 <= i0) return;
    RowMap m{off + i0, base, off, base, nullptr, i0, i1 - i0};
    rowsort(m, out_j, pairs, max_len, s);
}

void launch_rowsort_long(const uint64_t *off_cell, const uint64_t *off_orig, const uint32_t *perm,
                         uint64_t n, uint32_t *out_j, uint32_t *pairs, uint32_t max_len, uint32_t sorted_len,
                         hipStream_t s) {
    if (n == 0) return;
    RowMap m{off_cell, 0, off_orig, 0, perm, 0, n};
    rowsort_long(m, out_j, reinterpret_cast<uint2 *>(pairs), max_len, sorted_len, s);
}

void launch_rowsort_cells(const uint64_t *off_cell, const uint64_t *off_orig, const uint32_t *perm,
                          uint64_t n, uint32_t *out_j, uint32_t *pairs, uint32_t max_len, hipStream_t s) {
    RowMap m{off_cell, 0, off_orig, 0, perm, 0, n};
    rowsort(m, out_j, pairs, max_len, s);
}

}  // namespace sj
