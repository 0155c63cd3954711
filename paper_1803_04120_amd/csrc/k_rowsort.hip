// Result rows to sorted (i, j) pairs.
//
// After the fill pass every result row i (all j within eps of point i)
// occupies its own contiguous segment, in candidate order. Sorting each
// segment by j and writing (i, j) gives the key/value result sorted by key
// and value (Section IV-E sorts the key/value pairs after the kernel), and
// because rows are laid out in order of i the whole result is sorted by
// (i, j) without any global sort.
//
// Rows are sorted by size class, every class by a bitonic network over
// values held in registers (entries past a row's length hold ~0u and stay
// last):
//   <= 32          one lane per row, 16 or 32 registers (16 when no row is
//                  longer), fully unrolled (static register indices)
//   <= 64          16 lanes per row, 4 registers each, stages with a partner
//                  distance below 16 through 16-lane shuffles
//   <= 1024        one wave per row, 4, 8 or 16 registers per lane (the row
//                  rounded up to 256, 512 or 1024), element e = 64 k + lane
//                  in register k: partner distances below 64 are lane
//                  shuffles, larger ones register swaps -- no LDS, no barrier
//   <= 8192        one workgroup (4 waves) per row, 8, 16 or 32 registers per
//                  lane, element e = 256 k + thread: distances 64 and 128
//                  cross waves through LDS (two barriers per stage), the
//                  others as above
//   larger         one workgroup per row, in place in the row's own out_j
//                  segment in global memory, with the variant of the network
//                  whose comparators all put the smaller value first (each
//                  merge level opens with mirrored pairs): the virtual ~0u
//                  entries past the row never move, so the row needs no
//                  padding and no scratch
// No kernel appends rows to a shared queue (a queue counter is one address
// that every producer hits). The 33..64 class is found by scanning the row
// offsets (64 rows per wave and ballot); rows longer than 64 (and, apart,
// longer than 1024) are listed in row order by a stream compaction (a scan
// of the long-row flags), and the wave and workgroup kernels walk the list,
// so the long rows of a dense cluster -- adjacent in cell order -- spread
// over all waves.
//
// Row r's neighbour ids are read from out_j[in_off[r] - in_base, +len) and
// its entries are written at out_off[id] - out_base, +len, with
// id = perm ? perm[r] : r0 + r: as (i, j) pairs, or as the column ids of a
// compressed sparse row table (j only). A whole result is filled in cell
// order (the rows of one wave's points are adjacent, so the fill writes and
// these reads are contiguous) and scattered to the rows' places in order of
// i here; batches are filled directly in order of i (in_off = out_off).
// j values within a row are distinct, so no stability is needed. Unsorted
// output (the caller asked for rows in any internal order) moves each row
// with no network.
#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kWaveCap = 1024;
constexpr uint32_t kBlockCap = 8192;
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

// Where the sorted rows go: interleaved (i, j) pairs, or CSR column ids.
struct RowDst {
    uint2 *pairs;
    uint32_t *cols;
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

__device__ __forceinline__ void put(const RowDst &o, uint64_t at, uint32_t i, uint32_t j) {
    if (o.cols)
        o.cols[at] = j;
    else
        o.pairs[at] = make_uint2(i, j);
}

__device__ __forceinline__ uint32_t next_pow2(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

__device__ __forceinline__ void cas_asc(uint32_t &lo, uint32_t &hi) {
    const uint32_t a = lo, b = hi;
    lo = a < b ? a : b;
    hi = a < b ? b : a;
}

// Bitonic network over N = T R values of a group of T threads (T = 64 W),
// thread t holding element e = T k + t in v[k]. Partner distances of T or
// more swap registers; below 64 they are wave shuffles; in between they
// cross waves through lds (R T words; every thread of the group must call).
template <int R, int W>
__device__ __forceinline__ void group_bitonic(uint32_t (&v)[R], uint32_t *lds) {
    constexpr int T = 64 * W;
    const uint32_t t = threadIdx.x & static_cast<uint32_t>(T - 1);
#pragma unroll
    for (int kk = 2; kk <= T * R; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= T) {
                const int jr = j / T;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int kp = k ^ jr;
                    if (kp > k) {
                        const uint32_t e = static_cast<uint32_t>(k) * T + t;
                        if ((e & static_cast<uint32_t>(kk)) == 0)
                            cas_asc(v[k], v[kp]);
                        else
                            cas_asc(v[kp], v[k]);
                    }
                }
            } else {
                uint32_t p[R];
                if (j >= 64) {
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < R; ++k) lds[k * T + t] = v[k];
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < R; ++k) p[k] = lds[k * T + (t ^ static_cast<uint32_t>(j))];
                } else {
#pragma unroll
                    for (int k = 0; k < R; ++k) p[k] = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v[k]), j, 64));
                }
                const bool lower = (t & static_cast<uint32_t>(j)) == 0;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const uint32_t e = static_cast<uint32_t>(k) * T + t;
                    const bool asc = (e & static_cast<uint32_t>(kk)) == 0;
                    const uint32_t mn = v[k] < p[k] ? v[k] : p[k], mx = v[k] < p[k] ? p[k] : v[k];
                    v[k] = (lower == asc) ? mn : mx;
                }
            }
        }
    }
}

template <int N>
__global__ __launch_bounds__(kThreads) void k_rowsort_lane(RowMap m, RowDst o, const uint32_t *__restrict__ out_j) {
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
        if (static_cast<uint32_t>(k) < x.len) put(o, x.out + k, x.id, v[k]);
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
__global__ __launch_bounds__(kThreads) void k_rowsort_group16(RowMap m, RowDst o, const uint32_t *__restrict__ out_j,
                                                               uint32_t lo) {
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
                if (mine && e < x.len) put(o, x.out + e, x.id, v[k]);
            }
        }
    }
}

// list[pos[r]] = r for every row longer than lo entries
__global__ __launch_bounds__(kThreads) void k_compact_long(const uint64_t *__restrict__ off, uint64_t rows,
                                                           uint32_t lo, const uint32_t *__restrict__ pos,
                                                           uint32_t *__restrict__ list) {
    const uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r < rows && off[r + 1] - off[r] > lo) list[pos[r]] = static_cast<uint32_t>(r);
}

// The all-ascending (mirror) form of the bitonic sorter over 64 R values of
// one wave, lane l holding element e = 64 k + l in v[k]: the merge of two
// sorted blocks of size kk/2 first compares each e with its mirror
// e ^ (kk - 1), then with e ^ j for j = kk/4 .. 1, the lower index taking
// the minimum. Every block stays ascending, so the padding (kPad, the largest
// value) never leaves the positions at or past the row's length: registers
// k >= kact hold only padding at every stage, and every exchange with one of
// them is skipped (kact is uniform across the wave). A row of 257 entries
// costs 5 registers' work, not 8.
template <int R>
__device__ __forceinline__ void wave_bitonic_mirror(uint32_t (&v)[R], uint32_t kact) {
    const uint32_t lane = static_cast<uint32_t>(lane_id());
    // partner lane ^ m in the same register; hb: the highest bit of m
    auto lane_stage = [&](int m, uint32_t hb) {
        const bool lower = (lane & hb) == 0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (static_cast<uint32_t>(k) < kact) {
                // (the 16-register network is not unrolled whole: a partner
                // distance known only at run time would make the DPP choice a
                // branch per exchange)
                const uint32_t p = R <= 8 ? lane_xor(v[k], m)
                                          : static_cast<uint32_t>(__shfl_xor(static_cast<int>(v[k]), m, 64));
                v[k] = lower ? (v[k] < p ? v[k] : p) : (v[k] < p ? p : v[k]);
            }
        }
    };
    // registers k < k ^ r: elements (k, l) and (k ^ r, 63 - l)
    auto reg_mirror = [&](int r) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int kp = k ^ r;
            if (k < kp && static_cast<uint32_t>(kp) < kact) {
                const uint32_t a = v[k], b = v[kp];
                const uint32_t ra = static_cast<uint32_t>(__shfl_xor(static_cast<int>(a), 63, 64));
                const uint32_t rb = static_cast<uint32_t>(__shfl_xor(static_cast<int>(b), 63, 64));
                v[k] = a < rb ? a : rb;
                v[kp] = b < ra ? ra : b;
            }
        }
    };
    // registers k < k ^ r, same lane
    auto reg_half = [&](int r) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int kp = k ^ r;
            if (k < kp && static_cast<uint32_t>(kp) < kact) cas_asc(v[k], v[kp]);
        }
    };
#pragma unroll
    for (int kk = 2; kk <= 64 * R; kk <<= 1) {
        if (kk <= 64)
            lane_stage(kk - 1, static_cast<uint32_t>(kk >> 1));
        else
            reg_mirror((kk - 1) >> 6);
#pragma unroll
        for (int j = kk >> 2; j > 0; j >>= 1) {
            if (j >= 64)
                reg_half(j >> 6);
            else
                lane_stage(j, static_cast<uint32_t>(j));
        }
    }
}

// One row of 65..1024 entries per wave, in registers: R = 4, 8 or 16 by the
// row's length (uniform across the wave).
template <int R>
__device__ __forceinline__ void wave_sort_row(const RowRef &x, const RowDst &o, const uint32_t *out_j) {
    const uint32_t lane = static_cast<uint32_t>(lane_id());
    uint32_t v[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const uint32_t e = static_cast<uint32_t>(k) * 64 + lane;
        v[k] = e < x.len ? out_j[x.in + e] : kPad;
    }
    wave_bitonic_mirror<R>(v, (x.len + 63) / 64);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const uint32_t e = static_cast<uint32_t>(k) * 64 + lane;
        if (e < x.len) put(o, x.out + e, x.id, v[k]);
    }
}

// kWide = false: the rows of 65..512 entries (4 or 8 registers); true: those
// of 513..1024 (16 registers), a launch of its own so that the 16-register
// network's registers do not cost the common case waves per SIMD.
template <bool kWide>
__global__ __launch_bounds__(kThreads) void k_rowsort_wave(RowMap m, RowDst o, const uint32_t *__restrict__ out_j,
                                                            const uint32_t *__restrict__ list,
                                                            const uint32_t *__restrict__ count) {
    const int wave = threadIdx.x >> 6;
    const uint32_t nlong = *count;
    for (uint32_t w = blockIdx.x * kWaves + wave; w < nlong; w += gridDim.x * kWaves) {
        const RowRef x = row_ref(m, list[w]);
        if (!kWide && x.len <= 256)
            wave_sort_row<4>(x, o, out_j);
        else if (!kWide && x.len <= 512)
            wave_sort_row<8>(x, o, out_j);
        else if (kWide && x.len > 512 && x.len <= kWaveCap)
            wave_sort_row<16>(x, o, out_j);
        // longer: a workgroup kernel's
    }
}

// One row of (lo, 256 R] entries per workgroup (lo = 128 R), in registers,
// from the list of rows longer than 1024.
template <int R>
__global__ __launch_bounds__(kThreads) void k_rowsort_block(RowMap m, RowDst o, const uint32_t *__restrict__ out_j,
                                                             const uint32_t *__restrict__ list,
                                                             const uint32_t *__restrict__ count) {
    __shared__ uint32_t lds[R * kThreads];
    constexpr uint32_t lo = 128u * R, hi = 256u * R;
    const uint32_t t = threadIdx.x;
    const uint32_t nlong = *count;
    for (uint32_t b = blockIdx.x; b < nlong; b += gridDim.x) {
        const RowRef x = row_ref(m, list[b]);
        if (x.len <= lo || x.len > hi) continue;  // uniform across the workgroup
        uint32_t v[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const uint32_t e = static_cast<uint32_t>(k) * kThreads + t;
            v[k] = e < x.len ? out_j[x.in + e] : kPad;
        }
        group_bitonic<R, kWaves>(v, lds);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const uint32_t e = static_cast<uint32_t>(k) * kThreads + t;
            if (e < x.len) put(o, x.out + e, x.id, v[k]);
        }
        __syncthreads();  // the next row's first LDS stage must not overtake this one's reads
    }
}

// Rows longer than 8192: one workgroup per row, in place in out_j. Every
// comparator puts the smaller value at the lower index (each merge level
// opens with the mirrored pairs i, i ^ (kk - 1)), so the entries past the
// row -- virtually ~0u -- never move and comparators that reach them are
// skipped.
__global__ __launch_bounds__(kThreads) void k_rowsort_global(RowMap m, RowDst o, uint32_t *__restrict__ out_j,
                                                              const uint32_t *__restrict__ list,
                                                              const uint32_t *__restrict__ count) {
    const uint32_t nlong = *count;
    for (uint32_t b = blockIdx.x; b < nlong; b += gridDim.x) {
        const RowRef x = row_ref(m, list[b]);
        if (x.len <= kBlockCap) continue;
        uint32_t *T = out_j + x.in;
        const uint32_t len = x.len;
        const uint32_t N = next_pow2(len);
        for (uint32_t kk = 2; kk <= N; kk <<= 1) {
            const uint32_t half = kk >> 1;
            for (uint32_t q = threadIdx.x; q < N / 2; q += kThreads) {
                const uint32_t blk = q / half, off = q % half;
                const uint32_t i = blk * kk + off, l = blk * kk + kk - 1 - off;
                if (l < len) cas_asc(T[i], T[l]);
            }
            __threadfence();
            __syncthreads();
            for (uint32_t j = kk >> 2; j > 0; j >>= 1) {
                for (uint32_t q = threadIdx.x; q < N / 2; q += kThreads) {
                    const uint32_t i = 2 * j * (q / j) + (q % j), l = i + j;
                    if (l < len) cas_asc(T[i], T[l]);
                }
                __threadfence();
                __syncthreads();
            }
        }
        for (uint32_t e = threadIdx.x; e < len; e += kThreads) put(o, x.out + e, x.id, T[e]);
        __syncthreads();
    }
}

// Unsorted output: rows longer than lo moved as they are, 16 lanes per row.
__global__ __launch_bounds__(kThreads) void k_rowmove(RowMap m, RowDst o, const uint32_t *__restrict__ out_j,
                                                       uint32_t lo) {
    const uint32_t l = threadIdx.x & 15u;
    const uint64_t groups = static_cast<uint64_t>(gridDim.x) * (kThreads / 16);
    for (uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads / 16) + (threadIdx.x >> 4); r < m.rows;
         r += groups) {
        const uint32_t len = static_cast<uint32_t>(m.in_off[r + 1] - m.in_off[r]);
        if (len <= lo) continue;
        const RowRef x = row_ref(m, r);
        for (uint32_t e = l; e < len; e += 16) put(o, x.out + e, x.id, out_j[x.in + e]);
    }
}

template <int N>
void launch_lane(const RowMap &m, const RowDst &o, const uint32_t *out_j, hipStream_t s) {
    const uint64_t nb = (m.rows + kThreads - 1) / kThreads;
    KTimer kt_("rowsort_lane", s);
    k_rowsort_lane<N><<<static_cast<unsigned>(nb), kThreads, 0, s>>>(m, o, out_j);
    SJ_LAUNCH_CHECK();
}

// list of the rows longer than lo (in row order) and its length at
// pos[rows], both in the pos/list buffers
void compact_rows(const RowMap &m, uint32_t lo, DevBuf<uint32_t> &pos, DevBuf<uint32_t> &list, hipStream_t s) {
    pos.reset(m.rows + 1);
    list.reset(m.rows);
    scan_long_rows_exclusive(m.in_off, lo, pos.ptr, m.rows, s);
    k_compact_long<<<static_cast<unsigned>((m.rows + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        m.in_off, m.rows, lo, pos.ptr, list.ptr);
    SJ_LAUNCH_CHECK();
}

template <int R>
void launch_block_class(const RowMap &m, const RowDst &o, const uint32_t *out_j, const uint32_t *list,
                        const uint32_t *count, uint32_t max_len, hipStream_t s) {
    if (max_len <= 128u * R) return;
    KTimer kt_("rowsort_block", s);
    const unsigned g = static_cast<unsigned>(std::min<uint64_t>(m.rows, 2048));
    k_rowsort_block<R><<<g, kThreads, 0, s>>>(m, o, out_j, list, count);
    SJ_LAUNCH_CHECK();
}

// Rows longer than `sorted` (already sorted by the lane kernel or the fill).
void rowsort_long(const RowMap &m, const RowDst &o, uint32_t *out_j, uint32_t max_len, uint32_t sorted,
                  hipStream_t s) {
    const uint64_t chunks64 = (m.rows + 63) / 64;
    const unsigned grid = static_cast<unsigned>(std::min<uint64_t>((chunks64 + kWaves - 1) / kWaves, 8192));
    if (max_len > sorted && sorted < 64) {
        KTimer kt_("rowsort_group16", s);
        k_rowsort_group16<<<grid, kThreads, 0, s>>>(m, o, out_j, sorted);
        SJ_LAUNCH_CHECK();
    }
    if (max_len <= 64) return;
    DevBuf<uint32_t> pos, list;
    compact_rows(m, 64, pos, list, s);
    const unsigned gw = static_cast<unsigned>(std::min<uint64_t>((m.rows + kWaves - 1) / kWaves, 8192));
    {
        KTimer kt_("rowsort_wave", s);
        k_rowsort_wave<false><<<gw, kThreads, 0, s>>>(m, o, out_j, list.ptr, pos.ptr + m.rows);
        SJ_LAUNCH_CHECK();
    }
    if (max_len > 512) {
        KTimer kt_("rowsort_wave16", s);
        k_rowsort_wave<true><<<gw, kThreads, 0, s>>>(m, o, out_j, list.ptr, pos.ptr + m.rows);
        SJ_LAUNCH_CHECK();
    }
    if (max_len <= kWaveCap) return;
    DevBuf<uint32_t> pos2, list2;
    compact_rows(m, kWaveCap, pos2, list2, s);
    const uint32_t *count2 = pos2.ptr + m.rows;
    launch_block_class<8>(m, o, out_j, list2.ptr, count2, max_len, s);
    launch_block_class<16>(m, o, out_j, list2.ptr, count2, max_len, s);
    launch_block_class<32>(m, o, out_j, list2.ptr, count2, max_len, s);
    if (max_len > kBlockCap) {
        KTimer kt_("rowsort_global", s);
        const unsigned gb = static_cast<unsigned>(std::min<uint64_t>(m.rows, 1024));
        k_rowsort_global<<<gb, kThreads, 0, s>>>(m, o, out_j, list2.ptr, count2);
        SJ_LAUNCH_CHECK();
    }
}

void rowmove(const RowMap &m, const RowDst &o, const uint32_t *out_j, uint32_t lo, hipStream_t s) {
    if (m.rows == 0) return;
    KTimer kt_("rowmove", s);
    const uint64_t groups = (m.rows + 15) / 16;
    const unsigned g = static_cast<unsigned>(std::min<uint64_t>(groups, 16384));
    k_rowmove<<<g, kThreads, 0, s>>>(m, o, out_j, lo);
    SJ_LAUNCH_CHECK();
}

void rowsort(const RowMap &m, const RowDst &o, uint32_t *out_j, uint32_t max_len, bool sorted, hipStream_t s) {
    if (m.rows == 0) return;
    if (m.rows > 0x7fffffffULL) throw Error(SJ_EINVAL, "row sort: too many rows");
    if (!sorted) return rowmove(m, o, out_j, 0, s);
    if (max_len <= 16)
        launch_lane<16>(m, o, out_j, s);
    else
        launch_lane<32>(m, o, out_j, s);
    rowsort_long(m, o, out_j, max_len, max_len <= 16 ? 16 : 32, s);
}

RowDst dst_of(uint32_t *pairs, uint32_t *cols) { return RowDst{reinterpret_cast<uint2 *>(pairs), cols}; }

}  // namespace

void launch_rowsort(const uint64_t *off, uint64_t i0, uint64_t i1, uint64_t base, uint32_t *out_j,
                    uint32_t *pairs, uint32_t max_len, hipStream_t s, uint32_t *cols, bool sorted) {
    if (i1 <= i0) return;
    RowMap m{off + i0, base, off, base, nullptr, i0, i1 - i0};
    rowsort(m, dst_of(pairs, cols), out_j, max_len, sorted, s);
}

void launch_rowsort_long(const uint64_t *off_cell, const uint64_t *off_orig, const uint32_t *perm,
                         uint64_t n, uint32_t *out_j, uint32_t *pairs, uint32_t max_len, uint32_t sorted_len,
                         hipStream_t s, uint32_t *cols, bool sorted) {
    if (n == 0) return;
    RowMap m{off_cell, 0, off_orig, 0, perm, 0, n};
    if (!sorted) {
        if (max_len > sorted_len) rowmove(m, dst_of(pairs, cols), out_j, sorted_len, s);
        return;
    }
    rowsort_long(m, dst_of(pairs, cols), out_j, max_len, sorted_len, s);
}

void launch_rowsort_range(const uint64_t *off_cell, uint64_t r0, uint64_t r1, uint64_t in_base,
                          const uint64_t *off_out, const uint32_t *perm, uint32_t *out_j, uint32_t *pairs,
                          uint32_t max_len, uint32_t sorted_len, hipStream_t s, uint32_t *cols, bool sorted) {
    if (r1 <= r0) return;
    RowMap m{off_cell + r0, in_base, off_out, 0, perm + r0, 0, r1 - r0};
    const RowDst o = dst_of(pairs, cols);
    if (!sorted) {
        if (max_len > sorted_len) rowmove(m, o, out_j, sorted_len, s);
        return;
    }
    if (sorted_len == 0)
        rowsort(m, o, out_j, max_len, true, s);
    else
        rowsort_long(m, o, out_j, max_len, sorted_len, s);
}

void launch_rowsort_cells(const uint64_t *off_cell, const uint64_t *off_orig, const uint32_t *perm,
                          uint64_t n, uint32_t *out_j, uint32_t *pairs, uint32_t max_len, hipStream_t s,
                          uint32_t *cols, bool sorted) {
    RowMap m{off_cell, 0, off_orig, 0, perm, 0, n};
    rowsort(m, dst_of(pairs, cols), out_j, max_len, sorted, s);
}

}  // namespace sj
