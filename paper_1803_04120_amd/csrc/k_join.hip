// Adjacent-cell search and distance refine (Section IV-D, Algorithm 1) with
// the unicomp cell subset (Section V-B, Algorithm 2).
//
// Search (one thread per non-empty query cell). Instead of probing the 3^d
// cells one by one, the cells adjacent to C are grouped into "rows": cells
// that agree in dimensions 1..d-1 and span [c_0 - 1, c_0 + 1] in dimension
// 0. Cells of a row have consecutive linear ids, so one binary search in B
// finds the first occupied cell of the row, and because points are stored
// in cell order, all occupied cells of the row form ONE contiguous point
// range. A full search therefore yields at most 3^(d-1) ranges per cell;
// rows whose fixed coordinates are not in the occupancy masks M_j are
// skipped without a search. The unicomp subset keeps, for every dimension k
// with c_k odd, the cells that differ from C in dimension k, range freely in
// dimensions below k and equal C above k; for k = 0 these are the two single
// cells c_0 - 1 and c_0 + 1. The query's own cell is then evaluated as the
// triangle q >= p.
//
// Refine (one thread per query point, cell order). Each lane keeps its
// point in registers and scans its cell's ranges; candidate coordinates are
// read from the structure-of-arrays copy, so lanes of the same cell read the
// same addresses. Pair test in binary64, dimension order 0..d-1, no fused
// multiply-add: d2 <= fl(eps^2). The FP32 variant tests the shifted single
// precision copy first and re-decides only in the proven band [lo, hi].
//
// Emission. The count pass records each row's length: the query's own
// hits in a register, and under unicomp the mirrored pair (q, p) as an
// atomic increment of q's incoming count. The fill pass writes each row in
// place: own hits at [row start, +own), mirrored hits after them at a slot
// taken with an atomic on q's cursor.
#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t lower_bound_u64(const uint64_t *__restrict__ B, uint32_t n,
                                                    uint64_t key) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (B[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool occupied(const SearchArgs &a, uint32_t j, uint32_t c) {
    if (!a.masks) return true;
    return (a.masks[a.mask_off[j] + (c >> 5)] >> (c & 31u)) & 1u;
}

// Emits the ranges of one row: dimension-0 span [lo0, hi0] with the other
// coordinates given by `base_id` (their contribution to the linear id).
template <bool kWrite>
__device__ __forceinline__ void row_range(const SearchArgs &a, uint64_t base_id, uint32_t lo0,
                                          uint32_t hi0, uint32_t &count, uint2 *out) {
    const uint64_t klo = base_id + lo0;
    const uint64_t khi = base_id + hi0;
    uint32_t h = lower_bound_u64(a.B, a.ncells, klo);
    if (h >= a.ncells || a.B[h] > khi) return;
    const uint32_t first = h;
    while (h + 1 < a.ncells && a.B[h + 1] <= khi) ++h;
    if (kWrite) out[count] = make_uint2(a.starts[first], a.starts[h + 1]);
    ++count;
}

template <bool kWrite>
__device__ uint32_t search_cell(const SearchArgs &a, uint32_t cell, bool unicomp, uint2 *out) {
    const uint32_t d = a.d;
    uint32_t c[kMaxDim];
    for (uint32_t j = 0; j < d; ++j) c[j] = a.coords[static_cast<uint64_t>(cell) * d + j];
    uint32_t lo[kMaxDim], hi[kMaxDim];
    for (uint32_t j = 0; j < d; ++j) {
        lo[j] = c[j] > 0 ? c[j] - 1 : 0;
        hi[j] = c[j] + 1 < a.dims[j] ? c[j] + 1 : static_cast<uint32_t>(a.dims[j] - 1);
    }
    uint32_t count = 0;
    if (!unicomp) {
        // every combination of dimensions 1..d-1 within [lo, hi]
        uint32_t off[kMaxDim];
        for (uint32_t j = 1; j < d; ++j) off[j] = lo[j];
        while (true) {
            bool ok = true;
            uint64_t base = 0;
            for (uint32_t j = 1; j < d; ++j) {
                ok = ok && occupied(a, j, off[j]);
                base += off[j] * a.stride[j];
            }
            if (ok) row_range<kWrite>(a, base, lo[0], hi[0], count, out);
            uint32_t j = 1;
            while (j < d) {
                if (off[j] < hi[j]) {
                    ++off[j];
                    break;
                }
                off[j] = lo[j];
                ++j;
            }
            if (j >= d) break;
        }
        return count;
    }
    // unicomp block k = 0: the two cells c_0 -/+ 1 of the own row
    uint64_t own_rest = 0;
    for (uint32_t j = 1; j < d; ++j) own_rest += c[j] * a.stride[j];
    if (c[0] & 1u) {
        if (c[0] > 0 && occupied(a, 0, c[0] - 1))
            row_range<kWrite>(a, own_rest, c[0] - 1, c[0] - 1, count, out);
        if (c[0] + 1 < a.dims[0] && occupied(a, 0, c[0] + 1))
            row_range<kWrite>(a, own_rest, c[0] + 1, c[0] + 1, count, out);
    }
    // unicomp blocks k >= 1
    for (uint32_t k = 1; k < d; ++k) {
        if (!(c[k] & 1u)) continue;
        // dims 1..k-1 free in [lo, hi]; dim k in {c_k - 1, c_k + 1}; dims > k fixed
        uint64_t upper = 0;
        for (uint32_t j = k + 1; j < d; ++j) upper += c[j] * a.stride[j];
        for (int side = -1; side <= 1; side += 2) {
            if (side < 0 && c[k] == 0) continue;
            if (side > 0 && c[k] + 1 >= a.dims[k]) continue;
            const uint32_t ck = c[k] + side;
            if (!occupied(a, k, ck)) continue;
            const uint64_t fixed = upper + ck * a.stride[k];
            uint32_t off[kMaxDim];
            for (uint32_t j = 1; j < k; ++j) off[j] = lo[j];
            while (true) {
                bool ok = true;
                uint64_t base = fixed;
                for (uint32_t j = 1; j < k; ++j) {
                    ok = ok && occupied(a, j, off[j]);
                    base += off[j] * a.stride[j];
                }
                if (ok) row_range<kWrite>(a, base, lo[0], hi[0], count, out);
                uint32_t j = 1;
                while (j < k) {
                    if (off[j] < hi[j]) {
                        ++off[j];
                        break;
                    }
                    off[j] = lo[j];
                    ++j;
                }
                if (j >= k) break;
            }
        }
    }
    return count;
}

__global__ __launch_bounds__(kThreads) void k_search_count(SearchArgs a, int unicomp,
                                                            uint32_t *__restrict__ cnt) {
    const uint32_t h = blockIdx.x * kThreads + threadIdx.x;
    if (h >= a.ncells) return;
    cnt[h] = search_cell<false>(a, h, unicomp != 0, nullptr);
}

__global__ __launch_bounds__(kThreads) void k_search_fill(SearchArgs a, int unicomp,
                                                           const uint64_t *__restrict__ roff,
                                                           uint2 *__restrict__ rng) {
    const uint32_t h = blockIdx.x * kThreads + threadIdx.x;
    if (h >= a.ncells) return;
    search_cell<true>(a, h, unicomp != 0, rng + roff[h]);
}

// ------------------------------------------------------------------ join
template <int D, bool kBand>
struct Point {
    double x[D];
    float y[kBand ? D : 1];
};

template <int D, bool kBand>
__device__ __forceinline__ bool pair_within(const JoinArgs &a, const Point<D, kBand> &p,
                                            uint32_t q, uint32_t &rechecks) {
    if (kBand) {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const float t = __fsub_rn(p.y[j], a.Y[static_cast<size_t>(j) * a.n + q]);
            s = __fadd_rn(s, __fmul_rn(t, t));
        }
        if (s < a.lo) return true;
        if (s > a.hi) return false;
        ++rechecks;
    }
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double t = __dsub_rn(p.x[j], a.X[static_cast<size_t>(j) * a.n + q]);
        acc = __dadd_rn(acc, __dmul_rn(t, t));
    }
    return acc <= a.eps2;
}

// Lanes past the end of the query list stay in the kernel (inactive) so the
// wave-wide counter reduction at the end sees every lane.
template <int D, bool kUni, int kMode, bool kBand>
__global__ __launch_bounds__(kThreads) void k_join_guarded(JoinArgs a) {
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
    const bool active = t < a.nq;
    uint32_t own = 0, evals = 0, rechecks = 0;
    if (active) {
        const uint32_t p = a.qlist ? a.qlist[t] : a.qbase + t;
        const uint32_t h = a.cell_of[p];
        Point<D, kBand> pt;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            pt.x[j] = a.X[static_cast<size_t>(j) * a.n + p];
            if (kBand) pt.y[j] = a.Y[static_cast<size_t>(j) * a.n + p];
        }
        uint64_t my_row = 0;
        uint32_t perm_p = 0;
        if (kMode == kFill) {
            my_row = a.offc[p] - a.out_base;
            perm_p = a.perm[p];
        }
        // Fill positions come from the count pass; a write at or past the
        // buffer end (only possible if the two passes disagreed) is dropped
        // and flagged instead of being made.
        auto emit = [&](uint32_t q, bool mirror) {
            if (kMode == kCount) {
                ++own;
                if (mirror) atomicAdd(&a.in_cnt[q], 1u);
            } else {
                const uint64_t at = my_row + own;
                if (at < a.out_cap)
                    a.out_j[at] = a.perm[q];
                else
                    atomicOr(a.overflow, 1u);
                ++own;
                if (mirror) {
                    const uint32_t slot = atomicAdd(&a.cur[q], 1u);
                    const uint64_t at2 = a.offc[q] - a.out_base + a.own_cnt[q] + slot;
                    if (at2 < a.out_cap)
                        a.out_j[at2] = perm_p;
                    else
                        atomicOr(a.overflow, 1u);
                }
            }
        };
        if (kUni) {
            const uint32_t end = a.starts[h + 1];
            for (uint32_t q = p; q < end; ++q) {
                ++evals;
                if (pair_within<D, kBand>(a, pt, q, rechecks)) emit(q, q != p);
            }
        }
        const uint64_t r0 = a.roff[h], r1 = a.roff[h + 1];
        for (uint64_t e = r0; e < r1; ++e) {
            const uint2 r = a.rng[e];
            for (uint32_t q = r.x; q < r.y; ++q) {
                ++evals;
                if (pair_within<D, kBand>(a, pt, q, rechecks)) emit(q, kUni);
            }
        }
        if (kMode == kCount) a.own_cnt[p] = own;
    }
    if (kMode == kCount) {
        add_counter(a.evals, evals);
        if (kBand) add_counter(a.band_rechecks, rechecks);
    }
}

const char *const kJoinNames[8] = {"join_count_full_fp64", "join_count_full_fp32band",
                                   "join_count_unicomp_fp64", "join_count_unicomp_fp32band",
                                   "join_fill_full_fp64", "join_fill_full_fp32band",
                                   "join_fill_unicomp_fp64", "join_fill_unicomp_fp32band"};

template <int D, bool U, int M, bool BD>
void launch_one(const JoinArgs &a, unsigned nb, hipStream_t s) {
    KTimer kt_(kJoinNames[M * 4 + (U ? 2 : 0) + (BD ? 1 : 0)], s);
    k_join_guarded<D, U, M, BD><<<nb, kThreads, 0, s>>>(a);
    SJ_LAUNCH_CHECK();
}

template <int D>
void launch_join_d(const JoinArgs &a, int unicomp, int mode, int band, hipStream_t s) {
    const unsigned nb = (a.nq + kThreads - 1) / kThreads;
    if (nb == 0) return;
    const int sel = (mode == kFill ? 4 : 0) + (unicomp ? 2 : 0) + (band ? 1 : 0);
    switch (sel) {
        case 0: launch_one<D, false, kCount, false>(a, nb, s); break;
        case 1: launch_one<D, false, kCount, true>(a, nb, s); break;
        case 2: launch_one<D, true, kCount, false>(a, nb, s); break;
        case 3: launch_one<D, true, kCount, true>(a, nb, s); break;
        case 4: launch_one<D, false, kFill, false>(a, nb, s); break;
        case 5: launch_one<D, false, kFill, true>(a, nb, s); break;
        case 6: launch_one<D, true, kFill, false>(a, nb, s); break;
        case 7: launch_one<D, true, kFill, true>(a, nb, s); break;
        default: throw Error(SJ_EINVAL, "join: bad mode");
    }
}

// ------------------------------------------------------------ row plans
// Row lengths in original order (for the output offsets) and in cell order
// (for the fill layout). Every workgroup writes its longest row and its
// numbers of rows longer than 16, 24 and 32 entries to stats[4 b .. 4 b + 4)
// (no atomics: 512 workgroups adding to one cache line serialised).
constexpr int kRowStatBlocks = 512;
static_assert(kRowStatWords == 4 * static_cast<size_t>(kRowStatBlocks), "row statistics layout");
__global__ __launch_bounds__(kThreads) void k_row_lengths(const uint32_t *__restrict__ own,
                                                           const uint32_t *__restrict__ inc,
                                                           const uint32_t *__restrict__ perm,
                                                           uint64_t n, uint32_t *__restrict__ len,
                                                           uint32_t *__restrict__ len_cell,
                                                           uint32_t *__restrict__ stats) {
    uint32_t m = 0, c16 = 0, c24 = 0, c32 = 0;
    for (uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x; r < n;
         r += static_cast<uint64_t>(gridDim.x) * kThreads) {
        const uint32_t l = own[r] + (inc ? inc[r] : 0u);
        len[perm[r]] = l;
        len_cell[r] = l;
        m = l > m ? l : m;
        c16 += l > 16u;
        c24 += l > 24u;
        c32 += l > 32u;
    }
    m = wave_max(m);
    c16 = wave_sum(c16);
    c24 = wave_sum(c24);
    c32 = wave_sum(c32);
    __shared__ uint32_t sm[4][kThreads / 64];
    if (lane_id() == 0) {
        sm[0][threadIdx.x >> 6] = m;
        sm[1][threadIdx.x >> 6] = c16;
        sm[2][threadIdx.x >> 6] = c24;
        sm[3][threadIdx.x >> 6] = c32;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = sm[0][0], s16 = sm[1][0], s24 = sm[2][0], s32 = sm[3][0];
        for (int w = 1; w < kThreads / 64; ++w) {
            b = sm[0][w] > b ? sm[0][w] : b;
            s16 += sm[1][w];
            s24 += sm[2][w];
            s32 += sm[3][w];
        }
        uint32_t *o = stats + 4 * static_cast<size_t>(blockIdx.x);
        o[0] = b;
        o[1] = s16;
        o[2] = s24;
        o[3] = s32;
    }
}

// Original-order row offset of every cell-ordered point (gather through A).
__global__ __launch_bounds__(kThreads) void k_gather_offsets(const uint64_t *__restrict__ off,
                                                              const uint32_t *__restrict__ perm,
                                                              uint64_t n, uint64_t *__restrict__ offc) {
    const uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r < n) offc[r] = off[perm[r]];
}

__global__ __launch_bounds__(kThreads) void k_batch_flags(const uint32_t *__restrict__ perm,
                                                           uint64_t n, uint64_t i0, uint64_t i1,
                                                           uint32_t *__restrict__ flag) {
    const uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r >= n) return;
    const uint64_t i = perm[r];
    flag[r] = (i >= i0 && i < i1) ? 1u : 0u;
}

__global__ __launch_bounds__(kThreads) void k_batch_compact(const uint32_t *__restrict__ perm,
                                                             uint64_t n, uint64_t i0, uint64_t i1,
                                                             const uint32_t *__restrict__ pos,
                                                             uint32_t *__restrict__ qlist) {
    const uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r >= n) return;
    const uint64_t i = perm[r];
    if (i >= i0 && i < i1) qlist[pos[r]] = static_cast<uint32_t>(r);
}

__global__ void k_batch_bounds(const uint64_t *__restrict__ off, uint64_t n, uint64_t total,
                               uint32_t nb, uint64_t *__restrict__ rows) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    if (b == nb) {
        rows[b] = n;
        return;
    }
    const unsigned __int128 t128 = static_cast<unsigned __int128>(b) * total / nb;
    const uint64_t target = static_cast<uint64_t>(t128);
    uint64_t lo = 0, hi = n;  // first i in [0, n] with off[i] >= target
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (off[mid] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    rows[b] = lo;
}

// Batch b of a cell-ordered run plan starts at the first work unit u (a
// chunk, or a single point when chunks is null) whose first point's
// cell-order row offset is at least b * total / nb: unit[b], its first
// point pos[b] and that offset off[b]; entry nb is the end (units, n, total).
__global__ void k_batch_units(const uint2 *__restrict__ chunks, const uint64_t *__restrict__ off_cell,
                              uint64_t n, uint32_t units, uint64_t total, uint32_t nb,
                              uint32_t *__restrict__ unit, uint64_t *__restrict__ pos,
                              uint64_t *__restrict__ off) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    auto start = [&](uint32_t u) -> uint64_t { return u >= units ? n : (chunks ? chunks[u].x : u); };
    if (b == nb) {
        unit[b] = units;
        pos[b] = n;
        off[b] = total;
        return;
    }
    const unsigned __int128 t128 = static_cast<unsigned __int128>(b) * total / nb;
    const uint64_t target = static_cast<uint64_t>(t128);
    uint32_t lo = 0, hi = units;  // first u in [0, units] with off_cell[start(u)] >= target
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (off_cell[start(mid)] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    unit[b] = lo;
    pos[b] = start(lo);
    off[b] = off_cell[start(lo)];
}

// len_b[perm[r]] = len_cell[r] for the batch's points r in [r0, r1) (len_b
// cleared before): the batch's row lengths in order of i.
__global__ __launch_bounds__(kThreads) void k_batch_lengths(const uint32_t *__restrict__ len_cell,
                                                             const uint32_t *__restrict__ perm, uint64_t r0,
                                                             uint64_t r1, uint32_t *__restrict__ len_b) {
    const uint64_t r = r0 + blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r < r1) len_b[perm[r]] = len_cell[r];
}

inline unsigned blocks_for(uint64_t n) {
    return static_cast<unsigned>((n + kThreads - 1) / kThreads);
}

}  // namespace

void launch_batch_bounds(const uint64_t *off, uint64_t n, uint64_t total, uint32_t nb,
                         uint64_t *rows, hipStream_t s) {
    k_batch_bounds<<<(nb + 1 + 255) / 256, 256, 0, s>>>(off, n, total, nb, rows);
    SJ_LAUNCH_CHECK();
}

uint64_t build_ranges(const SearchArgs &a, int unicomp, uint64_t *roff, uint32_t **rng_out,
                      size_t *rng_cap, hipStream_t s) {
    if (a.ncells == 0) return 0;
    DevBuf<uint32_t> cnt(a.ncells);
    {
        KTimer kt_("search_count", s);
        k_search_count<<<blocks_for(a.ncells), kThreads, 0, s>>>(a, unicomp, cnt.ptr);
        SJ_LAUNCH_CHECK();
    }
    scan_exclusive_u32_to_u64(cnt.ptr, roff, a.ncells, s);
    HostStage hs;
    SJ_HIP(hipMemcpyAsync(hs.p, roff + a.ncells, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    const uint64_t total = *hs.as<uint64_t>();
    if (total > *rng_cap) {
        if (*rng_out) dev_free(*rng_out);
        const size_t cap = total + total / 8 + 64;
        *rng_out = static_cast<uint32_t *>(dev_alloc(cap * 2 * sizeof(uint32_t)));
        *rng_cap = cap;
    }
    {
        KTimer kt_("search_fill", s);
        k_search_fill<<<blocks_for(a.ncells), kThreads, 0, s>>>(a, unicomp, roff,
                                                                reinterpret_cast<uint2 *>(*rng_out));
        SJ_LAUNCH_CHECK();
    }
    SJ_HIP(hipStreamSynchronize(s));
    return total;
}

void launch_join(const JoinArgs &a, uint32_t d, int unicomp, int mode, int band, hipStream_t s) {
    switch (d) {
        case 1: launch_join_d<1>(a, unicomp, mode, band, s); break;
        case 2: launch_join_d<2>(a, unicomp, mode, band, s); break;
        case 3: launch_join_d<3>(a, unicomp, mode, band, s); break;
        case 4: launch_join_d<4>(a, unicomp, mode, band, s); break;
        case 5: launch_join_d<5>(a, unicomp, mode, band, s); break;
        case 6: launch_join_d<6>(a, unicomp, mode, band, s); break;
        case 7: launch_join_d<7>(a, unicomp, mode, band, s); break;
        case 8: launch_join_d<8>(a, unicomp, mode, band, s); break;
        default: throw Error(SJ_EINVAL, "join: d out of range");
    }
}

void launch_row_lengths(const uint32_t *own_cnt, const uint32_t *in_cnt, const uint32_t *perm,
                        uint64_t n, uint32_t *len_orig, uint32_t *len_cell, uint32_t *row_stats,
                        hipStream_t s) {
    KTimer kt_("row_lengths", s);
    k_row_lengths<<<kRowStatBlocks, kThreads, 0, s>>>(own_cnt, in_cnt, perm, n, len_orig, len_cell, row_stats);
    SJ_LAUNCH_CHECK();
}

// out[0] = P (off_orig[n]), out[1] = longest row, out[2] = evaluations,
// out[3] = band re-checks (both summed over the counter slots), out[4] =
// chunk count (0 without chunks), out[5..8) = rows longer than 16, 24, 32
// (row_stats[1..4)): the count pass reads these back at once.
__global__ __launch_bounds__(256) void k_count_summary(const uint64_t *__restrict__ off_orig, uint64_t n,
                                                        const uint32_t *__restrict__ max_len,
                                                        const unsigned long long *__restrict__ counters,
                                                        const uint32_t *__restrict__ nchunks,
                                                        uint64_t *__restrict__ out,
                                                        uint32_t *__restrict__ overflow) {
    __shared__ unsigned long long part[6][256 / 64];
    const int k = threadIdx.x;  // one counter slot and two row-stat blocks per thread
    unsigned long long e = counters[static_cast<size_t>(k) * kCounterStride];
    unsigned long long b = counters[static_cast<size_t>(kCounterSlots + k) * kCounterStride];
    unsigned long long mx = 0, c16 = 0, c24 = 0, c32 = 0;
    for (int q = k; q < kRowStatBlocks; q += 256) {
        const uint32_t *st = max_len + 4 * q;
        mx = st[0] > mx ? st[0] : mx;
        c16 += st[1];
        c24 += st[2];
        c32 += st[3];
    }
    for (int off = 32; off > 0; off >>= 1) {
        e += __shfl_xor(e, off, 64);
        b += __shfl_xor(b, off, 64);
        const unsigned long long om = __shfl_xor(mx, off, 64);
        mx = om > mx ? om : mx;
        c16 += __shfl_xor(c16, off, 64);
        c24 += __shfl_xor(c24, off, 64);
        c32 += __shfl_xor(c32, off, 64);
    }
    if (lane_id() == 0) {
        part[0][k >> 6] = e;
        part[1][k >> 6] = b;
        part[2][k >> 6] = mx;
        part[3][k >> 6] = c16;
        part[4][k >> 6] = c24;
        part[5][k >> 6] = c32;
    }
    __syncthreads();
    if (k == 0) {
        unsigned long long se = 0, sb = 0, m = 0, s16 = 0, s24 = 0, s32 = 0;
        for (int w = 0; w < 256 / 64; ++w) {
            se += part[0][w];
            sb += part[1][w];
            m = part[2][w] > m ? part[2][w] : m;
            s16 += part[3][w];
            s24 += part[4][w];
            s32 += part[5][w];
        }
        out[0] = off_orig[n];
        out[1] = m;
        out[5] = s16;
        out[6] = s24;
        out[7] = s32;
        out[2] = se;
        out[3] = sb;
        out[4] = nchunks ? *nchunks : 0;
        if (overflow) *overflow = 0;  // the fill's overflow flag starts clear
    }
}

void launch_count_summary(const uint64_t *off_orig, uint64_t n, const uint32_t *max_len,
                          const unsigned long long *counters, const uint32_t *nchunks, uint64_t *out,
                          uint32_t *overflow, hipStream_t s) {
    static_assert(kCounterSlots == 256, "one thread per counter slot");
    k_count_summary<<<1, 256, 0, s>>>(off_orig, n, max_len, counters, nchunks, out, overflow);
    SJ_LAUNCH_CHECK();
}

void launch_gather_offsets(const uint64_t *off_orig, const uint32_t *perm, uint64_t n,
                           uint64_t *offc, hipStream_t s) {
    KTimer kt_("row_offsets_gather", s);
    k_gather_offsets<<<blocks_for(n), kThreads, 0, s>>>(off_orig, perm, n, offc);
    SJ_LAUNCH_CHECK();
}

void launch_batch_units(const uint2 *chunks, const uint64_t *off_cell, uint64_t n, uint32_t units,
                        uint64_t total, uint32_t nb, uint32_t *unit, uint64_t *pos, uint64_t *off, hipStream_t s) {
    k_batch_units<<<(nb + 1 + 255) / 256, 256, 0, s>>>(chunks, off_cell, n, units, total, nb, unit, pos, off);
    SJ_LAUNCH_CHECK();
}

void launch_batch_lengths(const uint32_t *len_cell, const uint32_t *perm, uint64_t r0, uint64_t r1,
                          uint32_t *len_b, hipStream_t s) {
    if (r1 <= r0) return;
    k_batch_lengths<<<blocks_for(r1 - r0), kThreads, 0, s>>>(len_cell, perm, r0, r1, len_b);
    SJ_LAUNCH_CHECK();
}

uint32_t build_query_list(const uint32_t *perm, uint64_t n, uint64_t i0, uint64_t i1,
                          uint32_t *flags_scratch, uint32_t *qlist, hipStream_t s) {
    k_batch_flags<<<blocks_for(n), kThreads, 0, s>>>(perm, n, i0, i1, flags_scratch);
    SJ_LAUNCH_CHECK();
    scan_exclusive_u32(flags_scratch, flags_scratch, n, s);
    {
        KTimer kt_("batch_query_list", s);
        k_batch_compact<<<blocks_for(n), kThreads, 0, s>>>(perm, n, i0, i1, flags_scratch, qlist);
        SJ_LAUNCH_CHECK();
    }
    return static_cast<uint32_t>(i1 - i0);
}

}  // namespace sj
