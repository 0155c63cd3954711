// Grid-row tiled adjacent-cell search and refine (Section IV-D, Algorithm 1;
// unicomp of Section V-B, Algorithm 2), with neighbour-cell points staged in
// LDS.
//
// Work unit: one wave = one "chunk" of at most 64 consecutive query points
// (cell order) that all lie in one grid row, i.e. share their cell
// coordinates in dimensions 1..d-1. For such a chunk the cells adjacent to
// any of its points are the rows whose dimension-1..d-1 coordinates differ
// from the chunk's by at most one, restricted in dimension 0 to
// [c0(first) - 1, c0(last) + 1]; because points are stored in cell order,
// each of those rows is ONE contiguous point segment, found with two binary
// searches in B. The wave stages a segment's coordinates (and the dimension-0
// sub-cell coordinate of every candidate) in its LDS slot, tile by tile; each
// lane then finds, by binary search over the staged sub-cell coordinates,
// its window of candidates and evaluates exactly those. Inside a cell the
// points are ordered by their dimension-0 sub-cell (width w / S), so the
// window can be the sub-cells within w of the lane's own -- S on each side,
// 2 + 1/S cell widths instead of the 3 of cells c0 - 1 .. c0 + 1 -- a subset
// of the per-point search of Algorithm 1 that holds every pair within eps
// (its members differ by at most eps <= w in dimension 0), read from LDS
// instead of global memory.
//
// unicomp: rows whose block k >= 1 is gated by an odd dimension-k coordinate
// are the same for all points of a chunk (they share dimensions 1..d-1); in
// the chunk's own row a point evaluates its own cell as the triangle q >= p
// and the cells c0 - 1, c0 + 1 only if c0 is odd (block 0). The sub-cell
// window is symmetric (q is in p's window exactly when p is in q's), so each
// pair within eps is still evaluated exactly once.
//
// Pair test, counters and emission are those of the per-point kernel, with
// two additions of this kernel. From 4-D on the FP64 test sums the squared
// differences with fused multiply-adds and decides directly only outside a
// band around eps^2 that bounds that sum's distance from the predicate's
// left-to-right sum; a tile with a candidate inside the band is passed again
// for those candidates with the exact sum. From 5-D on the count pass stores
// every tested candidate's outcome as a bit (hit bits) and the fill of the
// same search (kReplay) emits from the bits instead of testing again.
//
// The distance join of a query set R with S (Section II: the self-join is
// its case R = S) runs the same kernel with the full search: the queries are
// R's points sorted into S's grid and cut into grid-row chunks of their own,
// the segments and staged candidates are S's.
#include <type_traits>

#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Candidates staged per tile; the fused fill keeps its rows in LDS too and
// stages half as many.
template <int D, int NS>
struct TileSize {
    static constexpr int base = D <= 6 ? 128 : 64;
    static constexpr int half = NS > 0 ? base / 2 : base;
    static constexpr int value = half < 64 ? 64 : half;  // at least one candidate per lane
};

// From this many dimensions on, the FP64 pair test takes the fused-square
// filter (2 operations per dimension instead of 3; the exact left-to-right
// sum only for candidates whose filter value falls in the band around eps^2).
#ifndef SJ_FUSED_MIN_D
#define SJ_FUSED_MIN_D 4
#endif
constexpr int kFusedMinD = SJ_FUSED_MIN_D;

__device__ __forceinline__ bool t_occupied(const TileArgs &t, uint32_t j, uint32_t c) {
    if (!t.masks) return true;
    return (t.masks[t.mask_off[j] + (c >> 5)] >> (c & 31u)) & 1u;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int D, bool kUni, int kMode, bool kBand, int NS>
__global__ __launch_bounds__(kThreads) void k_join_tiled(JoinArgs a, TileArgs t) {
    constexpr int TS = TileSize<D, NS>::value;
    constexpr int kRowStride = NS + 1;  // padded so lanes' slots fall in different banks
    using CT = typename std::conditional<kBand, float, double>::type;
    constexpr bool kFillM = kMode != kCount;          // a fill pass (tested or replayed)
    constexpr bool kRep = kMode == kReplay;           // the fill replays the count's hit bits
    constexpr bool kAgg = (kMode == kCount) && kUni;  // mirrored counts summed in LDS
    constexpr bool kPerm = kFillM;                    // candidate ids staged in LDS
    // unicomp fill: the lanes that hit each staged candidate collected as a
    // mask in LDS, its mirrored entries written after the tile with one
    // global slot reservation per candidate
    constexpr bool kMirAgg = kFillM && kUni;
    // hit bits: recorded by the count pass and read back by the fill pass of
    // the same FP64 search (the fill then stages no coordinates and tests
    // nothing). The FP32 pre-test's count spills registers with them (about
    // 1 KiB per lane from 6-D on) and runs 2.5 times slower, so it goes
    // without.
    constexpr bool kBits = !kBand && NS == 0 && D >= static_cast<int>(kHitBitsMinDim);
    // staged coordinates; the fused fill reuses the slot after the last
    // tile for its write-out table (row destination, row id, length)
    constexpr size_t kStageBytes = kRep ? 16 : sizeof(CT) * TS * D;
    constexpr size_t kOutBytes = NS > 0 ? 64 * (8 + 4 + 4) : 0;
    __shared__ __align__(16) unsigned char sx_all[kWaves][kStageBytes > kOutBytes ? kStageBytes : kOutBytes];
    __shared__ uint32_t sc_all[kWaves][TS];
    __shared__ uint32_t sa_all[kWaves][(kAgg || kPerm) ? TS : 1];
    __shared__ uint32_t sr_all[kWaves][NS > 0 ? 64 * kRowStride : 1];
    __shared__ unsigned long long sm_all[kWaves][kMirAgg ? TS : 1];
    __shared__ uint32_t sp_all[kWaves][kMirAgg ? 64 : 1];
    __shared__ uint32_t sb_all[kWaves];  // set when a candidate of the tile fell in the fused-square band
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    CT *sx = reinterpret_cast<CT *>(sx_all[wave]);
    uint64_t *swo = reinterpret_cast<uint64_t *>(sx_all[wave]);
    uint32_t *swp = reinterpret_cast<uint32_t *>(sx_all[wave] + 64 * 8);
    uint32_t *swl = reinterpret_cast<uint32_t *>(sx_all[wave] + 64 * 12);
    uint32_t *scx = sc_all[wave];
    uint32_t *saux = sa_all[wave];
    uint32_t *srow = sr_all[wave] + lane * (NS > 0 ? kRowStride : 0);
    unsigned long long *smask = sm_all[wave];
    uint32_t *sperm = sp_all[wave];  // the chunk's point ids by lane
    uint32_t *sband = &sb_all[wave];

    uint32_t own = 0, evals = 0, rechecks = 0;
    // chunks go to workgroups in launch order, which the hardware deals out
    // to the XCDs round robin: a dense cluster's many heavy chunks, adjacent
    // in cell order, spread over all XCDs
    const uint32_t chunk = t.chunk0 + blockIdx.x * kWaves + wave;
    const uint32_t nch = *t.nchunks_dev;
    if (chunk < (t.chunk_end < nch ? t.chunk_end : nch)) {  // uniform across the wave
        // hit bits: recorded by the count, read by the replay (a tested fill
        // takes none)
        const bool bits_on = kBits && kMode != kFill && t.bits != nullptr;
        if (kRep && !bits_on) return;  // a replay needs the bits (the host launches none without)
        // segment table of the chunk, 64 rows per register load; the first
        // load is issued before anything else (it needs only the chunk index)
        const uint2 *segs = t.segs + static_cast<size_t>(chunk) * t.rows_per_chunk;
        uint32_t seg_base = 0;
        uint2 seg_reg = static_cast<uint32_t>(lane) < t.rows_per_chunk ? segs[lane] : make_uint2(0, 0);
        const uint2 ch = t.chunks[chunk];
        const uint32_t p = ch.x + static_cast<uint32_t>(lane);
        const bool active = p < ch.y;
        double xp[D];
        CT yp[D];
        uint32_t c0p = 0;
        uint32_t p_cell_start = 0;  // first point of p's cell (unicomp)
        uint64_t my_row = 0;
        uint32_t perm_p = 0;
        uint32_t row_len = 0;  // fused fill: the row length from the count pass
        uint64_t row_dst = 0;  // fused fill: offset of the row of p in the result
        uint32_t n_own = 0;    // other fills: entries of p's own evaluation (count pass)
        uint32_t *wrow = a.out_j;
        uint32_t wlim = 0;
        if (active) {
            if (!kRep) {  // a replay tests nothing
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    xp[j] = a.Xq[static_cast<size_t>(j) * a.nqs + p];
                    if (kBand)
                        yp[j] = static_cast<CT>(a.Yq[static_cast<size_t>(j) * a.nqs + p]);
                    else
                        yp[j] = static_cast<CT>(xp[j]);
                }
            }
            c0p = t.cxq[p];
            if (kUni) p_cell_start = a.starts[a.cell_of[p]];
            if (kFillM) {
                my_row = a.offc[p] - a.out_base;
                perm_p = a.permq[p];
                if (NS > 0) row_len = static_cast<uint32_t>(a.offc[p + 1] - a.offc[p]);
                if (NS == 0) {
                    n_own = kUni ? a.own_cnt[p] : static_cast<uint32_t>(a.offc[p + 1] - a.offc[p]);
                    if (n_own > 0 && my_row + n_own <= a.out_cap) {
                        wrow = a.out_j + my_row;
                        wlim = n_own - 1;
                    }
                }
            }
        }
        if (kMirAgg) sperm[lane] = perm_p;  // read after the first tile's barrier
        if (!kBand && D >= kFusedMinD) *sband = 0u;
        // fused fill: rows that fit stay in the lane's LDS slot
        const bool row_in_lds = NS > 0 && row_len <= static_cast<uint32_t>(NS);
        // chunk geometry (uniform)
        const uint32_t h_first = a.cell_of[ch.x];
        uint32_t c[D];
#pragma unroll
        for (int j = 0; j < D; ++j) c[j] = t.coords[static_cast<size_t>(h_first) * D + j];

        auto test = [&](uint32_t i, uint32_t q) -> bool {
            if (kBand) {
                float s = 0.0f;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const float d0 = __fsub_rn(static_cast<float>(yp[j]), static_cast<float>(sx[i * D + j]));
                    s = __fadd_rn(s, __fmul_rn(d0, d0));
                }
                if (s < a.lo) return true;
                if (s > a.hi) return false;
                ++rechecks;
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double d0 = __dsub_rn(xp[j], a.X[static_cast<size_t>(j) * a.n + q]);
                    acc = __dadd_rn(acc, __dmul_rn(d0, d0));
                }
                return acc <= a.eps2;
            } else if (D >= kFusedMinD) {
                // fused-square filter: the sum by fused multiply-adds is
                // within 2 gamma_d of the definition's left-to-right sum, so
                // outside [flo, fhi] it decides as the definition does; a
                // candidate inside is left out here and noted, and the tile
                // is passed again for those candidates (test_band)
                double f = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double d0 = __dsub_rn(xp[j], static_cast<double>(sx[i * D + j]));
                    f = j == 0 ? __dmul_rn(d0, d0) : __fma_rn(d0, d0, f);
                }
                const bool in = f < a.flo;
                // a uniform branch on the compare masks, to a store only (no
                // value carried through the loop)
                if (__builtin_amdgcn_ballot_w64(f <= a.fhi) & ~__builtin_amdgcn_ballot_w64(in)) *sband = 1u;
                return in;
            } else {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double d0 = __dsub_rn(xp[j], static_cast<double>(sx[i * D + j]));
                    acc = __dadd_rn(acc, __dmul_rn(d0, d0));
                }
                return acc <= a.eps2;
            }
        };
        // second pass over a tile with band candidates: those candidates
        // only, decided by the definition's left-to-right sum
        auto test_band = [&](uint32_t i) -> bool {
            double dv[D];
            double f = 0.0, acc = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                dv[j] = __dsub_rn(xp[j], static_cast<double>(sx[i * D + j]));
                f = j == 0 ? __dmul_rn(dv[j], dv[j]) : __fma_rn(dv[j], dv[j], f);
                acc = __dadd_rn(acc, __dmul_rn(dv[j], dv[j]));
            }
            const bool band = !(f < a.flo) && f <= a.fhi;
            rechecks += band ? 1u : 0u;
            return band && acc <= a.eps2;
        };
        // One tested candidate (staged index i, point q, id its point id from
        // the staged ids, h the test result). The fused fill stores every
        // candidate into the lane's LDS slot -- hits at the row position,
        // misses into the slot's spare last word -- so the common path has
        // no branch; a row longer than the slot keeps its first entries there
        // and writes the rest to out_j.
        auto emit = [&](bool h, uint32_t i, uint32_t q, uint32_t id) {
            if (kMode == kCount) {
                own += h ? 1u : 0u;
                // every unicomp hit, the self pair too (taken back after the tile)
                if (kUni && h) atomicAdd(&saux[i], 1u);
            } else if (NS > 0) {
                const uint32_t slot = own < static_cast<uint32_t>(NS) ? own : static_cast<uint32_t>(NS);
                srow[h ? slot : static_cast<uint32_t>(NS)] = id;
                if (h && own >= static_cast<uint32_t>(NS)) {
                    // past the slot: at its place in the row in out_j (a row
                    // that disagrees with its count is caught at the end)
                    const uint64_t at = my_row + own;
                    a.out_j[at < a.out_cap ? at : a.out_cap - 1] = id;
                }
                own += h ? 1u : 0u;
            } else if (h) {
                // inside the row's own entries as the count pass sized them
                // (a row that finds more rewrites its last entry; the
                // disagreement is flagged at the end of the chunk)
                wrow[own < wlim ? own : wlim] = id;
                ++own;
                // every unicomp hit, the self pair too (its bit cleared after the tile)
                if (kMirAgg) atomicOr(&smask[i], 1ull << lane);
            }
        };
        // candidates [i0, i1) of the staged tile, kUnroll of them loaded and
        // tested before any is emitted
        // (two from 4-D on: four candidates' coordinates would take the
        // registers of two waves per SIMD; the count takes one branch per
        // step for the rare mirrored hits)
        constexpr int kUnroll = D <= 3 ? 4 : 2;
        // fill with hit bits: the set bits of the run's words, in order
        // (all the run's words loaded first: one memory latency per run)
        auto replay = [&](uint32_t T0, uint32_t i0, uint32_t i1, uint64_t wb) {
            const uint32_t ns = i1 - i0;
            constexpr int kWords = TS / 32;
            uint32_t wv[kWords];
#pragma unroll
            for (int k = 0; k < kWords; ++k)
                wv[k] = static_cast<uint32_t>(32 * k) < ns
                            ? t.bits[(wb + static_cast<uint64_t>(k)) * 64 + static_cast<uint64_t>(lane)]
                            : 0u;
#pragma unroll
            for (int k = 0; k < kWords; ++k) {
                uint32_t w = wv[k];
                while (w) {
                    const uint32_t b = static_cast<uint32_t>(__builtin_clz(w));
                    w &= ~(0x80000000u >> b);
                    const uint32_t i = i0 + 32 * static_cast<uint32_t>(k) + b;
                    emit(true, i, T0 + i, saux[i]);
                }
            }
        };
        auto run = [&](auto redo, auto with_bits, uint32_t T0, uint32_t i0, uint32_t i1, uint64_t wb) {
            constexpr bool kRedo = decltype(redo)::value;
            constexpr bool kB = kBits && decltype(with_bits)::value;
            auto tst = [&](uint32_t i, uint32_t q) -> bool {
                if constexpr (kRedo)
                    return test_band(i);
                else
                    return test(i, q);
            };
            if (i0 >= i1) return;
            if constexpr (kRep) {
                replay(T0, i0, i1, wb);
                return;
            }
            if (!kRedo) evals += i1 - i0;
            // count with hit bits: the run's outcomes shifted into hw, a word
            // stored each 32 candidates (ts counts the wave's steps: every
            // lane still in the loop has taken as many)
            constexpr bool rec = kMode == kCount && !kRedo && kB;
            uint32_t hw = 0, ts = 0;
            uint32_t *const wrow_bits = kB ? t.bits + wb * 64 + static_cast<uint64_t>(lane) : nullptr;
            uint32_t i = i0;
            // from 4-D on the loop runs a per-lane trip count against a
            // wave-uniform step (one compare per step); below, the plain
            // bound is faster (2-D full count: 46.7 against 61.6 us)
            const uint32_t nit = (i1 - i0) / kUnroll;
            for (uint32_t it = 0; D >= 4 ? it < nit : i + kUnroll <= i1; ++it, i += kUnroll) {
                bool h[kUnroll];
                uint32_t id[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) id[u] = kPerm ? saux[i + u] : 0u;
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) h[u] = tst(i + u, T0 + i + u);
                if (rec) {
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) hw = (hw << 1) | (h[u] ? 1u : 0u);
                    ts += kUnroll;
                    if ((ts & 31u) == 0u) {
                        wrow_bits[static_cast<uint64_t>((ts >> 5) - 1) * 64] = hw;
                        own += static_cast<uint32_t>(__popc(hw));
                        hw = 0;
                    }
                }
                if (kMode == kCount && kRedo && kB) {
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        if (h[u]) {
                            const uint32_t sk = i + u - i0;
                            atomicOr(wrow_bits + static_cast<uint64_t>(sk >> 5) * 64, 0x80000000u >> (sk & 31u));
                        }
                }
                if (kMode == kCount) {
                    bool any = false;
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) {
                        if (!rec) own += h[u] ? 1u : 0u;  // recorded: counted per word
                        any = any || h[u];
                    }
                    if (kUni && any) {
#pragma unroll
                        for (int u = 0; u < kUnroll; ++u)
                            if (h[u]) atomicAdd(&saux[i + u], 1u);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) emit(h[u], i + u, T0 + i + u, id[u]);
                }
            }
            for (; i < i1; ++i) {
                const uint32_t id = kPerm ? saux[i] : 0u;
                const bool h = tst(i, T0 + i);
                if (rec) {
                    // own hits counted with the word below
                    hw = (hw << 1) | (h ? 1u : 0u);
                    if (kUni && h) atomicAdd(&saux[i], 1u);
                    continue;
                }
                if (kMode == kCount && kRedo && kB && h) {
                    const uint32_t sk = i - i0;
                    atomicOr(wrow_bits + static_cast<uint64_t>(sk >> 5) * 64, 0x80000000u >> (sk & 31u));
                }
                emit(h, i, T0 + i, id);
            }
            if (rec) {
                const uint32_t ns = i1 - i0, r = ns & 31u;
                if (r) {
                    wrow_bits[static_cast<uint64_t>(ns >> 5) * 64] = hw << (32u - r);
                    own += static_cast<uint32_t>(__popc(hw));
                }
            }
        };
        // the run with or without hit bits, chosen once per run (uniform)
        auto run_sel = [&](auto redo, uint32_t T0, uint32_t i0, uint32_t i1, uint64_t wb) {
            if constexpr (kBits) {
                if (bits_on) {
                    run(redo, std::true_type{}, T0, i0, i1, wb);
                    return;
                }
            }
            run(redo, std::false_type{}, T0, i0, i1, wb);
        };
        auto evaluate_tile = [&](auto redo, uint32_t T0, uint32_t len, bool own_row, uint64_t wb) {
            // the sub-cells within w of p's own in dimension 0 (S of them on
            // each side: a neighbour differs by at most eps <= w); unicomp's
            // own row with an even cell: the own cell's sub-cells only
            const uint32_t S = 1u << t.sub_shift;
            uint32_t lo_c = c0p >= S ? c0p - S : 0, hi_c = c0p + S;
            if (kUni && own_row && !((c0p >> t.sub_shift) & 1u)) {
                lo_c = (c0p >> t.sub_shift) << t.sub_shift;
                hi_c = lo_c + S - 1;
            }
            if (scx[0] > hi_c || scx[len - 1] < lo_c) return;
            // both window ends by one branchless search over the TS staged
            // entries (those past len hold ~0u), the two chains interleaved
            uint32_t i_lo = 0, i_hi = 0;
#pragma unroll
            for (uint32_t half = TS / 2; half > 0; half >>= 1) {
                i_lo = scx[i_lo + half] < lo_c ? i_lo + half : i_lo;
                i_hi = scx[i_hi + half] <= hi_c ? i_hi + half : i_hi;
            }
            i_lo += scx[i_lo] < lo_c ? 1u : 0u;
            i_hi += scx[i_hi] <= hi_c ? 1u : 0u;
            i_lo = i_lo < len ? i_lo : len;
            i_hi = i_hi < len ? i_hi : len;
            if (kUni && own_row) {
                // own cell as the triangle q >= p: skip q in [start of p's
                // cell, p), a contiguous run of the tile
                const uint32_t s_lo = p_cell_start > T0 ? (p_cell_start - T0 < len ? p_cell_start - T0 : len) : 0;
                const uint32_t s_hi = p > T0 ? (p - T0 < len ? p - T0 : len) : 0;
                run_sel(redo, T0, i_lo, i_hi < s_lo ? i_hi : s_lo, wb);
                run_sel(redo, T0, i_lo > s_hi ? i_lo : s_hi, i_hi, wb + (len + 31) / 32);
            } else {
                run_sel(redo, T0, i_lo, i_hi, wb);
            }
        };
        // Row index of an offset vector o (o_j in {-1,0,1}, j = 1..d-1):
        // sum_j (o_j + 1) 3^(j-1); the own row is all zeros.
        uint32_t own_idx = 0;
        {
            uint32_t p3 = 1;
            for (int j = 1; j < D; ++j) {
                own_idx += p3;
                p3 *= 3;
            }
        }
        // The chunk's candidate rows as one stream of tiles. Full search: rows
        // 0 .. 3^(d-1) - 1. unicomp: the own row, then for every k >= 1 with
        // c_k odd the rows of block k (o_k = -1 or +1, o_j free for j < k,
        // o_j = 0 above).
        uint32_t odd_mask = 0;  // bit k: c_k odd
#pragma unroll
        for (int j = 1; j < D; ++j) odd_mask |= (c[j] & 1u) << j;
        int st_k = 0;          // unicomp: 0 = own row next, else current block k
        uint32_t st_p3k = 1;   // 3^(k-1)
        uint32_t st_i = 0;     // position inside the current block (or row counter)
        auto next_row = [&](uint32_t &ridx, bool &own_row) -> bool {
            if (!kUni) {
                if (st_i >= t.rows_per_chunk) return false;
                ridx = st_i;
                own_row = st_i == own_idx;
                ++st_i;
                return true;
            }
            if (st_k == 0) {
                st_k = 1;
                st_p3k = 1;
                st_i = 0;
                ridx = own_idx;
                own_row = true;
                return true;
            }
            while (st_k < D) {
                if (((odd_mask >> st_k) & 1u) && st_i < 2 * st_p3k) {
                    const uint32_t upper = own_idx - (3 * st_p3k - 1) / 2;
                    const uint32_t side = st_i < st_p3k ? 0u : 2u;
                    const uint32_t low = st_i < st_p3k ? st_i : st_i - st_p3k;
                    ridx = upper + side * st_p3k + low;
                    own_row = false;
                    ++st_i;
                    return true;
                }
                ++st_k;
                st_p3k *= 3;
                st_i = 0;
            }
            return false;
        };
        auto segment = [&](uint32_t ridx) -> uint2 {
            const uint32_t base = ridx & ~63u;
            if (base != seg_base) {
                seg_base = base;
                const uint32_t r = base + static_cast<uint32_t>(lane);
                seg_reg = r < t.rows_per_chunk ? segs[r] : make_uint2(0, 0);
            }
            const int l = static_cast<int>(ridx - base);
            return make_uint2(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(seg_reg.x), l)),
                              static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(seg_reg.y), l)));
        };
        // tile cursor: candidates [T0, min(T0 + TS, P1)) of row ridx
        struct Tile {
            uint32_t ridx, T0, P1;
            bool own_row, valid;
        };
        auto advance = [&](Tile tl) -> Tile {
            if (tl.valid && tl.T0 + TS < tl.P1) {
                tl.T0 += TS;
                return tl;
            }
            uint32_t r;
            bool o;
            while (next_row(r, o)) {
                const uint2 sg = segment(r);
                if (sg.x < sg.y) return Tile{r, sg.x, sg.y, o, true};
            }
            tl.valid = false;
            return tl;
        };
        Tile cur = advance(Tile{0, 0, 0, false, false});
        // fused fill: the row's place in the result (needs perm_p; used at
        // the end)
        if (NS > 0 && active) row_dst = a.off_orig[perm_p];
        // hit bits: the chunk's next free word row (uniform); a tile takes
        // ceil(len / 32) word rows per run (two runs in unicomp's own row)
        uint64_t wcur = bits_on ? t.cbase[chunk] : 0;
        while (cur.valid) {
            const uint32_t len = (cur.P1 - cur.T0) < static_cast<uint32_t>(TS) ? (cur.P1 - cur.T0) : TS;
            const uint64_t wb = wcur;
            wcur += static_cast<uint64_t>((len + 31) / 32) * ((kUni && cur.own_row) ? 2u : 1u);
            wave_sync_lds();
            // stage the tile straight from memory. Holding the next tile in
            // registers while this one is evaluated was measured: no faster
            // for the fused fill or the full count, slower for the unicomp
            // count (its loads wait behind the flush atomics) and from 4-D on
            // (the registers cost waves per SIMD).
            for (uint32_t i = lane; i < len; i += 64) {
                const size_t q = cur.T0 + i;
                if (!kRep) {
#pragma unroll
                    for (int j = 0; j < D; ++j)
                        sx[i * D + j] = kBand ? static_cast<CT>(a.Y[static_cast<size_t>(j) * a.n + q])
                                              : static_cast<CT>(a.X[static_cast<size_t>(j) * a.n + q]);
                }
                scx[i] = t.cx[q];
                if (kAgg) saux[i] = 0;
                if (kPerm) saux[i] = a.perm[q];
                if (kMirAgg) smask[i] = 0;
            }
            for (uint32_t i = len + lane; i < static_cast<uint32_t>(TS); i += 64) scx[i] = ~0u;
            const Tile nxt = advance(cur);
            wave_sync_lds();
            if (active) evaluate_tile(std::false_type{}, cur.T0, len, cur.own_row, wb);
            if (!kBand && D >= kFusedMinD && !kRep) {
                if (__builtin_amdgcn_readfirstlane(*sband)) {
                    *sband = 0u;
                    if (active) evaluate_tile(std::true_type{}, cur.T0, len, cur.own_row, wb);
                }
            }
            if (kAgg && cur.own_row && active && p >= cur.T0 && p - cur.T0 < len) {
                // the self pair is no mirrored hit: its add taken back (p is
                // always in its own window, so it was tested and hit)
                atomicSub(&saux[p - cur.T0], 1u);
            }
            if (kAgg) {
                // one global add per candidate that collected mirrored hits
                wave_sync_lds();
                for (uint32_t i = lane; i < len; i += 64) {
                    const uint32_t cnt = saux[i];
                    if (cnt) atomicAdd(&a.in_cnt[cur.T0 + i], cnt);
                }
            }
            if (kMirAgg && cur.own_row && active && p >= cur.T0 && p - cur.T0 < len) {
                // the self pair is no mirrored entry
                atomicAnd(&smask[p - cur.T0], ~(1ull << lane));
            }
            if (kMirAgg) {
                // each candidate's mirrored entries: one slot reservation in
                // its row, then the ids of the lanes that hit it, in a run
                wave_sync_lds();
                for (uint32_t i = lane; i < len; i += 64) {
                    unsigned long long m = smask[i];
                    if (m) {
                        const uint32_t q = cur.T0 + i;
                        const uint32_t slot = atomicAdd(&a.cur[q], static_cast<uint32_t>(__popcll(m)));
                        uint64_t at = a.offc[q] - a.out_base + a.own_cnt[q] + slot;
                        while (m) {
                            const int b = __builtin_ctzll(m);
                            m &= m - 1;
                            if (at < a.out_cap)
                                a.out_j[at] = sperm[b];
                            else
                                atomicOr(a.overflow, 1u);
                            ++at;
                        }
                    }
                }
            }
            cur = nxt;
        }
        if (kMode == kCount && active) a.own_cnt[p] = own;
        if (kFillM && NS == 0 && active && (own != n_own || my_row + n_own > a.out_cap))
            atomicOr(a.overflow, 1u);  // count and fill disagree, or the row is past the buffer
        if (kFillM && NS > 0 && !kUni) {
            // the row of p is complete: sort it in registers; a row longer
            // than the LDS slot is in out_j for the row-sort kernels
            constexpr int kNs = NS <= 0 ? 1 : (NS <= 16 ? 16 : (NS <= 32 ? 32 : 64));  // sort width >= NS
            const uint32_t len = own;
            uint32_t lds_len = 0;
            if (active && own != row_len) atomicOr(a.overflow, 1u);  // count and fill disagree
            const bool sort_here = active && row_in_lds && len <= static_cast<uint32_t>(NS > 0 ? NS : 1);
            // network width: the wave's longest row rounded up to 4, 8, 16
            // or kNs (entries past a row's length hold ~0u and stay last)
            const uint32_t wlen = wave_max(sort_here ? len : 0u);
            auto sort_row = [&](auto width) {
                constexpr int W = decltype(width)::value;
                uint32_t v[W];
#pragma unroll
                for (int k = 0; k < W; ++k) v[k] = static_cast<uint32_t>(k) < len ? srow[k] : 0xffffffffu;
                register_bitonic<W>(v);
#pragma unroll
                for (int k = 0; k < W; ++k)
                    if (static_cast<uint32_t>(k) < len) srow[k] = v[k];
            };
            if (sort_here) {
                if (wlen <= 4)
                    sort_row(std::integral_constant<int, 4>{});
                else if (wlen <= 8)
                    sort_row(std::integral_constant<int, 8>{});
                else if (kNs > 16 && wlen <= 16)
                    sort_row(std::integral_constant<int, (kNs > 16 ? 16 : kNs)>{});
                else
                    sort_row(std::integral_constant<int, kNs>{});
                lds_len = len;
            }
            wave_sync_lds();  // last tile's reads of the staging slot are done
            swo[lane] = row_dst;
            swp[lane] = perm_p;
            swl[lane] = lds_len;
            wave_sync_lds();
            // write-out: L lanes per row (the wave's longest row rounded up
            // to a power of two), 64 / L rows per pass, so each store
            // instruction covers whole rows (contiguous (i, j) pairs) instead
            // of one pair in each of 64 different rows
            const uint32_t wout = wave_max(lds_len);
            const int lb = wout <= 1u ? 0 : 32 - __clz(static_cast<int>(wout - 1u));
            const int sub = lane >> lb, k = lane & ((1 << lb) - 1);
            const uint32_t *srows = sr_all[wave];
            for (int r0 = 0; r0 < (wout ? 64 : 0); r0 += (64 >> lb)) {
                const int r = r0 + sub;
                const uint32_t rl = swl[r];
                if (static_cast<uint32_t>(k) < rl) {
                    const uint64_t v = static_cast<uint64_t>(swp[r]) |
                                       (static_cast<uint64_t>(srows[r * kRowStride + k]) << 32);
                    __builtin_nontemporal_store(v, reinterpret_cast<unsigned long long *>(a.pairs + swo[r] + k));
                }
            }
            // rows longer than the slot but at most 64 long: in out_j (written
            // above by this wave); sorted four at a time, one row per 16-lane
            // group with 4 entries per lane
            // a row longer than 64 is sorted by the row-sort kernels, from
            // out_j: its first NS entries join the rest there
            if (active && !row_in_lds && row_len > 64u) {
                const uint32_t m = own < static_cast<uint32_t>(NS) ? own : static_cast<uint32_t>(NS);
                for (uint32_t e = 0; e < m; ++e) {
                    const uint64_t at = my_row + e;
                    a.out_j[at < a.out_cap ? at : a.out_cap - 1] = srow[e];
                }
            }
            uint64_t longm = ballot(active && !row_in_lds && row_len <= 64u);
            if (longm) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // own stores before own loads
            const uint32_t grp = static_cast<uint32_t>(lane) >> 4, gl = static_cast<uint32_t>(lane) & 15u;
            while (longm) {
                // the group's row: the grp-th lowest remaining long row
                uint64_t take = longm;
                int pick = -1;
#pragma unroll
                for (uint32_t g = 0; g < 4; ++g) {
                    if (take) {
                        const int b0 = __builtin_ctzll(take);
                        if (g == grp) pick = b0;
                        take &= take - 1;
                    }
                }
                longm = take;
                // every lane takes part in every shuffle (a lane that skipped
                // one would leave its own value unreadable to the others)
                const int src_lane = pick >= 0 ? pick : 0;
                const uint32_t rl_any = static_cast<uint32_t>(__shfl(static_cast<int>(row_len), src_lane, 64));
                const uint32_t rid = static_cast<uint32_t>(__shfl(static_cast<int>(perm_p), src_lane, 64));
                const uint64_t src = __shfl(my_row, src_lane, 64), dst = __shfl(row_dst, src_lane, 64);
                const uint32_t rl = pick >= 0 ? rl_any : 0u;
                uint32_t v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t e = static_cast<uint32_t>(k) * 16 + gl;
                    // the first NS entries in the row's LDS slot, the rest in out_j
                    v[k] = e < rl ? (e < static_cast<uint32_t>(NS) ? srows[src_lane * kRowStride + e] : a.out_j[src + e])
                                  : 0xffffffffu;
                }
                group16_bitonic64(v);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t e = static_cast<uint32_t>(k) * 16 + gl;
                    if (e < rl)
                        __builtin_nontemporal_store(static_cast<uint64_t>(rid) | (static_cast<uint64_t>(v[k]) << 32),
                                                    reinterpret_cast<unsigned long long *>(a.pairs + dst + e));
                }
            }
        }
    }
    if (kMode == kCount) {
        add_counter(a.evals, evals);
        if (kBand || D >= kFusedMinD) add_counter(a.band_rechecks, rechecks);
    }
}

const char *const kTiledNames[8] = {"tiled_count_full_fp64", "tiled_count_full_fp32band",
                                    "tiled_count_unicomp_fp64", "tiled_count_unicomp_fp32band",
                                    "tiled_fill_full_fp64", "tiled_fill_full_fp32band",
                                    "tiled_fill_unicomp_fp64", "tiled_fill_unicomp_fp32band"};

template <int D, bool U, int M, bool BD, int NS>
void launch_tiled_one(const JoinArgs &a, const TileArgs &t, hipStream_t s) {
    const uint32_t span = t.chunk_end < t.nchunks ? t.chunk_end - t.chunk0 : t.nchunks - t.chunk0;
    const unsigned nb = (span + kWaves - 1) / kWaves;
    if (nb == 0) return;
    KTimer kt_(NS ? (BD ? "tiled_fill_sort_full_fp32band" : "tiled_fill_sort_full_fp64")
                  : kTiledNames[(M == kCount ? 0 : 4) + (U ? 2 : 0) + (BD ? 1 : 0)],
               s);
    k_join_tiled<D, U, M, BD, NS><<<nb, kThreads, 0, s>>>(a, t);
    SJ_LAUNCH_CHECK();
}

template <int D>
void launch_tiled_d(const JoinArgs &a, const TileArgs &t, int unicomp, int mode, int band,
                    hipStream_t s, uint32_t fused_sort) {
    if (mode == kReplay) {
        if (band || fused_sort) throw Error(SJ_EINVAL, "tiled join: a replayed fill is FP64 without a fused sort");
        if constexpr (D >= static_cast<int>(kHitBitsMinDim)) {
            if (unicomp)
                launch_tiled_one<D, true, kReplay, false, 0>(a, t, s);
            else
                launch_tiled_one<D, false, kReplay, false, 0>(a, t, s);
            return;
        }
        throw Error(SJ_EINVAL, "tiled join: no hit bits below their dimension");
    }
    const int sel = (mode == kFill ? 4 : 0) + (unicomp ? 2 : 0) + (band ? 1 : 0);
    if (sel == 4 && fused_sort == 16) return launch_tiled_one<D, false, kFill, false, 16>(a, t, s);
    if (sel == 4 && fused_sort == 24) return launch_tiled_one<D, false, kFill, false, 24>(a, t, s);
    if (sel == 4 && fused_sort == 32) return launch_tiled_one<D, false, kFill, false, 32>(a, t, s);
    if (sel == 5 && fused_sort == 16) return launch_tiled_one<D, false, kFill, true, 16>(a, t, s);
    if (sel == 5 && fused_sort == 24) return launch_tiled_one<D, false, kFill, true, 24>(a, t, s);
    if (sel == 5 && fused_sort == 32) return launch_tiled_one<D, false, kFill, true, 32>(a, t, s);
    if (fused_sort) throw Error(SJ_EINVAL, "tiled join: fused sort needs a full fill");
    switch (sel) {
        case 0: launch_tiled_one<D, false, kCount, false, 0>(a, t, s); break;
        case 1: launch_tiled_one<D, false, kCount, true, 0>(a, t, s); break;
        case 2: launch_tiled_one<D, true, kCount, false, 0>(a, t, s); break;
        case 3: launch_tiled_one<D, true, kCount, true, 0>(a, t, s); break;
        case 4: launch_tiled_one<D, false, kFill, false, 0>(a, t, s); break;
        case 5: launch_tiled_one<D, false, kFill, true, 0>(a, t, s); break;
        case 6: launch_tiled_one<D, true, kFill, false, 0>(a, t, s); break;
        case 7: launch_tiled_one<D, true, kFill, true, 0>(a, t, s); break;
        default: throw Error(SJ_EINVAL, "tiled join: bad mode");
    }
}

// ------------------------------------------------------------ chunk list
// First point of every grid row (row index = exclusive scan of the row-head
// flags, total at row_of[ncells]); row_pt[nrows] = n.
__global__ __launch_bounds__(kThreads) void k_row_points(const uint64_t *__restrict__ row_of,
                                                          const uint32_t *__restrict__ starts,
                                                          uint32_t ncells, uint32_t n,
                                                          uint32_t *__restrict__ row_pt) {
    const uint32_t h = blockIdx.x * kThreads + threadIdx.x;
    if (h < ncells && row_of[h + 1] != row_of[h]) row_pt[row_of[h]] = starts[h];  // h heads a row
    if (h == 0) row_pt[row_of[ncells]] = n;
}

__global__ __launch_bounds__(kThreads) void k_emit_chunks(const uint32_t *__restrict__ row_pt,
                                                           const uint64_t *__restrict__ row_of,
                                                           const uint64_t *__restrict__ ch_off,
                                                           uint32_t ncells, uint2 *__restrict__ chunks,
                                                           uint32_t *__restrict__ nchunks_dev) {
    const uint32_t r = blockIdx.x * kThreads + threadIdx.x;
    if (r == 0) *nchunks_dev = static_cast<uint32_t>(ch_off[ncells]);
    if (r >= ncells || r >= row_of[ncells]) return;
    const uint32_t s = row_pt[r], e = row_pt[r + 1];
    uint64_t k = ch_off[r];
    for (uint32_t q = s; q < e; q += 64, ++k) chunks[k] = make_uint2(q, q + 64 < e ? q + 64 : e);
}

// Point segment of every (chunk, row) pair: the chunk's dimension-0 window
// [c0(first) - 1, c0(last) + 1] in the row with offset vector o (index
// sum_j (o_j + 1) 3^(j-1)); empty if the row leaves the grid or a fixed
// coordinate is not in its occupancy mask.
__global__ __launch_bounds__(kThreads) void k_chunk_segments(TileArgs t, const uint32_t *__restrict__ cell_of,
                                                              const uint32_t *__restrict__ starts,
                                                              uint32_t d, uint2 *__restrict__ segs) {
    const uint64_t idx = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    const uint64_t total = static_cast<uint64_t>(*t.nchunks_dev) * t.rows_per_chunk;
    if (idx >= total) return;
    const uint32_t chunk = static_cast<uint32_t>(idx / t.rows_per_chunk);
    uint32_t r = static_cast<uint32_t>(idx % t.rows_per_chunk);
    const uint2 ch = t.chunks[chunk];
    const uint32_t hf = cell_of[ch.x], hl = cell_of[ch.y - 1];
    const uint32_t a0 = t.coords[static_cast<size_t>(hf) * d], b0 = t.coords[static_cast<size_t>(hl) * d];
    const uint32_t lo0 = a0 > 0 ? a0 - 1 : 0;
    const uint32_t hi0 = b0 + 1 < t.dims[0] ? b0 + 1 : static_cast<uint32_t>(t.dims[0] - 1);
    uint64_t base = 0;
    bool ok = true;
    for (uint32_t j = 1; j < d; ++j) {
        const int o = static_cast<int>(r % 3) - 1;
        r /= 3;
        const int64_t cj = static_cast<int64_t>(t.coords[static_cast<size_t>(hf) * d + j]) + o;
        if (cj < 0 || cj >= static_cast<int64_t>(t.dims[j])) {
            ok = false;
            break;
        }
        if (t.masks && !((t.masks[t.mask_off[j] + (cj >> 5)] >> (cj & 31)) & 1u)) {
            ok = false;
            break;
        }
        base += static_cast<uint64_t>(cj) * t.stride[j];
    }
    uint2 sg = make_uint2(0, 0);
    if (ok && t.ncells > 0) {
        // lower bounds of both ends in B, the two searches interleaved
        // (their loads are independent, so each step costs one latency)
        const uint64_t k_lo = base + lo0, k_hi = base + hi0 + 1;
        uint32_t g_lo = 0, g_hi = 0, len = t.ncells;
        while (len > 1) {
            const uint32_t half = len >> 1;
            const uint64_t v_lo = t.B[g_lo + half], v_hi = t.B[g_hi + half];
            g_lo = v_lo < k_lo ? g_lo + half : g_lo;
            g_hi = v_hi < k_hi ? g_hi + half : g_hi;
            len -= half;
        }
        g_lo += t.B[g_lo] < k_lo ? 1u : 0u;
        g_hi += t.B[g_hi] < k_hi ? 1u : 0u;
        if (g_lo < g_hi) sg = make_uint2(starts[g_lo], starts[g_hi]);
    }
    segs[idx] = sg;
}

// Word rows of hit bits each chunk's count pass takes: for every candidate
// row the chunk visits (all rows; unicomp: its own row and the rows of the
// blocks k >= 1 whose dimension-k coordinate is odd), ceil(segment / 32) per
// run -- a tile of len candidates takes ceil(len / 32) and the tiles of a
// segment are multiples of 32 but the last -- twice in unicomp's own row
// (the triangle's two runs). One thread per chunk; slot nslots - 1 (past the
// chunks) gets 0, so that the exclusive scan ends in the total. *big is
// set when a chunk needs 2^32 - 1 or more.
__global__ __launch_bounds__(kThreads) void k_chunk_words(TileArgs t, const uint32_t *__restrict__ cell_of,
                                                           uint32_t d, int unicomp, uint32_t nslots,
                                                           uint32_t *__restrict__ cwords, uint32_t *__restrict__ big) {
    const uint32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= nslots) return;
    const uint32_t nch = *t.nchunks_dev;
    uint64_t w = 0;
    if (c < nch && c + 1 < nslots) {
        const uint2 ch = t.chunks[c];
        const uint32_t hf = cell_of[ch.x];
        uint32_t odd = 0;
        for (uint32_t j = 1; j < d; ++j) odd |= (t.coords[static_cast<size_t>(hf) * d + j] & 1u) << j;
        for (uint32_t r = 0; r < t.rows_per_chunk; ++r) {
            const uint2 sg = t.segs[static_cast<size_t>(c) * t.rows_per_chunk + r];
            if (sg.x >= sg.y) continue;
            uint32_t rr = r, top = 0;
            for (uint32_t j = 1; j < d; ++j) {
                if (rr % 3 != 1) top = j;
                rr /= 3;
            }
            const bool own = top == 0;
            if (unicomp && !own && !((odd >> top) & 1u)) continue;
            w += static_cast<uint64_t>((sg.y - sg.x + 31) / 32) * ((unicomp && own) ? 2u : 1u);
        }
    }
    if (w >= 0xffffffffull) {
        atomicOr(big, 1u);
        w = 0;
    }
    cwords[c] = static_cast<uint32_t>(w);
}

__global__ void k_zero_word(uint32_t *p) {
    if (threadIdx.x == 0) *p = 0;
}

inline unsigned nblk(uint64_t n) { return static_cast<unsigned>((n + kThreads - 1) / kThreads); }

}  // namespace

uint32_t build_chunks(const uint32_t *coords, const uint32_t *starts, uint32_t ncells, uint32_t n, uint32_t d,
                      uint64_t rows_bound, uint2 **chunks_out, size_t *chunks_cap, uint32_t *nchunks_dev,
                      hipStream_t s) {
    // chunk list only; row segments come from build_chunk_segments
    if (ncells == 0 || n == 0) {
        k_zero_word<<<1, 64, 0, s>>>(nchunks_dev);
        SJ_LAUNCH_CHECK();
        return 0;
    }
    const uint64_t bound = static_cast<uint64_t>(n) / 64 + std::min<uint64_t>(ncells, rows_bound);
    if (bound >= 0xffffffffULL) throw Error(SJ_ECAPACITY, "too many join chunks");
    // rows are bounded by the cells, so every array below is sized by ncells
    DevBuf<uint32_t> row_pt(static_cast<size_t>(ncells) + 1);
    DevBuf<uint64_t> row_of(static_cast<size_t>(ncells) + 1), choff(static_cast<size_t>(ncells) + 1);
    scan_row_heads_exclusive(coords, d, row_of.ptr, ncells, s);
    k_row_points<<<nblk(ncells), kThreads, 0, s>>>(row_of.ptr, starts, ncells, n, row_pt.ptr);
    SJ_LAUNCH_CHECK();
    scan_row_chunks_exclusive(row_pt.ptr, row_of.ptr, choff.ptr, ncells, s);
    if (bound > *chunks_cap) {
        if (*chunks_out) dev_free(*chunks_out);
        *chunks_out = static_cast<uint2 *>(dev_alloc(bound * sizeof(uint2)));
        *chunks_cap = bound;
    }
    k_emit_chunks<<<nblk(ncells), kThreads, 0, s>>>(row_pt.ptr, row_of.ptr, choff.ptr, ncells, *chunks_out,
                                                   nchunks_dev);
    SJ_LAUNCH_CHECK();
    return static_cast<uint32_t>(bound);
}

void build_chunk_segments(const TileArgs &t, const uint32_t *cell_of, const uint32_t *starts,
                          uint32_t d, uint2 *segs, hipStream_t s) {
    const uint64_t total = static_cast<uint64_t>(t.nchunks) * t.rows_per_chunk;
    if (!total) return;
    KTimer kt_("chunk_segments", s);
    k_chunk_segments<<<static_cast<unsigned>((total + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        t, cell_of, starts, d, segs);
    SJ_LAUNCH_CHECK();
}

void launch_chunk_words(const TileArgs &t, const uint32_t *cell_of, uint32_t d, int unicomp, uint32_t nslots,
                        uint32_t *cwords, uint32_t *big, hipStream_t s) {
    if (!nslots) return;
    KTimer kt_("chunk_words", s);
    k_chunk_words<<<(nslots + kThreads - 1) / kThreads, kThreads, 0, s>>>(t, cell_of, d, unicomp, nslots, cwords,
                                                                          big);
    SJ_LAUNCH_CHECK();
}

void launch_join_tiled(const JoinArgs &a, const TileArgs &t, uint32_t d, int unicomp, int mode,
                       int band, hipStream_t s, uint32_t fused_sort) {
    switch (d) {
        case 1: launch_tiled_d<1>(a, t, unicomp, mode, band, s, fused_sort); break;
        case 2: launch_tiled_d<2>(a, t, unicomp, mode, band, s, fused_sort); break;
        case 3: launch_tiled_d<3>(a, t, unicomp, mode, band, s, fused_sort); break;
        case 4: launch_tiled_d<4>(a, t, unicomp, mode, band, s, fused_sort); break;
        case 5: launch_tiled_d<5>(a, t, unicomp, mode, band, s, fused_sort); break;
        case 6: launch_tiled_d<6>(a, t, unicomp, mode, band, s, fused_sort); break;
        case 7: launch_tiled_d<7>(a, t, unicomp, mode, band, s, fused_sort); break;
        case 8: launch_tiled_d<8>(a, t, unicomp, mode, band, s, fused_sort); break;
        default: throw Error(SJ_EINVAL, "tiled join: d out of range");
    }
}

}  // namespace sj
