// All-pairs distance join: the GPU brute-force comparison of Section VI-B
// (a nested-loop join that compares every point with every point, with no
// index), producing the same result as the grid join -- every ordered pair
// (i, j) with d2 <= fl(eps * eps) under the binary64 pair test of Section III
// -- sorted by (i, j).
//
// The paper's kernel gives each of |D| threads one point that it compares
// with all others. Here a workgroup of 256 lanes holds Q query rows per lane
// in registers and streams the candidates through LDS in tiles of 256
// points, copied straight from the caller's row-major array (a tile is one
// contiguous block, so the copy is coalesced); every lane reads a
// candidate's coordinates from the same LDS address (a broadcast) and tests
// it against its Q queries, so one LDS read serves Q distance evaluations.
// The candidates of a row are split into `splits` consecutive ranges (a
// second grid dimension) when there are too few query blocks to fill the
// chip's 256 CUs.
//
// Emission without any sort: a count pass gives the hits of every (row,
// range) cell, an exclusive scan over the cells in (row, range) order gives
// their offsets, and the fill pass writes the hits of each cell in candidate
// order. Candidates are visited in ascending j, so every row comes out
// sorted and the rows lie in ascending i.
//
// The pair test is the binary64 formula in dimension order 0..d-1, every
// operation rounded on its own (no fused multiply-add), so it decides every
// pair exactly as the grid join and the oracle do.
#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 256;  // candidates per LDS tile

template <int D>
struct BruteQ {  // query rows per lane: enough independent chains per LDS read
    static constexpr int value = D <= 4 ? 4 : 2;
};

template <int D, int kMode>
__global__ __launch_bounds__(kThreads) void k_brute(BruteArgs a) {
    constexpr int Q = BruteQ<D>::value;
    __shared__ double sx[kTile * D];
    const uint64_t qbase = static_cast<uint64_t>(blockIdx.x) * (kThreads * Q);
    const uint32_t s = blockIdx.y;
    const uint64_t c_begin = static_cast<uint64_t>(s) * a.span;
    const uint64_t c_end = c_begin + a.span < a.n ? c_begin + a.span : a.n;
    double xq[Q][D];
    bool act[Q];
    uint32_t cnt[Q];
    uint64_t at[Q], at_end[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint64_t i = qbase + static_cast<uint64_t>(q) * kThreads + threadIdx.x;
        act[q] = i < a.n;
        cnt[q] = 0;
        at[q] = at_end[q] = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) xq[q][j] = act[q] ? a.pts[i * D + j] : 0.0;
        if (kMode == kFill && act[q]) {
            const uint64_t cell = i * a.splits + s;
            at[q] = a.off[cell];
            at_end[q] = a.off[cell + 1];
        }
    }
    for (uint64_t T0 = c_begin; T0 < c_end; T0 += kTile) {
        const uint32_t len = static_cast<uint32_t>(c_end - T0 < kTile ? c_end - T0 : kTile);
        __syncthreads();  // the previous tile's reads are done
        const double *src = a.pts + T0 * D;
        for (uint32_t e = threadIdx.x; e < len * D; e += kThreads) sx[e] = src[e];
        __syncthreads();
        for (uint32_t t = 0; t < len; ++t) {
            double c[D];
#pragma unroll
            for (int j = 0; j < D; ++j) c[j] = sx[t * D + j];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double d0 = __dsub_rn(xq[q][j], c[j]);
                    acc = __dadd_rn(acc, __dmul_rn(d0, d0));
                }
                const bool h = act[q] && acc <= a.eps2;
                if (kMode == kCount) {
                    cnt[q] += h ? 1u : 0u;
                } else if (h) {
                    if (at[q] < at_end[q]) {
                        const uint64_t i = qbase + static_cast<uint64_t>(q) * kThreads + threadIdx.x;
                        a.pairs[at[q]] = make_uint2(static_cast<uint32_t>(i), static_cast<uint32_t>(T0 + t));
                    } else {
                        atomicOr(a.overflow, 1u);
                    }
                    ++at[q];
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (!act[q]) continue;
        const uint64_t i = qbase + static_cast<uint64_t>(q) * kThreads + threadIdx.x;
        if (kMode == kCount)
            a.count[i * a.splits + s] = cnt[q];
        else if (at[q] != at_end[q])
            atomicOr(a.overflow, 1u);  // the fill found fewer hits than the count
    }
}

template <int D>
void launch_brute_d(const BruteArgs &a, int mode, hipStream_t s) {
    constexpr int Q = BruteQ<D>::value;
    const uint64_t qblocks = (a.n + kThreads * Q - 1) / (kThreads * Q);
    const dim3 grid(static_cast<unsigned>(qblocks), a.splits);
    if (mode == kCount) {
        KTimer kt_("brute_count", s);
        k_brute<D, kCount><<<grid, kThreads, 0, s>>>(a);
    } else {
        KTimer kt_("brute_fill", s);
        k_brute<D, kFill><<<grid, kThreads, 0, s>>>(a);
    }
    SJ_LAUNCH_CHECK();
}

}  // namespace

uint32_t brute_rows_per_block(uint32_t d) {
    switch (d) {
        case 1: return kThreads * BruteQ<1>::value;
        case 2: return kThreads * BruteQ<2>::value;
        case 3: return kThreads * BruteQ<3>::value;
        case 4: return kThreads * BruteQ<4>::value;
        case 5: return kThreads * BruteQ<5>::value;
        case 6: return kThreads * BruteQ<6>::value;
        case 7: return kThreads * BruteQ<7>::value;
        default: return kThreads * BruteQ<8>::value;
    }
}

uint32_t brute_tile() { return kTile; }

void launch_brute(const BruteArgs &a, uint32_t d, int mode, hipStream_t s) {
    if (a.n == 0) return;
    switch (d) {
        case 1: launch_brute_d<1>(a, mode, s); break;
        case 2: launch_brute_d<2>(a, mode, s); break;
        case 3: launch_brute_d<3>(a, mode, s); break;
        case 4: launch_brute_d<4>(a, mode, s); break;
        case 5: launch_brute_d<5>(a, mode, s); break;
        case 6: launch_brute_d<6>(a, mode, s); break;
        case 7: launch_brute_d<7>(a, mode, s); break;
        case 8: launch_brute_d<8>(a, mode, s); break;
        default: throw Error(SJ_EINVAL, "brute force: d out of range");
    }
}

}  // namespace sj
