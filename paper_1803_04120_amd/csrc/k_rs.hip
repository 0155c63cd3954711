// Distance join of a query set R with an indexed set S (the self-join is the
// case R = S, Section II). Each query row takes its cell in S's grid without
// clamping -- a query outside S's bounding box probes only the part of its
// 3^d neighbourhood that lies inside the grid -- and tests the points of
// those cells with the self-join's predicate (Section III: squared distance
// in binary64, dimension order 0..d-1, no fused multiply-add, d2 <= eps^2).
// Dimension 0 varies fastest in the linear cell id, so the cells of one
// neighbourhood row are consecutive ids: one lower bound in B per row. The
// queries are taken in S's cell order (sorted by the index's cell key), so
// the threads of a wave mostly probe the same cells.
#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t rs_lower_bound(const uint64_t *__restrict__ B, uint32_t n, uint64_t key) {
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

// kMode 0: per-query counts, by query row and by probe position; 1: neighbour
// ids (S's original rows) into out_j[off[k] ...], where off is the scan of the
// counts in probe order: the segments of a wave's queries are adjacent, so its
// writes land in few lines. The row sort then moves each segment to its row.
template <int D, int kMode>
__global__ __launch_bounds__(kThreads) void k_join_rs(RsArgs a) {
    const uint64_t k = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (k >= a.nr) return;
    const uint64_t r = a.qperm[k];  // neighbouring threads probe neighbouring cells
    double q[D];
#pragma unroll
    for (int j = 0; j < D; ++j) q[j] = a.R[r * D + j];
    // neighbourhood box [lo_j, hi_j] of existing cells
    int64_t lo[D], hi[D];
    bool any = a.ncells > 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double t = floor((q[j] - a.g.gmin[j]) / a.g.w);
        const double top = static_cast<double>(a.g.dims[j]);
        if (!(t >= -1.0) || !(t <= top)) {  // NaN, or more than one cell outside
            any = false;
            lo[j] = 0;
            hi[j] = -1;
            continue;
        }
        const int64_t c = static_cast<int64_t>(t);
        lo[j] = c - 1 > 0 ? c - 1 : 0;
        hi[j] = c + 1 < static_cast<int64_t>(a.g.dims[j]) - 1 ? c + 1 : static_cast<int64_t>(a.g.dims[j]) - 1;
        if (lo[j] > hi[j]) any = false;
    }
    uint32_t found = 0;
    uint64_t at = kMode == 1 ? a.off[k] : 0;
    // fill: hits are held by their place in an aligned group of four output
    // positions (w0..w3, places [glo, ghi) of the group at gbase); a whole
    // group goes out as one 16-byte store, a partial one (at the ends of the
    // query's segment) as aligned pairs and single words
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0, glo = 4, ghi = 0;
    uint64_t gbase = 0;
    auto flush = [&]() {
        if (glo == 0 && ghi == 4) {
            *reinterpret_cast<uint4 *>(a.out_j + gbase) = make_uint4(w0, w1, w2, w3);
            return;
        }
        if (glo == 0 && ghi >= 2) {
            *reinterpret_cast<uint2 *>(a.out_j + gbase) = make_uint2(w0, w1);
        } else {
            if (glo == 0 && ghi > 0) a.out_j[gbase] = w0;
            if (glo <= 1 && ghi > 1) a.out_j[gbase + 1] = w1;
        }
        if (glo <= 2 && ghi == 4) {
            *reinterpret_cast<uint2 *>(a.out_j + gbase + 2) = make_uint2(w2, w3);
        } else {
            if (glo <= 2 && ghi > 2) a.out_j[gbase + 2] = w2;
            if (ghi > 3) a.out_j[gbase + 3] = w3;
        }
    };
    if (any) {
        // odometer over dimensions 1..d-1; dimension 0 is the id range
        int64_t o[D];
#pragma unroll
        for (int j = 0; j < D; ++j) o[j] = lo[j];
        while (true) {
            uint64_t base = 0;
#pragma unroll
            for (int j = 1; j < D; ++j) base += static_cast<uint64_t>(o[j]) * a.g.stride[j];
            const uint64_t k0 = base + static_cast<uint64_t>(lo[0]), k1 = base + static_cast<uint64_t>(hi[0]);
            uint32_t h = rs_lower_bound(a.B, a.ncells, k0);
            if (h < a.ncells && a.B[h] <= k1) {
                uint32_t he = h;
                while (he + 1 < a.ncells && a.B[he + 1] <= k1) ++he;
                const uint32_t p0 = a.starts[h], p1 = a.starts[he + 1];
                for (uint32_t p = p0; p < p1; ++p) {
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        const double t = __dsub_rn(q[j], a.X[static_cast<size_t>(j) * a.ns + p]);
                        acc = __dadd_rn(acc, __dmul_rn(t, t));
                    }
                    if (acc <= a.eps2) {
                        if (kMode == 1) {
                            const uint32_t v = a.perm[p];
                            if (at >= a.out_cap) {
                                atomicOr(a.overflow, 1u);
                            } else {
                                const uint32_t g = static_cast<uint32_t>(at & 3);
                                if (glo == 4) {  // first held hit of this group
                                    gbase = at - g;
                                    glo = g;
                                }
                                w0 = g == 0 ? v : w0;
                                w1 = g == 1 ? v : w1;
                                w2 = g == 2 ? v : w2;
                                w3 = g == 3 ? v : w3;
                                ghi = g + 1;
                                if (g == 3) {
                                    flush();
                                    glo = 4;
                                }
                            }
                            ++at;
                        }
                        ++found;
                    }
                }
            }
            int j = 1;
            while (j < D && o[j] == hi[j]) {
                o[j] = lo[j];
                ++j;
            }
            if (j >= D) break;
            ++o[j];
        }
    }
    if (kMode == 1 && glo != 4) flush();
    if (kMode == 0) {
        a.count[r] = found;
        a.count_k[k] = found;
    } else if (at != a.off[k + 1]) {
        atomicOr(a.overflow, 1u);  // the fill disagrees with the count
    }
}

// out[0] = max over counts[0..n); out must be 0 on entry. One atomic per
// block: atomics from every wave on the one address serialise in L2.
__global__ __launch_bounds__(kThreads) void k_rs_max(const uint32_t *__restrict__ counts, uint64_t n,
                                                      uint32_t *__restrict__ out) {
    __shared__ uint32_t wmax[kThreads / 64];
    uint32_t m = 0;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kThreads)
        m = counts[i] > m ? counts[i] : m;
    m = wave_max(m);
    if (lane_id() == 0) wmax[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 1; w < kThreads / 64; ++w) m = wmax[w] > m ? wmax[w] : m;
        if (m) atomicMax(out, m);
    }
}

// Tiled form: the cell key of every query row in S's grid, the row index as
// payload, and the number of rows left out (counted per wave, only by waves
// that have one: adds from every wave to one address would serialise). A
// query whose
// cell in some dimension is more than one cell outside the grid, or that has
// a coordinate that is not finite, has no adjacent cell: it gets the key
// 2^key_bits, past every cell id, and sorts last. A query one cell outside
// (cell -1 or dims) takes the edge cell instead: that only widens its
// candidate window, the distance test decides.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_rs_query_keys(const double *__restrict__ R, uint64_t nr, GridParams g,
                                                             int key_bits, K *__restrict__ keys,
                                                             uint32_t *__restrict__ ids,
                                                             uint32_t *__restrict__ nleft) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    bool valid = true;
    if (i < nr) {
        valid = true;
        uint64_t key = 0;
        for (uint32_t j = 0; j < g.d; ++j) {
            const double f = floor((R[i * g.d + j] - g.gmin[j]) / g.w);
            const double top = static_cast<double>(g.dims[j]);
            if (!(f >= -1.0) || !(f <= top)) {
                valid = false;
                break;
            }
            const uint64_t c = f <= 0.0 ? 0 : (f >= top - 1.0 ? g.dims[j] - 1 : static_cast<uint64_t>(f));
            key += c * g.stride[j];
        }
        keys[i] = static_cast<K>(valid ? key : (uint64_t{1} << key_bits));
        ids[i] = static_cast<uint32_t>(i);
    }
    const uint32_t w = wave_sum(valid ? 0u : 1u);
    if (lane_id() == 0 && w) atomicAdd(nleft, w);
}

template <int D>
void launch_rs_d(const RsArgs &a, int mode, hipStream_t s) {
    const unsigned nb = static_cast<unsigned>((a.nr + kThreads - 1) / kThreads);
    if (mode == 0) {
        KTimer kt_("rs_count", s);
        k_join_rs<D, 0><<<nb, kThreads, 0, s>>>(a);
    } else {
        KTimer kt_("rs_fill", s);
        k_join_rs<D, 1><<<nb, kThreads, 0, s>>>(a);
    }
    SJ_LAUNCH_CHECK();
}

}  // namespace

void launch_join_rs(const RsArgs &a, int mode, hipStream_t s) {
    if (a.nr == 0) return;
    switch (a.g.d) {
        case 1: launch_rs_d<1>(a, mode, s); break;
        case 2: launch_rs_d<2>(a, mode, s); break;
        case 3: launch_rs_d<3>(a, mode, s); break;
        case 4: launch_rs_d<4>(a, mode, s); break;
        case 5: launch_rs_d<5>(a, mode, s); break;
        case 6: launch_rs_d<6>(a, mode, s); break;
        case 7: launch_rs_d<7>(a, mode, s); break;
        case 8: launch_rs_d<8>(a, mode, s); break;
        default: throw Error(SJ_EINVAL, "two-set join: dimension out of range");
    }
}

void launch_rs_query_keys_u32(const double *R, uint64_t nr, const GridParams &g, int key_bits, uint32_t *keys,
                              uint32_t *ids, uint32_t *nleft, hipStream_t s) {
    if (nr == 0) return;
    KTimer kt_("rs_query_keys", s);
    k_rs_query_keys<uint32_t><<<static_cast<unsigned>((nr + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        R, nr, g, key_bits, keys, ids, nleft);
    SJ_LAUNCH_CHECK();
}

void launch_rs_query_keys_u64(const double *R, uint64_t nr, const GridParams &g, int key_bits, uint64_t *keys,
                              uint32_t *ids, uint32_t *nleft, hipStream_t s) {
    if (nr == 0) return;
    KTimer kt_("rs_query_keys", s);
    k_rs_query_keys<uint64_t><<<static_cast<unsigned>((nr + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        R, nr, g, key_bits, keys, ids, nleft);
    SJ_LAUNCH_CHECK();
}

void launch_rs_max(const uint32_t *counts, uint64_t n, uint32_t *out, hipStream_t s) {
    if (n == 0) return;
    const unsigned nb = static_cast<unsigned>(std::min<uint64_t>(256, (n + kThreads - 1) / kThreads));
    k_rs_max<<<nb, kThreads, 0, s>>>(counts, n, out);
    SJ_LAUNCH_CHECK();
}

}  // namespace sj
