// Grid-index construction kernels (Section IV-B and IV-C).
//
//   bbox        min/max per dimension and a NaN/Inf flag (g_j^min, g_j^max)
//   cell ids    c_j = clamp(floor((x_j - g_j^min) / w), 0, |g_j| - 1),
//               id = c_0 + |g_0| (c_1 + |g_1| (c_2 + ...))  (dimension 0 fastest,
//               as in the worked example of Section IV-D); the sort key
//               appends the dimension-0 sub-cell (width w / 2^sub_shift), so
//               that inside a cell the points are ordered by it
//   cells       after the sort by id: head flags, inclusive scan -> cell of
//               each point, B (distinct ids) and G (first point of each cell)
//   coords/M    per-cell coordinates and the per-dimension occupancy
//               bitmaps M_j
//   gather      cell-ordered structure-of-arrays copy of the coordinates
//               (X[j * n + r] = x[A[r]][j]) so the join reads each dimension
//               of consecutive candidates from consecutive addresses, instead
//               of the indirection D[A[k]] of Algorithm 1.
#include <cmath>

#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;

// Per-block partials: [min x kMaxDim][max x kMaxDim][non-finite flag].
constexpr int kBboxPart = 2 * kMaxDim + 1;

// D coordinates per point; each thread loads kBboxUnroll points before it
// folds any of them in, so that many loads are in flight per thread.
constexpr int kBboxUnroll = 4;

template <int D>
__global__ __launch_bounds__(kThreads) void k_bbox_partial(const double *__restrict__ pts,
                                                            uint64_t n, double *__restrict__ part) {
    double mn[kMaxDim], mx[kMaxDim];
#pragma unroll
    for (int j = 0; j < kMaxDim; ++j) {
        mn[j] = INFINITY;
        mx[j] = -INFINITY;
    }
    uint32_t flag = 0;
    auto fold = [&](const double (&v)[D]) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            flag |= !isfinite(v[j]);
            mn[j] = fmin(mn[j], v[j]);
            mx[j] = fmax(mx[j], v[j]);
        }
    };
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kThreads;
    uint64_t i = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    for (; i + (kBboxUnroll - 1) * stride < n; i += kBboxUnroll * stride) {
        double v[kBboxUnroll][D];
#pragma unroll
        for (int u = 0; u < kBboxUnroll; ++u)
#pragma unroll
            for (int j = 0; j < D; ++j) v[u][j] = pts[(i + u * stride) * D + j];
#pragma unroll
        for (int u = 0; u < kBboxUnroll; ++u) fold(v[u]);
    }
    for (; i < n; i += stride) {
        double v[D];
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = pts[i * D + j];
        fold(v);
    }
    __shared__ double smn[kThreads / 64][kMaxDim], smx[kThreads / 64][kMaxDim];
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double a = mn[j], b = mx[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a = fmin(a, __shfl_xor(a, off, 64));
            b = fmax(b, __shfl_xor(b, off, 64));
        }
        if (lane_id() == 0) {
            smn[wave][j] = a;
            smx[wave][j] = b;
        }
    }
    __shared__ uint32_t sbad;
    if (threadIdx.x == 0) sbad = 0;
    __syncthreads();
    if (ballot(flag != 0) != 0 && lane_id() == 0) sbad = 1;
    __syncthreads();
    double *mine = part + static_cast<size_t>(blockIdx.x) * kBboxPart;
    if (threadIdx.x < D) {
        const int j = threadIdx.x;
        double a = smn[0][j], b = smx[0][j];
        for (int w = 1; w < kThreads / 64; ++w) {
            a = fmin(a, smn[w][j]);
            b = fmax(b, smx[w][j]);
        }
        mine[j] = a;
        mine[kMaxDim + j] = b;
    }
    if (threadIdx.x == 0) mine[2 * kMaxDim] = sbad ? 1.0 : 0.0;
}

// Second stage: one workgroup reduces the per-block partials (all threads
// stride over the partials, then a wave/LDS reduction per dimension).
__global__ __launch_bounds__(kThreads) void k_bbox_final(const double *__restrict__ part,
                                                          uint32_t nblocks, uint32_t d,
                                                          double *__restrict__ out,
                                                          uint32_t *__restrict__ bad) {
    __shared__ double smn[kThreads / 64][kMaxDim], smx[kThreads / 64][kMaxDim];
    const int wave = threadIdx.x >> 6;
    {
        double f = 0.0;
        for (uint32_t k = threadIdx.x; k < nblocks; k += kThreads) f = fmax(f, part[k * kBboxPart + 2 * kMaxDim]);
        const bool any = __syncthreads_or(f != 0.0);
        if (threadIdx.x == 0) *bad = any ? 1u : 0u;
    }
    for (uint32_t j = 0; j < d; ++j) {
        double a = INFINITY, b = -INFINITY;
        for (uint32_t k = threadIdx.x; k < nblocks; k += kThreads) {
            a = fmin(a, part[k * kBboxPart + j]);
            b = fmax(b, part[k * kBboxPart + kMaxDim + j]);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a = fmin(a, __shfl_xor(a, off, 64));
            b = fmax(b, __shfl_xor(b, off, 64));
        }
        if (lane_id() == 0) {
            smn[wave][j] = a;
            smx[wave][j] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < d) {
        const int j = threadIdx.x;
        double a = smn[0][j], b = smx[0][j];
        for (int w = 1; w < kThreads / 64; ++w) {
            a = fmin(a, smn[w][j]);
            b = fmax(b, smx[w][j]);
        }
        out[j] = a;
        out[kMaxDim + j] = b;
    }
}

// Dimension-j cell coordinate of value v: clamp(floor((v - g_j^min) / w),
// 0, |g_j| - 1); |g_j| < 2^31. Every kernel that needs a cell coordinate of
// a point uses this one function, so they agree bit for bit.
__device__ __forceinline__ uint32_t cell_coord(double v, const GridParams &g, int j) {
    const double t = (v - g.gmin[j]) / g.w;
    const double top = static_cast<double>(g.dims[j] - 1);
    const double f = floor(t);
    return static_cast<uint32_t>(f <= 0.0 ? 0 : (f >= top ? g.dims[j] - 1 : static_cast<uint64_t>(f)));
}

// Dimension-0 coordinate in sub-cells of width w / 2^sub_shift, clamped to
// the grid like cell_coord. t * 2^sub_shift is exact, so the sub-cell
// shifted right by sub_shift is cell_coord(v, g, 0) (NaN gives 0).
__device__ __forceinline__ uint32_t sub_coord0(double v, const GridParams &g) {
    const double t = (v - g.gmin[0]) / g.w;
    const double f = floor(t * static_cast<double>(1u << g.sub_shift));
    const uint64_t top = (g.dims[0] << g.sub_shift) - 1;
    return static_cast<uint32_t>(!(f > 0.0) ? 0 : (f >= static_cast<double>(top) ? top : static_cast<uint64_t>(f)));
}

// Sort key of every point: its cell id, shifted left by sub_shift with the
// point's dimension-0 sub-cell inside the cell appended (sub_shift 0: the
// cell id).
template <typename K>
__global__ __launch_bounds__(kThreads) void k_cell_keys(const double *__restrict__ pts, uint64_t n,
                                                         GridParams g, K *__restrict__ keys,
                                                         uint32_t *__restrict__ ids) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (i >= n) return;
    uint64_t key = 0;
    for (uint32_t j = 0; j < g.d; ++j)
        key += static_cast<uint64_t>(cell_coord(pts[i * g.d + j], g, static_cast<int>(j))) * g.stride[j];
    if (g.sub_shift)
        key = (key << g.sub_shift) | (sub_coord0(pts[i * g.d], g) & ((1u << g.sub_shift) - 1u));
    keys[i] = static_cast<K>(key);
    ids[i] = static_cast<uint32_t>(i);
}

template <typename K>
__global__ __launch_bounds__(kThreads) void k_cell_tables(const K *__restrict__ k, uint64_t n, int shift,
                                                           uint32_t *__restrict__ cell_of,
                                                           uint64_t *__restrict__ B,
                                                           uint32_t *__restrict__ starts) {
    const uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r >= n) return;
    const uint32_t h = cell_of[r] - 1u;  // inclusive scan of head flags
    cell_of[r] = h;
    if (r == 0 || (k[r] >> shift) != (k[r - 1] >> shift)) {
        B[h] = static_cast<uint64_t>(k[r] >> shift);
        starts[h] = static_cast<uint32_t>(r);
    }
    if (r == n - 1) starts[h + 1] = static_cast<uint32_t>(n);
}

// Per-cell coordinates decoded from the linear id; occupancy bitmaps M_j
// (privatised in LDS when they fit); largest cell.
constexpr uint32_t kMaskLdsWords = 8192;

__global__ __launch_bounds__(kThreads) void k_cell_coords(const uint64_t *__restrict__ B,
                                                           const uint32_t *__restrict__ starts,
                                                           const uint32_t *__restrict__ last_cell,
                                                           GridParams g,
                                                           uint32_t *__restrict__ coords,
                                                           uint32_t *__restrict__ masks,
                                                           MaskOffsets mask_off,
                                                           uint32_t mask_words,
                                                           uint32_t *__restrict__ max_pts) {
    __shared__ uint32_t lmask[kMaskLdsWords];
    const uint64_t ncells = static_cast<uint64_t>(*last_cell) + 1;  // cell of the last sorted point + 1
    const bool use_lds = masks != nullptr && mask_words <= kMaskLdsWords;
    if (use_lds)
        for (uint32_t i = threadIdx.x; i < mask_words; i += kThreads) lmask[i] = 0;
    __syncthreads();
    uint32_t mp = 0;
    // cell h: coordinates decoded from its id, occupancy bits, size
    auto cell = [&](uint64_t h, uint64_t id, uint32_t sz) {
        for (uint32_t j = 0; j < g.d; ++j) {
            uint32_t c;
            if (id < (1ull << 32) && g.dims[j] < (1ull << 32)) {  // 32-bit division when it fits
                const uint32_t id32 = static_cast<uint32_t>(id), dj = static_cast<uint32_t>(g.dims[j]);
                c = id32 % dj;
                id = id32 / dj;
            } else {
                c = static_cast<uint32_t>(id % g.dims[j]);
                id /= g.dims[j];
            }
            coords[h * g.d + j] = c;
            if (!masks) continue;
            const uint32_t w = mask_off.off[j] + (c >> 5);
            const uint32_t bit = 1u << (c & 31u);
            // most bits are set by the first cells that have them: test first
            if (use_lds) {
                if (!(lmask[w] & bit)) atomicOr(&lmask[w], bit);
            } else {
                atomicOr(&masks[w], bit);
            }
        }
        mp = sz > mp ? sz : mp;
    };
    // four cells per thread and step, their loads issued before any is used
    constexpr int kU = 4;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kThreads;
    for (uint64_t h0 = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x; h0 < ncells;
         h0 += kU * stride) {
        uint64_t ids[kU];
        uint32_t s0[kU], s1[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint64_t h = h0 + u * stride;
            const bool in = h < ncells;
            ids[u] = in ? B[h] : 0;
            s0[u] = in ? starts[h] : 0;
            s1[u] = in ? starts[h + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (h0 + u * stride < ncells) cell(h0 + u * stride, ids[u], s1[u] - s0[u]);
    }
    mp = wave_max(mp);
    __shared__ uint32_t smp[kThreads / 64];
    if (lane_id() == 0) smp[threadIdx.x >> 6] = mp;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = smp[0];
        for (int w = 1; w < kThreads / 64; ++w) m = smp[w] > m ? smp[w] : m;
        atomicMax(max_pts, m);
    }
    if (use_lds)
        for (uint32_t i = threadIdx.x; i < mask_words; i += kThreads)
            if (lmask[i]) atomicOr(&masks[i], lmask[i]);
}

// Zeroes p[0..n) and q[0..m) in one launch.
__global__ void k_zero2_u32(uint32_t *p, uint64_t n, uint32_t *q, uint64_t m) {
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n + m; i += step) {
        if (i < n)
            p[i] = 0;
        else
            q[i - n] = 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_gather_soa(const double *__restrict__ pts,
                                                          const uint32_t *__restrict__ perm,
                                                          uint64_t n, uint32_t d,
                                                          double *__restrict__ X, GridParams g,
                                                          uint32_t *__restrict__ cx) {
    const uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r >= n) return;
    const uint64_t i = perm[r];
    for (uint32_t j = 0; j < d; ++j) X[j * n + r] = pts[i * d + j];
    cx[r] = sub_coord0(pts[i * d], g);
}

// Even d with 16-byte aligned rows: one 16-byte load per coordinate pair.
template <int D>
__global__ __launch_bounds__(kThreads) void k_gather_soa_v2(const double2 *__restrict__ pts,
                                                             const uint32_t *__restrict__ perm,
                                                             uint64_t n, double *__restrict__ X, GridParams g,
                                                             uint32_t *__restrict__ cx) {
    const uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r >= n) return;
    const uint64_t i = perm[r];
    double2 v[D / 2];
#pragma unroll
    for (int k = 0; k < D / 2; ++k) v[k] = pts[i * (D / 2) + k];
#pragma unroll
    for (int k = 0; k < D / 2; ++k) {
        X[(2 * k) * n + r] = v[k].x;
        X[(2 * k + 1) * n + r] = v[k].y;
    }
    cx[r] = sub_coord0(v[0].x, g);
}

__global__ __launch_bounds__(kThreads) void k_make_f32(const double *__restrict__ X, uint64_t n,
                                                        uint32_t d, GridParams shift,
                                                        float *__restrict__ Y) {
    const uint64_t r = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (r >= n) return;
    for (uint32_t j = 0; j < d; ++j)
        Y[j * n + r] = static_cast<float>(X[j * n + r] - shift.gmin[j]);
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, uint64_t n, T v) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

inline unsigned blocks_for(uint64_t n) {
    return static_cast<unsigned>((n + kThreads - 1) / kThreads);
}

}  // namespace

// Zeroes up to four word ranges with one launch.
__global__ void k_zero_spans(ZeroSpans z) {
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    const uint64_t tid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
    for (int k = 0; k < z.count; ++k)
        for (uint64_t i = tid; i < z.words[k]; i += step) z.p[k][i] = 0;
}

void launch_zero_spans(const ZeroSpans &z, hipStream_t s) {
    uint64_t most = 0;
    for (int k = 0; k < z.count; ++k) most = std::max<uint64_t>(most, z.words[k]);
    if (!most) return;
    const unsigned nb = static_cast<unsigned>(std::min<uint64_t>(2048, (most + kThreads - 1) / kThreads));
    k_zero_spans<<<nb, kThreads, 0, s>>>(z);
    SJ_LAUNCH_CHECK();
}

void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
    if (!n) return;
    const unsigned nb = static_cast<unsigned>(std::min<uint64_t>(4096, (n + kThreads - 1) / kThreads));
    k_fill<uint32_t><<<nb, kThreads, 0, s>>>(p, n, v);
    SJ_LAUNCH_CHECK();
}

void launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
    if (!n) return;
    const unsigned nb = static_cast<unsigned>(std::min<uint64_t>(4096, (n + kThreads - 1) / kThreads));
    k_fill<uint64_t><<<nb, kThreads, 0, s>>>(p, n, v);
    SJ_LAUNCH_CHECK();
}

// Y[j][r] = fl32(X[j][r] - shift_j); the shift travels in GridParams::gmin.
void launch_make_f32(const double *X, uint64_t n, uint32_t d, const double *shift, float *Y,
                     hipStream_t s) {
    GridParams g{};
    for (uint32_t j = 0; j < d && j < static_cast<uint32_t>(kMaxDim); ++j) g.gmin[j] = shift[j];
    {
        KTimer kt_("make_f32", s);
        k_make_f32<<<blocks_for(n), kThreads, 0, s>>>(X, n, d, g, Y);
        SJ_LAUNCH_CHECK();
    }
}

void launch_bbox(const double *pts, uint64_t n, uint32_t d, double *bbox_out, uint32_t *bad,
                 hipStream_t s) {
    const uint32_t nb = static_cast<uint32_t>(std::min<uint64_t>(1024, (n + kThreads - 1) / kThreads));
    DevBuf<double> part(static_cast<size_t>(nb) * kBboxPart);
    {
        KTimer kt_("bbox", s);
        switch (d) {
            case 1: k_bbox_partial<1><<<nb, kThreads, 0, s>>>(pts, n, part.ptr); break;
            case 2: k_bbox_partial<2><<<nb, kThreads, 0, s>>>(pts, n, part.ptr); break;
            case 3: k_bbox_partial<3><<<nb, kThreads, 0, s>>>(pts, n, part.ptr); break;
            case 4: k_bbox_partial<4><<<nb, kThreads, 0, s>>>(pts, n, part.ptr); break;
            case 5: k_bbox_partial<5><<<nb, kThreads, 0, s>>>(pts, n, part.ptr); break;
            case 6: k_bbox_partial<6><<<nb, kThreads, 0, s>>>(pts, n, part.ptr); break;
            case 7: k_bbox_partial<7><<<nb, kThreads, 0, s>>>(pts, n, part.ptr); break;
            case 8: k_bbox_partial<8><<<nb, kThreads, 0, s>>>(pts, n, part.ptr); break;
            default: throw Error(SJ_EINVAL, "bbox: dimension out of range");
        }
        SJ_LAUNCH_CHECK();
    }
    k_bbox_final<<<1, kThreads, 0, s>>>(part.ptr, nb, d, bbox_out, bad);
    SJ_LAUNCH_CHECK();
}

void launch_cell_keys_u64(const double *pts, uint64_t n, const GridParams &g, uint64_t *keys,
                          uint32_t *ids, hipStream_t s) {
    {
        KTimer kt_("cell_keys", s);
        k_cell_keys<uint64_t><<<blocks_for(n), kThreads, 0, s>>>(pts, n, g, keys, ids);
        SJ_LAUNCH_CHECK();
    }
}

void launch_cell_keys_u32(const double *pts, uint64_t n, const GridParams &g, uint32_t *keys,
                          uint32_t *ids, hipStream_t s) {
    {
        KTimer kt_("cell_keys", s);
        k_cell_keys<uint32_t><<<blocks_for(n), kThreads, 0, s>>>(pts, n, g, keys, ids);
        SJ_LAUNCH_CHECK();
    }
}

template <typename K>
void build_cells(const K *sorted_keys, uint64_t n, int shift, uint32_t *cell_of, uint64_t *B, uint32_t *starts,
                 hipStream_t s) {
    scan_head_flags_inclusive<K>(sorted_keys, shift, cell_of, n, s);
    {
        KTimer kt_("cell_tables", s);
        k_cell_tables<K><<<blocks_for(n), kThreads, 0, s>>>(sorted_keys, n, shift, cell_of, B, starts);
        SJ_LAUNCH_CHECK();
    }
}

template void build_cells<uint64_t>(const uint64_t *, uint64_t, int, uint32_t *, uint64_t *, uint32_t *,
                                    hipStream_t);
template void build_cells<uint32_t>(const uint32_t *, uint64_t, int, uint32_t *, uint64_t *, uint32_t *,
                                    hipStream_t);

void launch_cell_coords_masks(const uint64_t *B, const uint32_t *starts, uint64_t ncells_bound,
                              const uint32_t *last_cell, const GridParams &g, uint32_t *coords, uint32_t *masks,
                              const MaskOffsets &mask_off, uint32_t mask_words, uint32_t *max_pts,
                              hipStream_t s) {
    const uint64_t mw = masks ? mask_words : 0;
    k_zero2_u32<<<static_cast<unsigned>(std::min<uint64_t>(64, mw / 256 + 1)), 256, 0, s>>>(masks, mw, max_pts, 1);
    SJ_LAUNCH_CHECK();
    // few workgroups: each flushes its LDS copy of the masks with atomics
    const unsigned nb = static_cast<unsigned>(std::min<uint64_t>(256, (ncells_bound + kThreads - 1) / kThreads));
    {
        KTimer kt_("cell_coords_masks", s);
        k_cell_coords<<<nb, kThreads, 0, s>>>(B, starts, last_cell, g, coords, masks, mask_off, mask_words,
                                             max_pts);
        SJ_LAUNCH_CHECK();
    }
}

void launch_gather_soa(const double *pts, const uint32_t *perm, uint64_t n, uint32_t d, double *X,
                       const GridParams &g, uint32_t *cx, hipStream_t s) {
    {
        KTimer kt_("gather_soa", s);
        const bool al16 = (reinterpret_cast<uintptr_t>(pts) & 15u) == 0;
        const double2 *p2 = reinterpret_cast<const double2 *>(pts);
        if (al16 && d == 2)
            k_gather_soa_v2<2><<<blocks_for(n), kThreads, 0, s>>>(p2, perm, n, X, g, cx);
        else if (al16 && d == 4)
            k_gather_soa_v2<4><<<blocks_for(n), kThreads, 0, s>>>(p2, perm, n, X, g, cx);
        else if (al16 && d == 6)
            k_gather_soa_v2<6><<<blocks_for(n), kThreads, 0, s>>>(p2, perm, n, X, g, cx);
        else if (al16 && d == 8)
            k_gather_soa_v2<8><<<blocks_for(n), kThreads, 0, s>>>(p2, perm, n, X, g, cx);
        else
            k_gather_soa<<<blocks_for(n), kThreads, 0, s>>>(pts, perm, n, d, X, g, cx);
        SJ_LAUNCH_CHECK();
    }
}

}  // namespace sj
