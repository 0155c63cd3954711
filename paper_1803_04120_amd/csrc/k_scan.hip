// Device-wide prefix sums. Used for the cell table (head flags), chunk and
// row offsets, and the radix-sort digit tables.
//
// Two kernels: (1) every tile of 2048 inputs writes its sum; (2) every tile
// adds up the sums of the tiles before it (all threads of the workgroup
// share that reduction; at most 2048 tiles, ~4M inputs) and scans itself.
// Longer inputs first scan the tile sums in place with a third kernel.
// Inputs come through a loader, so a scan can consume a value computed on
// the fly (the head flag of a sorted key, key[r] != key[r-1]) instead of a
// materialised array.
#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;
constexpr size_t kInlineTiles = 2048;

template <typename T>
struct ArrayLoad {
    const T *p;
    __device__ __forceinline__ T operator()(size_t i) const { return p[i]; }
};

template <typename K>
struct HeadFlagLoad {
    const K *k;
    int shift;  // keys equal after this right shift are one cell
    __device__ __forceinline__ uint32_t operator()(size_t i) const {
        return (i == 0 || (k[i] >> shift) != (k[i - 1] >> shift)) ? 1u : 0u;
    }
};

// Up to two independent scans of the same length run in one launch
// (blockIdx.y picks the operand set); each has its own tile-sum row.
template <typename Tout, typename Load>
struct ScanOps {
    Load in[2];
    Tout *out[2];
    Tout *total[2];
};

// Grid-row head flag of cell h: its dimension-1..d-1 coordinates differ
// from those of cell h - 1 (cells sorted by linear id, dimension 0 fastest).
struct RowHeadLoad {
    const uint32_t *coords;
    uint32_t d;
    __device__ __forceinline__ uint32_t operator()(size_t h) const {
        if (h == 0) return 1u;
        uint32_t f = 0;
        for (uint32_t j = 1; j < d; ++j) f |= coords[h * d + j] != coords[(h - 1) * d + j];
        return f;
    }
};

// Chunks of grid row r (ceil(points / 64)); rows past the row count (the
// total of the row-head scan, row_of[ncells]) have none.
struct RowChunksLoad {
    const uint32_t *row_pt;
    const uint64_t *row_of;
    size_t ncells;
    __device__ __forceinline__ uint32_t operator()(size_t r) const {
        if (r >= row_of[ncells]) return 0u;
        return (row_pt[r + 1] - row_pt[r] + 63u) / 64u;
    }
};

// 1 for a row longer than lo entries (row lengths from offsets).
struct LongRowLoad {
    const uint64_t *off;
    uint32_t lo;
    __device__ __forceinline__ uint32_t operator()(size_t r) const { return off[r + 1] - off[r] > lo ? 1u : 0u; }
};

template <typename Tacc, typename Load>
__global__ __launch_bounds__(kThreads) void k_tile_sum(ScanOps<Tacc, Load> ops, size_t n,
                                                        Tacc *__restrict__ part_all) {
    __shared__ Tacc lds[kThreads / 64];
    const Load in = ops.in[blockIdx.y];
    const size_t nb = (n + kTile - 1) / kTile;
    Tacc *part = part_all + blockIdx.y * (nb + 1);
    const size_t base = static_cast<size_t>(blockIdx.x) * kTile;
    Tacc s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const size_t i = base + static_cast<size_t>(k) * kThreads + threadIdx.x;
        if (i < n) s += static_cast<Tacc>(in(i));
    }
    Tacc tot;
    block_exclusive_scan<Tacc, kThreads>(s, &tot, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Exclusive scan of part[0..m) in place by one block; part[m] gets the total.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_partials(T *__restrict__ part_all, size_t m) {
    __shared__ T lds[kThreads / 64];
    T *part = part_all + blockIdx.x * (m + 1);
    T carry = 0;
    for (size_t base = 0; base < m; base += kThreads) {
        const size_t i = base + threadIdx.x;
        const T v = i < m ? part[i] : T(0);
        T tot;
        const T ex = block_exclusive_scan<T, kThreads>(v, &tot, lds);
        if (i < m) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) part[m] = carry;
}

// inline_prefix: part holds raw tile sums and every tile sums the ones before
// it; otherwise part already holds the exclusive tile offsets (+ total at nb).
template <typename Tout, bool kInclusive, typename Load>
__global__ __launch_bounds__(kThreads) void k_tile_scan(ScanOps<Tout, Load> ops, size_t n,
                                                         const Tout *__restrict__ part_all,
                                                         int inline_prefix) {
    __shared__ Tout tile[kTile];
    __shared__ Tout lds[kThreads / 64];
    const Load in = ops.in[blockIdx.y];
    Tout *out = ops.out[blockIdx.y];
    Tout *total_out = ops.total[blockIdx.y];
    const size_t base = static_cast<size_t>(blockIdx.x) * kTile;
    const size_t nb = (n + kTile - 1) / kTile;
    const Tout *part = part_all + blockIdx.y * (nb + 1);
    Tout prefix = 0, grand = 0;
    if (inline_prefix) {
        Tout s = 0, all = 0;
        for (size_t b = threadIdx.x; b < nb; b += kThreads) {
            const Tout v = part[b];
            if (b < blockIdx.x) s += v;
            all += v;
        }
        Tout tot;
        block_exclusive_scan<Tout, kThreads>(s, &tot, lds);
        prefix = tot;
        Tout tot2;
        block_exclusive_scan<Tout, kThreads>(all, &tot2, lds);
        grand = tot2;
    } else {
        prefix = part[blockIdx.x];
        grand = part[nb];
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = k * kThreads + threadIdx.x;
        tile[i] = (base + i < n) ? static_cast<Tout>(in(base + i)) : Tout(0);
    }
    __syncthreads();
    Tout loc[kItems];
    Tout s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        loc[k] = tile[threadIdx.x * kItems + k];
        s += loc[k];
    }
    Tout tot;
    Tout run = block_exclusive_scan<Tout, kThreads>(s, &tot, lds) + prefix;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (kInclusive) {
            run += loc[k];
            tile[threadIdx.x * kItems + k] = run;
        } else {
            tile[threadIdx.x * kItems + k] = run;
            run += loc[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = k * kThreads + threadIdx.x;
        if (base + i < n) out[base + i] = tile[i];
    }
    if (total_out && blockIdx.x == 0 && threadIdx.x == 0) *total_out = grand;
}

template <typename T>
__global__ void k_set_values(T *p, T *q, T v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (p) *p = v;
        if (q) *q = v;
    }
}

// nscans = 1 or 2 (ops.in[1] etc. unused for one).
template <typename Tout, bool kInclusive, typename Load>
void scan_impl(const ScanOps<Tout, Load> &ops, unsigned nscans, size_t n, hipStream_t s,
               Tout *part_ws = nullptr) {
    if (n == 0) {
        if (ops.total[0] || (nscans > 1 && ops.total[1])) {
            k_set_values<Tout><<<1, 64, 0, s>>>(ops.total[0], nscans > 1 ? ops.total[1] : nullptr, Tout(0));
            SJ_LAUNCH_CHECK();
        }
        return;
    }
    const size_t nb = (n + kTile - 1) / kTile;
    if (nb > 0x7fffffffULL) throw Error(SJ_EINVAL, "scan: input too large");
    DevBuf<Tout> part_own;
    Tout *part = part_ws;
    if (!part) {
        part_own.reset(nscans * (nb + 1));
        part = part_own.ptr;
    }
    k_tile_sum<Tout, Load><<<dim3(static_cast<unsigned>(nb), nscans), kThreads, 0, s>>>(ops, n, part);
    SJ_LAUNCH_CHECK();
    const int inline_prefix = nb <= kInlineTiles ? 1 : 0;
    if (!inline_prefix) {
        k_scan_partials<Tout><<<nscans, kThreads, 0, s>>>(part, nb);
        SJ_LAUNCH_CHECK();
    }
    KTimer kt_("scan", s);
    k_tile_scan<Tout, kInclusive, Load><<<dim3(static_cast<unsigned>(nb), nscans), kThreads, 0, s>>>(
        ops, n, part, inline_prefix);
    SJ_LAUNCH_CHECK();
}

template <typename Tout, bool kInclusive, typename Load>
void scan_one(Load in, Tout *out, size_t n, Tout *total, hipStream_t s) {
    ScanOps<Tout, Load> ops{{in, in}, {out, out}, {total, nullptr}};
    scan_impl<Tout, kInclusive, Load>(ops, 1, n, s);
}

}  // namespace

void scan_exclusive_u32_to_u64(const uint32_t *in, uint64_t *out, size_t n, hipStream_t s) {
    scan_one<uint64_t, false>(ArrayLoad<uint32_t>{in}, out, n, out + n, s);
}

size_t scan_partials(size_t n) { return (n + kTile - 1) / kTile + 1; }

void scan_exclusive_u32_to_u64_ws(const uint32_t *in, uint64_t *out, size_t n, uint64_t *part, hipStream_t s) {
    ScanOps<uint64_t, ArrayLoad<uint32_t>> ops{{{in}, {in}}, {out, out}, {out + n, nullptr}};
    scan_impl<uint64_t, false>(ops, 1, n, s, part);
}

void scan_exclusive_u32_to_u64_x2(const uint32_t *in0, uint64_t *out0, const uint32_t *in1,
                                  uint64_t *out1, size_t n, hipStream_t s) {
    ScanOps<uint64_t, ArrayLoad<uint32_t>> ops{{{in0}, {in1}}, {out0, out1}, {out0 + n, out1 + n}};
    scan_impl<uint64_t, false>(ops, 2, n, s);
}

void scan_inclusive_u32(uint32_t *data, size_t n, hipStream_t s) {
    scan_one<uint32_t, true>(ArrayLoad<uint32_t>{data}, data, n, nullptr, s);
}

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, size_t n, hipStream_t s) {
    scan_one<uint32_t, false>(ArrayLoad<uint32_t>{in}, out, n, nullptr, s);
}

void scan_row_heads_exclusive(const uint32_t *coords, uint32_t d, uint64_t *row_of, size_t ncells,
                              hipStream_t s) {
    scan_one<uint64_t, false>(RowHeadLoad{coords, d}, row_of, ncells, row_of + ncells, s);
}

void scan_row_chunks_exclusive(const uint32_t *row_pt, const uint64_t *row_of, uint64_t *ch_off, size_t ncells,
                               hipStream_t s) {
    scan_one<uint64_t, false>(RowChunksLoad{row_pt, row_of, ncells}, ch_off, ncells, ch_off + ncells, s);
}

void scan_long_rows_exclusive(const uint64_t *off, uint32_t lo, uint32_t *pos, size_t rows, hipStream_t s) {
    scan_one<uint32_t, false>(LongRowLoad{off, lo}, pos, rows, pos + rows, s);
}

template <typename K>
void scan_head_flags_inclusive(const K *sorted_keys, int shift, uint32_t *out, size_t n, hipStream_t s) {
    scan_one<uint32_t, true>(HeadFlagLoad<K>{sorted_keys, shift}, out, n, nullptr, s);
}
template void scan_head_flags_inclusive<uint32_t>(const uint32_t *, int, uint32_t *, size_t, hipStream_t);
template void scan_head_flags_inclusive<uint64_t>(const uint64_t *, int, uint32_t *, size_t, hipStream_t);

}  // namespace sj
