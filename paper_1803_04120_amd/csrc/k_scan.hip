// Device-wide prefix sums (reduce, scan the tile sums, rescan the tiles).
// Used for the cell table (head flags), candidate-range offsets, result-row
// offsets and the radix-sort digit tables.
#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;

template <typename Tin, typename Tacc>
__global__ __launch_bounds__(kThreads) void k_tile_sum(const Tin *__restrict__ in, size_t n,
                                                        Tacc *__restrict__ part) {
    __shared__ Tacc lds[kThreads / 64];
    const size_t base = static_cast<size_t>(blockIdx.x) * kTile;
    Tacc s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const size_t i = base + static_cast<size_t>(k) * kThreads + threadIdx.x;
        if (i < n) s += static_cast<Tacc>(in[i]);
    }
    Tacc tot;
    block_exclusive_scan<Tacc, kThreads>(s, &tot, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Exclusive scan of part[0..m) in place by one block; part[m] gets the total.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_partials(T *__restrict__ part, size_t m) {
    __shared__ T lds[kThreads / 64];
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

template <typename Tin, typename Tout, bool kInclusive>
__global__ __launch_bounds__(kThreads) void k_tile_scan(const Tin *in, Tout *out, size_t n,
                                                         const Tout *__restrict__ part,
                                                         Tout *total_out) {
    __shared__ Tout tile[kTile];
    __shared__ Tout lds[kThreads / 64];
    const size_t base = static_cast<size_t>(blockIdx.x) * kTile;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = k * kThreads + threadIdx.x;
        tile[i] = (base + i < n) ? static_cast<Tout>(in[base + i]) : Tout(0);
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
    Tout run = block_exclusive_scan<Tout, kThreads>(s, &tot, lds) + part[blockIdx.x];
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
    if (total_out && blockIdx.x == 0 && threadIdx.x == 0) {
        const size_t nb = (n + kTile - 1) / kTile;
        *total_out = part[nb];
    }
}

template <typename T>
__global__ void k_set_value(T *p, T v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

template <typename Tin, typename Tout, bool kInclusive>
void scan_impl(const Tin *in, Tout *out, size_t n, Tout *total_out, hipStream_t s) {
    if (n == 0) {
        if (total_out) {
            k_set_value<Tout><<<1, 64, 0, s>>>(total_out, Tout(0));
            SJ_LAUNCH_CHECK();
        }
        return;
    }
    const size_t nb = (n + kTile - 1) / kTile;
    if (nb > 0x7fffffffULL) throw Error(SJ_EINVAL, "scan: input too large");
    DevBuf<Tout> part(nb + 1);
    k_tile_sum<Tin, Tout><<<static_cast<unsigned>(nb), kThreads, 0, s>>>(in, n, part.ptr);
    SJ_LAUNCH_CHECK();
    k_scan_partials<Tout><<<1, kThreads, 0, s>>>(part.ptr, nb);
    SJ_LAUNCH_CHECK();
    {
        KTimer kt_("scan", s);
        k_tile_scan<Tin, Tout, kInclusive><<<static_cast<unsigned>(nb), kThreads, 0, s>>>(
            in, out, n, part.ptr, total_out);
        SJ_LAUNCH_CHECK();
    }
}

}  // namespace

void scan_exclusive_u32_to_u64(const uint32_t *in, uint64_t *out, size_t n, hipStream_t s) {
    scan_impl<uint32_t, uint64_t, false>(in, out, n, out + n, s);
}

void scan_inclusive_u32(uint32_t *data, size_t n, hipStream_t s) {
    scan_impl<uint32_t, uint32_t, true>(data, data, n, nullptr, s);
}

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, size_t n, hipStream_t s) {
    scan_impl<uint32_t, uint32_t, false>(in, out, n, nullptr, s);
}

}  // namespace sj
