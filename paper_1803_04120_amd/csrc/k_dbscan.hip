// DBSCAN over the join's neighbour table: the density-based clustering that
// Section I names as a consumer of the self-join (and whose GPU
// neighbourhood computation the batching of Section V-A comes from).
//
// Input: the self-join result as a compressed sparse row table -- row i of
// the table holds every j with d2(i, j) <= eps^2, i itself included -- so
// |N_eps(i)| is the row length. With that table the clustering of Ester et
// al. is fixed except for border points reachable from two clusters; the
// labels here are:
//   core point   (row length >= min_pts): the smallest index of the core
//                points of its cluster, a cluster being a connected
//                component of the graph of core points joined by the table's
//                entries;
//   border point (not core, some core point in its row): the label of the
//                smallest-index core point in its row;
//   noise        -1.
//
// Components by lock-free union-find over the label array itself: a core
// point starts as its own parent; for every table entry (i, j) with both
// ends core and j > i the two trees are joined by hooking the larger root
// under the smaller with a compare-and-swap (retried from the new parent if
// another thread hooked it first). A parent is never larger than its child,
// so the root of a finished tree is its smallest member, and path halving
// (a node re-pointed at its grandparent, an ancestor) is safe under races.
// Parent loads and path-halving stores are relaxed device-scope atomics, so
// no lane spins on a stale cached parent.
#include "sj_internal.h"
#include "sj_device.h"

namespace sj {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int32_t ld(int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t find_root(int32_t *par, int32_t x) {
    while (true) {
        const int32_t p = ld(par + x);
        if (p == x) return x;
        const int32_t gp = ld(par + p);
        if (gp == p) return p;
        st(par + x, gp);  // path halving
        x = gp;
    }
}

// The same walk without path halving: in the final pass every core point
// overwrites its own entry with its root, and a halving store racing with
// that write could put back an intermediate ancestor.
__device__ __forceinline__ int32_t find_root_ro(int32_t *par, int32_t x) {
    while (true) {
        const int32_t p = ld(par + x);
        if (p == x) return x;
        x = p;
    }
}

__device__ __forceinline__ void unite(int32_t *par, int32_t a, int32_t b) {
    while (true) {
        a = find_root(par, a);
        b = find_root(par, b);
        if (a == b) return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        // hook the larger root a under the smaller root b
        const int32_t old = atomicCAS(par + a, a, b);
        if (old == a) return;
        a = old;  // a was hooked meanwhile: continue from its parent
    }
}

__device__ __forceinline__ bool is_core(const uint64_t *off, uint64_t i, uint32_t min_pts) {
    return off[i + 1] - off[i] >= min_pts;
}

__global__ __launch_bounds__(kThreads) void k_db_init(const uint64_t *__restrict__ off, uint64_t n, uint32_t min_pts,
                                                       int32_t *__restrict__ label) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    if (i < n) label[i] = is_core(off, i, min_pts) ? static_cast<int32_t>(i) : -1;
}

// One 16-lane group per row: the entries j > i of a core row i whose row is
// also core are united with i.
__global__ __launch_bounds__(kThreads) void k_db_union(const uint64_t *__restrict__ off,
                                                        const uint32_t *__restrict__ cols, uint64_t n,
                                                        uint32_t min_pts, int32_t *label) {
    const uint32_t l = threadIdx.x & 15u;
    const uint64_t groups = static_cast<uint64_t>(gridDim.x) * (kThreads / 16);
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(kThreads / 16) + (threadIdx.x >> 4); i < n; i += groups) {
        if (!is_core(off, i, min_pts)) continue;
        const uint64_t a = off[i], b = off[i + 1];
        for (uint64_t e = a + l; e < b; e += 16) {
            const uint32_t j = cols[e];
            if (j > i && is_core(off, j, min_pts)) unite(label, static_cast<int32_t>(i), static_cast<int32_t>(j));
        }
    }
}

// Every core point points straight at its root; roots are counted. Only
// own-entry stores of roots happen here, so every entry any walk reads is
// an ancestor of its node and every walk ends at the true root.
__global__ __launch_bounds__(kThreads) void k_db_compress(const uint64_t *__restrict__ off, uint64_t n,
                                                           uint32_t min_pts, int32_t *label,
                                                           unsigned long long *nclusters) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kThreads) + threadIdx.x;
    bool root = false;
    if (i < n && is_core(off, i, min_pts)) {
        const int32_t r = find_root_ro(label, static_cast<int32_t>(i));
        st(label + i, r);
        root = r == static_cast<int32_t>(i);
    }
    const uint64_t m = ballot(root);
    if (lane_id() == 0 && m) atomicAdd(nclusters, static_cast<unsigned long long>(__popcll(m)));
}

// A border point takes the label of the smallest-index core point in its
// row; a non-core point with none stays noise.
__global__ __launch_bounds__(kThreads) void k_db_border(const uint64_t *__restrict__ off,
                                                         const uint32_t *__restrict__ cols, uint64_t n,
                                                         uint32_t min_pts, int32_t *__restrict__ label) {
    const uint32_t l = threadIdx.x & 15u;
    const uint64_t groups = static_cast<uint64_t>(gridDim.x) * (kThreads / 16);
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(kThreads / 16) + (threadIdx.x >> 4); i < n; i += groups) {
        if (is_core(off, i, min_pts)) continue;  // uniform across the group
        uint32_t best = 0xffffffffu;
        const uint64_t a = off[i], b = off[i + 1];
        for (uint64_t e = a + l; e < b; e += 16) {
            const uint32_t j = cols[e];
            if (j < best && is_core(off, j, min_pts)) best = j;
        }
#pragma unroll
        for (int w = 8; w > 0; w >>= 1) {
            const uint32_t o = static_cast<uint32_t>(__shfl_xor(static_cast<int>(best), w, 16));
            best = o < best ? o : best;
        }
        if (l == 0 && best != 0xffffffffu) label[i] = label[best];
    }
}

inline unsigned blocks_for(uint64_t n) { return static_cast<unsigned>((n + kThreads - 1) / kThreads); }
inline unsigned group_blocks(uint64_t n) {
    return static_cast<unsigned>(std::min<uint64_t>((n + kThreads / 16 - 1) / (kThreads / 16), 65536));
}

}  // namespace

void launch_dbscan(const uint64_t *off, const uint32_t *cols, uint64_t n, uint32_t min_pts, int32_t *label,
                   unsigned long long *nclusters, hipStream_t s) {
    if (n == 0) return;
    if (n > 0x7fffffffULL) throw Error(SJ_EINVAL, "dbscan: more than 2^31 - 1 points");
    k_db_init<<<blocks_for(n), kThreads, 0, s>>>(off, n, min_pts, label);
    SJ_LAUNCH_CHECK();
    {
        KTimer kt_("dbscan_union", s);
        k_db_union<<<group_blocks(n), kThreads, 0, s>>>(off, cols, n, min_pts, label);
        SJ_LAUNCH_CHECK();
    }
    k_db_compress<<<blocks_for(n), kThreads, 0, s>>>(off, n, min_pts, label, nclusters);
    SJ_LAUNCH_CHECK();
    k_db_border<<<group_blocks(n), kThreads, 0, s>>>(off, cols, n, min_pts, label);
    SJ_LAUNCH_CHECK();
}

}  // namespace sj
