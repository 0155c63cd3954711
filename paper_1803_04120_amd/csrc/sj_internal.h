// Internal declarations shared by the HIP translation units of libsj.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <exception>
#include <stdexcept>
#include <string>

#include "sj.h"
#include "sj_args.h"

namespace sj {

// Error carried from the internals to the C ABI boundary, where it becomes
// a return code and the thread-local message.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char *what, const char *file, int line);
#define SJ_HIP(call) ::sj::hip_check((call), #call, __FILE__, __LINE__)
#define SJ_LAUNCH_CHECK() ::sj::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// ---------------------------------------------------------------------
// Device memory: a caching pool keyed by rounded size. Blocks are handed
// back only after the owning call has synchronised its stream.
// ---------------------------------------------------------------------
void *dev_alloc(size_t bytes);
void dev_free(void *p);

// Page-locked host blocks of kStageBytes for small device-to-host readbacks
// (a copy into pageable memory goes through the runtime's own staging and
// returns later). Pooled for the life of the process.
constexpr size_t kStageBytes = 4096;
void *stage_acquire();
void stage_release(void *p);
// One staging block for the scope. If the scope ends by an exception, a copy
// into the block may still be in flight: the block is then not reused.
struct HostStage {
    void *p;
    HostStage() : p(stage_acquire()) {}
    ~HostStage() {
        if (std::uncaught_exceptions() == 0) stage_release(p);
    }
    HostStage(const HostStage &) = delete;
    HostStage &operator=(const HostStage &) = delete;
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};
void pool_trim();
// Bytes of device memory held by the pool: cached (free for reuse) and live.
void pool_info(uint64_t *cached, uint64_t *live);
void pool_enter();
void pool_leave_after_sync();

template <typename T>
struct DevBuf {
    T *ptr = nullptr;
    size_t count = 0;
    DevBuf() = default;
    explicit DevBuf(size_t n) { reset(n); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), count(o.count) { o.ptr = nullptr; o.count = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); ptr = o.ptr; count = o.count; o.ptr = nullptr; o.count = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void reset(size_t n) {
        release();
        count = n;
        ptr = n ? static_cast<T *>(dev_alloc(n * sizeof(T))) : nullptr;
    }
    // grow-only reuse
    void ensure(size_t n) { if (n > count) reset(n); }
    void release() { if (ptr) dev_free(ptr); ptr = nullptr; count = 0; }
    size_t bytes() const { return count * sizeof(T); }
};

// ---------------------------------------------------------------------
// Per-kernel timing with HIP events, on the stream each kernel is launched
// on. Off unless enabled through the ABI; the events of a call are resolved
// after the call has synchronised its stream.
// ---------------------------------------------------------------------
bool profiling_enabled();
struct KTimer {
    KTimer(const char *name, hipStream_t s);
    ~KTimer();
    const char *name_;
    hipStream_t s_;
    hipEvent_t e0_ = nullptr, e1_ = nullptr;
};
void profile_resolve_pending();
void profile_reset();
void profile_set(bool on);
void profile_select(const char *prefix);
int profile_read(void *out, uint32_t cap, uint32_t *count);

// ---------------------------------------------------------------------
// Primitives (k_scan.hip, k_sort.hip)
// ---------------------------------------------------------------------
// out[i] = sum_{k<i} in[k] for i in [0, n]; out[n] is the total.
void scan_exclusive_u32_to_u64(const uint32_t *in, uint64_t *out, size_t n, hipStream_t s);
// Two such scans of equal length in one pair of launches.
void scan_exclusive_u32_to_u64_x2(const uint32_t *in0, uint64_t *out0, const uint32_t *in1,
                                  uint64_t *out1, size_t n, hipStream_t s);
// The same with the tile sums in a caller buffer of scan_partials(n) u64
// (allocates nothing).
size_t scan_partials(size_t n);
void scan_exclusive_u32_to_u64_ws(const uint32_t *in, uint64_t *out, size_t n, uint64_t *part, hipStream_t s);
// in place inclusive scan of u32.
void scan_inclusive_u32(uint32_t *data, size_t n, hipStream_t s);
// exclusive scan of u32 into u32 (no total), in place allowed.
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, size_t n, hipStream_t s);
// Exclusive scan of the grid-row head flags of the cells (coordinates
// cell-major, d per cell): row_of[h] = rows starting before cell h,
// row_of[ncells] = number of rows.
void scan_row_heads_exclusive(const uint32_t *coords, uint32_t d, uint64_t *row_of, size_t ncells,
                              hipStream_t s);
// ch_off[r] = chunks of the grid rows before r (ceil(points / 64) each, from
// the rows' first points row_pt), ch_off[ncells] = all chunks.
void scan_row_chunks_exclusive(const uint32_t *row_pt, const uint64_t *row_of, uint64_t *ch_off, size_t ncells,
                               hipStream_t s);
// pos[r] = rows before r longer than lo entries (lengths off[r+1] - off[r]),
// pos[rows] = their number.
void scan_long_rows_exclusive(const uint64_t *off, uint32_t lo, uint32_t *pos, size_t rows, hipStream_t s);
// Inclusive scan of the head flags (key[r] >> shift != key[r-1] >> shift, 1
// at r = 0) of a sorted key array: out[r] = 1 + number of distinct shifted
// keys before r.
template <typename K>
void scan_head_flags_inclusive(const K *sorted_keys, int shift, uint32_t *out, size_t n, hipStream_t s);

// Stable LSD radix sort of (key, value) by the low `bits` bits of key.
// The passes alternate between the two buffer pairs: returns false when the
// sorted data ends in keys/vals, true when it ends in keys_alt/vals_alt.
bool radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                    size_t n, int bits, hipStream_t s);
bool radix_sort_u32(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                    size_t n, int bits, hipStream_t s);

// ---------------------------------------------------------------------
// Index kernels (k_index.hip)
// ---------------------------------------------------------------------
// bbox_out[0..d) = min, [8..8+d) = max; *bad = nonzero if a NaN/Inf was seen.
void launch_bbox(const double *pts, uint64_t n, uint32_t d, double *bbox_out, uint32_t *bad,
                 hipStream_t s);
void launch_cell_keys_u64(const double *pts, uint64_t n, const GridParams &g, uint64_t *keys,
                          uint32_t *ids, hipStream_t s);
void launch_cell_keys_u32(const double *pts, uint64_t n, const GridParams &g, uint32_t *keys,
                          uint32_t *ids, hipStream_t s);
// Sort keys: the cell id, or with g.sub_shift > 0 the cell id shifted left by
// it and the dimension-0 sub-cell appended (ids[i] = i).
// head flags + inclusive scan + cell tables over sorted keys; keys equal
// after a right shift by `shift` are one cell. cell_of receives the cell of
// each cell-ordered point, B the distinct shifted keys, starts the first
// point of each cell (starts[|G|] is written as n); |G| = cell_of[n - 1] + 1
// (left on the device: no host sync).
template <typename K>
void build_cells(const K *sorted_keys, uint64_t n, int shift, uint32_t *cell_of, uint64_t *B, uint32_t *starts,
                 hipStream_t s);
// Word offset of each dimension's occupancy mask.
struct MaskOffsets {
    uint32_t off[kMaxDim];
};
// per-cell coordinates (cell-major, d per cell), occupancy masks, and the
// largest cell (written to *max_pts on the device). The cell count is read
// on the device (*last_cell + 1, the cell of the last sorted point);
// ncells_bound (>= it) sizes the launch.
void launch_cell_coords_masks(const uint64_t *B, const uint32_t *starts, uint64_t ncells_bound,
                              const uint32_t *last_cell, const GridParams &g, uint32_t *coords, uint32_t *masks,
                              const MaskOffsets &mask_off, uint32_t mask_words, uint32_t *max_pts,
                              hipStream_t s);
// Cell-ordered copy X[j][r] = pts[perm[r]][j] and the dimension-0 cell
// coordinate of every cell-ordered point, cx[r] (the cell-key formula).
void launch_gather_soa(const double *pts, const uint32_t *perm, uint64_t n, uint32_t d, double *X,
                       const GridParams &g, uint32_t *cx, hipStream_t s);
void launch_make_f32(const double *X, uint64_t n, uint32_t d, const double *shift, float *Y,
                     hipStream_t s);
void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
// Up to four ranges of 32-bit words to clear in one launch.
struct ZeroSpans {
    uint32_t *p[4];
    uint64_t words[4];
    int count;
    void add(void *ptr, uint64_t nwords) {
        if (!ptr || !nwords) return;
        p[count] = static_cast<uint32_t *>(ptr);
        words[count] = nwords;
        ++count;
    }
};
void launch_zero_spans(const ZeroSpans &z, hipStream_t s);
void launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);

// ---------------------------------------------------------------------
// Search and join (k_join.hip)
// ---------------------------------------------------------------------
// Candidate point ranges of every cell: counts, scan, fill. Returns the
// number of ranges R (host sync); roff gets |G|+1 entries, rng 2R values.
uint64_t build_ranges(const SearchArgs &a, int unicomp, uint64_t *roff /*[ncells+1]*/,
                      uint32_t **rng_out, size_t *rng_cap, hipStream_t s);

void launch_join(const JoinArgs &a, uint32_t d, int unicomp, int mode, int band, hipStream_t s);

// Grid-row tiled join (k_tile.hip).
// Builds the chunk list without a host sync: a grid row holds p points
// in ceil(p / 64) <= p / 64 + 1 chunks, so there are at most
// floor(n / 64) + rows chunks, rows <= min(ncells, rows_bound). Returns that
// bound; the exact count goes to *nchunks_dev.
uint32_t build_chunks(const uint32_t *coords, const uint32_t *starts, uint32_t ncells, uint32_t n, uint32_t d,
                      uint64_t rows_bound, uint2 **chunks_out, size_t *chunks_cap, uint32_t *nchunks_dev,
                      hipStream_t s);
void build_chunk_segments(const TileArgs &t, const uint32_t *cell_of, const uint32_t *starts,
                          uint32_t d, uint2 *segs, hipStream_t s);
// Word rows of hit bits per chunk (k_tile.hip): cwords[0, nslots) with
// cwords[nslots - 1] = 0; *big set (atomic or) if a chunk overflows 32 bits.
void launch_chunk_words(const TileArgs &t, const uint32_t *cell_of, uint32_t d, int unicomp, uint32_t nslots,
                        uint32_t *cwords, uint32_t *big, hipStream_t s);
void launch_join_tiled(const JoinArgs &a, const TileArgs &t, uint32_t d, int unicomp, int mode,
                       int band, hipStream_t s, uint32_t fused_sort = 0);

// Row lengths in original order and in cell order; row_stats
// (4 x kRowStatWords/4 words, no clearing needed) gets per-workgroup longest
// rows and numbers of rows longer than 16, 24 and 32.
constexpr size_t kRowStatWords = 4 * 512;
void launch_row_lengths(const uint32_t *own_cnt, const uint32_t *in_cnt, const uint32_t *perm,
                        uint64_t n, uint32_t *len_orig, uint32_t *len_cell, uint32_t *row_stats,
                        hipStream_t s);
// Gathers the count pass results into out[0..8): P, longest row,
// evaluations, band re-checks, chunk count (nchunks may be null), rows
// longer than 16, 24, 32 (max_len = the row_stats of launch_row_lengths);
// also clears the fill's overflow flag (may be null).
void launch_count_summary(const uint64_t *off_orig, uint64_t n, const uint32_t *max_len,
                          const unsigned long long *counters, const uint32_t *nchunks, uint64_t *out,
                          uint32_t *overflow, hipStream_t s);
void launch_gather_offsets(const uint64_t *off_orig, const uint32_t *perm, uint64_t n,
                           uint64_t *offc, hipStream_t s);
// cell-ordered points whose original id lies in [i0, i1), in cell order.
// Returns the count (host sync).
uint32_t build_query_list(const uint32_t *perm, uint64_t n, uint64_t i0, uint64_t i1,
                          uint32_t *flags_scratch, uint32_t *qlist, hipStream_t s);
// Cell-ordered batch plan: batch b starts at work unit unit[b] (a chunk, or
// a point when chunks is null), point pos[b], cell-order row offset off[b];
// entry nb holds (units, n, total).
void launch_batch_units(const uint2 *chunks, const uint64_t *off_cell, uint64_t n, uint32_t units,
                        uint64_t total, uint32_t nb, uint32_t *unit, uint64_t *pos, uint64_t *off, hipStream_t s);
// len_b[perm[r]] = len_cell[r] for r in [r0, r1).
void launch_batch_lengths(const uint32_t *len_cell, const uint32_t *perm, uint64_t r0, uint64_t r1,
                          uint32_t *len_b, hipStream_t s);
// rows[b] = first row i with off[i] >= floor(b * total / nb), b in [0, nb];
// rows[nb] = n.
void launch_batch_bounds(const uint64_t *off, uint64_t n, uint64_t total, uint32_t nb,
                         uint64_t *rows, hipStream_t s);

// Two-set join (k_rs.hip): mode 0 counts each query row's neighbours into
// a.count, mode 1 writes them (S rows, unsorted) into a.out_j at a.off.
void launch_join_rs(const RsArgs &a, int mode, hipStream_t s);
// Tiled two-set join: keys[i] = cell id of query row i in g (clamped by one
// cell at the grid's edge), 2^key_bits for a row with no adjacent cell;
// ids[i] = i; *nleft (0 on entry) += rows of the second kind.
void launch_rs_query_keys_u32(const double *R, uint64_t nr, const GridParams &g, int key_bits, uint32_t *keys,
                              uint32_t *ids, uint32_t *nleft, hipStream_t s);
void launch_rs_query_keys_u64(const double *R, uint64_t nr, const GridParams &g, int key_bits, uint64_t *keys,
                              uint32_t *ids, uint32_t *nleft, hipStream_t s);
// *out (0 on entry) = max of counts[0..n).
void launch_rs_max(const uint32_t *counts, uint64_t n, uint32_t *out, hipStream_t s);

// All-pairs join (k_brute.hip): mode kCount writes a.count, kFill a.pairs.
void launch_brute(const BruteArgs &a, uint32_t d, int mode, hipStream_t s);
uint32_t brute_rows_per_block(uint32_t d);  // query rows per workgroup
uint32_t brute_tile();                      // candidates per LDS tile

// DBSCAN over a CSR neighbour table (k_dbscan.hip): label[i] = smallest core
// index of i's cluster, -1 for noise; *nclusters (0 on entry) += clusters.
void launch_dbscan(const uint64_t *off, const uint32_t *cols, uint64_t n, uint32_t min_pts, int32_t *label,
                   unsigned long long *nclusters, hipStream_t s);

// ---------------------------------------------------------------------
// Row sort and pair expansion (k_rowsort.hip)
// ---------------------------------------------------------------------
// Sorts each row's neighbour ids and writes interleaved (i, j) pairs -- or,
// with cols set, only the j of each entry (compressed sparse row columns);
// with sorted false the rows are moved unsorted.
// Rows [i0, i1); row i occupies [off[i] - base, off[i+1] - base) of out_j
// and of the output. max_len is the longest row.
void launch_rowsort(const uint64_t *off, uint64_t i0, uint64_t i1, uint64_t base,
                    uint32_t *out_j, uint32_t *pairs, uint32_t max_len, hipStream_t s,
                    uint32_t *cols = nullptr, bool sorted = true);
// Whole result filled in cell order: row r (cell-ordered point r) occupies
// out_j[off_cell[r], off_cell[r+1]) and goes to output [off_orig[perm[r]], ...)
// with i = perm[r].
void launch_rowsort_cells(const uint64_t *off_cell, const uint64_t *off_orig, const uint32_t *perm,
                          uint64_t n, uint32_t *out_j, uint32_t *pairs, uint32_t max_len, hipStream_t s,
                          uint32_t *cols = nullptr, bool sorted = true);
// Rows of the cell-ordered points [r0, r1): row r occupies
// out_j[off_cell[r] - in_base, +len) and goes to off_out[perm[r]]; only the
// rows longer than sorted_len (0: all rows).
void launch_rowsort_range(const uint64_t *off_cell, uint64_t r0, uint64_t r1, uint64_t in_base,
                          const uint64_t *off_out, const uint32_t *perm, uint32_t *out_j, uint32_t *pairs,
                          uint32_t max_len, uint32_t sorted_len, hipStream_t s, uint32_t *cols = nullptr,
                          bool sorted = true);
// Same layout; handles only the rows longer than sorted_len (a fused fill
// has written the others).
void launch_rowsort_long(const uint64_t *off_cell, const uint64_t *off_orig, const uint32_t *perm,
                         uint64_t n, uint32_t *out_j, uint32_t *pairs, uint32_t max_len, uint32_t sorted_len,
                         hipStream_t s, uint32_t *cols = nullptr, bool sorted = true);

}  // namespace sj
