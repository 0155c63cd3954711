// Argument blocks passed by value to the join kernels, and the constants
// their layout depends on. Kept apart from the host-side declarations so
// that a kernel's definition is its own source file, sj_device.h and this
// header.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sj {

constexpr int kMaxDim = 8;

// From this many dimensions on, the grid-row kernel's count pass records hit
// bits for the fill pass (below it the fill is bound by its writes, not by
// its tests, and recording costs more than it saves).
constexpr uint32_t kHitBitsMinDim = 5;

// ---------------------------------------------------------------------
// Grid description (Section IV-B), passed by value to kernels.
// ---------------------------------------------------------------------
struct GridParams {
    double gmin[kMaxDim];
    double w;
    uint64_t dims[kMaxDim];
    uint64_t stride[kMaxDim];
    uint32_t d;
    // Within a cell, points are ordered by their dimension-0 sub-cell of
    // width w / 2^sub_shift (then by id): the tiled join narrows each
    // point's dimension-0 window to the sub-cells within w of its own.
    uint32_t sub_shift;
};

struct SearchArgs {
    const uint64_t *B;
    const uint32_t *starts;
    const uint32_t *coords;
    const uint32_t *masks;
    uint32_t mask_off[kMaxDim];
    uint64_t dims[kMaxDim];
    uint64_t stride[kMaxDim];
    uint32_t ncells;
    uint32_t d;
};

struct JoinArgs {
    const double *X;          // d x n, cell order (the candidates)
    const float *Y;           // d x n, cell order, shifted (band path) or null
    uint32_t n;
    // query points of the tiled kernel, d x nqs in cell order (for the
    // self-join the candidates themselves; for R x S the queries of R in
    // S's grid): coordinates, their FP32 copy, and each one's row id
    const double *Xq;
    const float *Yq;
    uint32_t nqs;
    const uint32_t *permq;
    const uint32_t *cell_of;
    const uint32_t *starts;
    const uint64_t *roff;
    const uint2 *rng;
    const uint32_t *qlist;    // query points (cell order) or null for qbase + [0, nq)
    uint32_t nq;
    uint32_t qbase;           // first query position when qlist is null
    double eps2;
    float lo, hi;
    // fused-square filter band around eps2: a fused multiply-add sum below
    // flo is a pair, above fhi (or NaN) is not, else the exact sum decides
    double flo, fhi;
    // count outputs
    uint32_t *own_cnt;
    uint32_t *in_cnt;
    // fill
    const uint64_t *offc;     // row offset of each cell-ordered point's row
    uint64_t out_base;
    uint64_t out_cap;         // entries of out_j; writes at or past it set *overflow
    uint32_t *overflow;
    uint32_t *cur;
    uint32_t *out_j;
    const uint32_t *perm;     // A
    // counters
    unsigned long long *evals;
    unsigned long long *band_rechecks;
    // fill with the row sort fused in (each point's row is complete when its
    // own evaluation ends): rows of at most the kernel's register-sort size
    // are sorted and written as (i, j) pairs at off_orig[perm[p]]; longer
    // rows stay in out_j for the row-sort kernels
    const uint64_t *off_orig;
    uint2 *pairs;
};
// kReplay: the fill pass of a search whose count recorded hit bits (it
// stages no coordinates and tests nothing; grid-row kernel, FP64, from
// kHitBitsMinDim dimensions on)
enum JoinMode { kCount = 0, kFill = 1, kReplay = 2 };

// Grid-row tiled join (k_tile.hip): chunks of <= 64 cell-ordered points of
// one grid row, candidate rows staged in LDS.
struct TileArgs {
    const uint64_t *B;
    uint32_t ncells;
    const uint32_t *coords;
    const uint32_t *masks;
    uint32_t mask_off[kMaxDim];
    uint64_t dims[kMaxDim];
    uint64_t stride[kMaxDim];
    const uint32_t *cx;       // dimension-0 sub-cell coordinate of each cell-ordered point
    const uint32_t *cxq;      // the same for the query points (cx for the self-join)
    uint32_t sub_shift;       // sub-cells per cell in dimension 0: 2^sub_shift
    const uint2 *chunks;      // [first, end) point range of each chunk
    uint32_t nchunks;         // upper bound on the chunk count (launch size)
    const uint32_t *nchunks_dev;  // the chunk count (device)
    uint32_t chunk0;          // first chunk of the launch (a batch's range; 0 for all)
    uint32_t chunk_end;       // end of the launch's chunk range (~0u: up to the count)
    uint32_t rows_per_chunk;  // 3^(d-1)
    const uint2 *segs;        // [chunk * rows_per_chunk + row] candidate point segment
    // hit bits (null: off): the count pass records every tested candidate's
    // outcome, the fill pass of the same search reads them instead of
    // testing again. A run of s candidates of one lane takes ceil(s / 32)
    // words, one word row of 64 lanes each ([word row][lane], candidate k
    // of the run at bit 31 - k % 32 of word k / 32); a chunk's word rows
    // start at cbase[chunk].
    uint32_t *bits;
    const uint64_t *cbase;
};

// Distance join of a query set R with an indexed set S (k_rs.hip).
struct RsArgs {
    const double *R;          // nr x d, row-major
    uint64_t nr;
    const uint32_t *qperm;    // query rows in S's cell order (thread k takes row qperm[k])
    const double *X;          // S: d x ns, cell order
    uint64_t ns;
    const uint32_t *perm;     // S's A (cell-ordered position -> row of S)
    const uint64_t *B;        // S's non-empty cell ids, ascending
    const uint32_t *starts;   // S's cell starts (ncells + 1)
    uint32_t ncells;
    GridParams g;             // S's grid
    double eps2;
    uint32_t *count;          // count pass: neighbours of each query row (by row)
    uint32_t *count_k;        // count pass: the same counts in probe order (by k)
    const uint64_t *off;      // fill pass: offsets in probe order (nr + 1)
    uint32_t *out_j;          // fill pass: S rows, the k-th probed query at off[k]
    uint64_t out_cap;
    uint32_t *overflow;       // set when a fill write falls outside its row
};

// All-pairs join (k_brute.hip): every query row against every point, the
// candidates split into `splits` consecutive ranges of `span` points so that
// small inputs still fill the chip.
struct BruteArgs {
    const double *pts;        // n x d, row-major (the caller's layout)
    uint64_t n;
    uint32_t splits;          // candidate ranges per query row
    uint64_t span;            // points per range (a multiple of the tile)
    double eps2;
    uint32_t *count;          // count pass: hits of row i in range s at [i * splits + s]
    const uint64_t *off;      // fill pass: exclusive scan of count (n * splits + 1 entries)
    uint2 *pairs;             // fill pass: (i, j) pairs, row i range s at off[i * splits + s]
    uint32_t *overflow;       // set if a fill write would leave its range
};

}  // namespace sj
