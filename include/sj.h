/*
 * sj.h -- C ABI of the MI355X (gfx950) epsilon-distance similarity self-join.
 *
 * Given n points in d dimensions (2 <= d <= 6 is the tuned range, 1 <= d <= 8
 * is accepted) and a distance eps, the library returns every ordered pair
 * (i, j) of point ids with squared Euclidean distance <= eps * eps, sorted by
 * (i, j). This is the self-join of Section III; the method is the grid
 * index of Section IV (non-empty cells only, bounded search of the 3^d
 * adjacent cells), the duplicate-search removal "unicomp" of Section V-B
 * (Algorithm 2) and result batching of Section V-A.
 *
 * Pair membership is exact with respect to this definition, evaluated in
 * IEEE binary64 with dimension order 0..d-1 and no fused multiply-add:
 *     d2(i,j) = (...((x_i0-x_j0)^2 + (x_i1-x_j1)^2) + ...),  pair iff d2 <= fl(eps*eps).
 * The FP32 option pre-tests in single precision and re-decides every pair in
 * a proven error band around eps^2 with the FP64 formula, so the pair set is
 * the same.
 *
 * Conventions for every entry point:
 *  - Return value 0 (SJ_OK) on success or a negative SJ_E* code; the
 *    thread-local message of the last failure is given by sj_last_error().
 *    No C++ exception crosses this boundary.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). All
 *    device work of a call is queued on it; calls return after the work they
 *    queued has finished unless stated otherwise.
 *  - Point arrays are row-major n x d binary64 (point i at pts[i*d .. i*d+d-1]),
 *    owned by the caller and not retained after the call returns.
 *  - Pair arrays are interleaved uint32 (i0, j0, i1, j1, ...), 8 bytes per pair.
 *  - Ids are 0-based row indices of the input; n must be below 2^32 - 1.
 *  - Not thread-safe on one index: calls on the same sj_index must not overlap.
 *    Distinct indexes may be used from different threads and streams.
 */
#ifndef SJ_H
#define SJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------- */
#define SJ_OK         0
#define SJ_EINVAL    -1   /* bad argument: d outside [1,8], eps <= 0 or not finite,
                             NaN/Inf coordinate, NULL pointer, n too large */
#define SJ_ENOMEM    -2   /* device or pinned-host allocation failed */
#define SJ_EGRID     -3   /* the grid cannot be represented even after widening cells */
#define SJ_EDEVICE   -4   /* a HIP runtime call failed */
#define SJ_ESTATE    -5   /* call out of order (e.g. sj_join_fill before sj_join_count) */
#define SJ_ECAPACITY -6   /* output buffer or batch capacity too small */

/* ---- options ---------------------------------------------------------- */
#define SJ_FP64      0    /* distances in binary64 */
#define SJ_FP32_BAND 1    /* binary32 pre-test, binary64 re-decision inside the band; on the grid-row
                             kernel up to 5-D only: from 6-D on the binary64 path is faster and runs
                             instead (same pairs; sj_stats.precision_used says which ran) */

typedef struct sj_join_opts {
    int32_t  unicomp;              /* 1: evaluate each unordered pair of adjacent
                                      cells once (Section V-B); 0: all 3^d cells */
    int32_t  precision;            /* SJ_FP64 or SJ_FP32_BAND */
    uint64_t batch_capacity_pairs; /* max pairs per delivered batch; 0 = no limit */
    uint32_t min_batches;          /* at least this many batches (Section V-A uses 3) */
    int32_t  sort_output;          /* 1: every row's j ascending, so the pairs are sorted
                                      by (i, j) (the key/value sort of Section IV-E);
                                      0: rows still in ascending i with the row offsets
                                      of the sorted form, but the j of a row in an
                                      unspecified order (the separate row-sort kernels
                                      are replaced by a plain row move) */
} sj_join_opts;

/* Fills *o with unicomp=1, precision=SJ_FP64, no capacity limit, 1 batch,
 * sort_output=1. */
void sj_default_opts(sj_join_opts *o);

/* ---- statistics --------------------------------------------------------- */
typedef struct sj_stats {
    uint64_t n;                 /* points */
    uint32_t d;                 /* dimensions */
    uint32_t key_bits;          /* bits of the linearised cell id */
    uint64_t cells;             /* |G| = |B|, non-empty cells (Section IV-C) */
    uint64_t grid_dims[8];      /* |g_j| per dimension */
    double   eps;
    double   cell_width;        /* w >= eps (slightly wider, see the header of the index code) */
    uint32_t max_cell_points;   /* largest |C_h| */
    uint32_t precision_used;    /* SJ_FP64 or SJ_FP32_BAND actually used in the last join */
    uint64_t ranges;            /* candidate point ranges of the last join's cell search */
    uint64_t evals;             /* distance evaluations of the last count pass */
    uint64_t band_rechecks;     /* candidates of the last count pass re-decided by the exact FP64 sum: from the
                                   FP32 band, or (grid-row kernel, 4-D and up) from the FP64 fused-square band */
    uint64_t pairs;             /* pairs of the last join */
    uint64_t max_row_pairs;     /* longest result row of the last join */
    uint32_t batches;           /* batches of the last join */
    uint32_t unicomp_used;
    double   ms_build;          /* wall time of sj_build_index */
    double   ms_count;          /* wall time of the last sj_join_count */
    double   ms_fill;           /* wall time of the last fill / batch loop */
    uint64_t chunks;            /* wave work units of the grid-row tiled join (0 if unused) */
    uint32_t fill_unicomp;      /* 1 if the last fill evaluated the unicomp subset */
    uint32_t reserved0;
    uint64_t hit_bit_bytes;     /* device bytes of the hit bits the last count pass recorded for its fill
                                   (grid-row kernel, FP64, 5-D and up; 0 when none were recorded) */
} sj_stats;

/* ---- the index (Section IV-C: B, G, A, M plus the cell-ordered points) -- */
typedef struct sj_index sj_index;

/*
 * Builds the grid index of Section IV-B/IV-C on the GPU: bounding box,
 * cell ids, sort of points by cell (A), non-empty cell ids (B) with their
 * point ranges (G), per-dimension occupancy masks (M) and a cell-ordered
 * structure-of-arrays copy of the coordinates.
 *   pts           n x d row-major binary64; device pointer if pts_on_device,
 *                 else host memory (copied to the device).
 *   eps           join distance, finite and > 0.
 *   out           receives the index; release it with sj_destroy_index.
 * n == 0 is valid (an empty index; every join returns 0 pairs).
 */
int sj_build_index(const double *pts, uint64_t n, uint32_t d, double eps,
                   int pts_on_device, void *stream, sj_index **out);

/* Releases the index of Section IV-C (B, G, A, M and the cell-ordered
 * points) and all its device memory. NULL is ignored. The caller must not
 * use the index afterwards, and no call on it may still be running. */
void sj_destroy_index(sj_index *idx);

/*
 * Count pass of the join (Algorithm 1's search and refine, Section V-B's
 * unicomp when opts->unicomp): computes every result row's length and the
 * row offsets, and returns the number of pairs P in *total_pairs. It must
 * precede sj_join_fill on the same index; opts is remembered for the fill.
 * From 5-D on (binary64, grid-row kernel) it also records every tested
 * candidate's outcome for the fill ("hit bits", sj_stats.hit_bit_bytes), in
 * device memory the index holds until a whole-result fill has read them, the
 * next count, or sj_destroy_index; it takes them only when they fit in 40% of
 * the device memory that is free or cached by the library's pool
 * (SJ_HIT_BITS=0 in the environment: never).
 */
int sj_join_count(sj_index *idx, const sj_join_opts *opts, void *stream,
                  uint64_t *total_pairs);

/*
 * Fill pass: writes all P pairs, sorted by (i, j), to the device buffer
 * `pairs_dev` (2 * P uint32, owned by the caller). capacity_pairs must be at
 * least P (else SJ_ECAPACITY and nothing is written).
 */
int sj_join_fill(sj_index *idx, uint32_t *pairs_dev, uint64_t capacity_pairs,
                 void *stream);

/*
 * Fill pass into a compressed sparse row (CSR) neighbour table instead of
 * pairs: row_off_dev receives n + 1 uint64 row offsets (row i holds
 * cols_dev[row_off[i] .. row_off[i+1]), row_off[n] = P) and cols_dev the P
 * neighbour ids j, 4 bytes per entry instead of the 8 of an (i, j) pair --
 * the neighbour table that the DBSCAN use of the self-join consumes
 * (Section I; the batching of Section V-A comes from that use). Rows hold
 * the same j as the pair form: ascending if the count pass's
 * opts->sort_output was 1, else in an unspecified order. Both buffers are
 * device memory owned by the caller; capacity is the entries cols_dev holds
 * (SJ_ECAPACITY if below P, nothing written). Needs a preceding
 * sj_join_count, like sj_join_fill.
 */
int sj_join_fill_csr(sj_index *idx, uint64_t *row_off_dev, uint32_t *cols_dev, uint64_t capacity,
                     void *stream);

/*
 * DBSCAN (Ester et al.; the clustering Section I names as a user of the
 * self-join) over a CSR neighbour table as sj_join_fill_csr writes it: row i
 * lists every point within eps of point i, i itself included, so i is a
 * core point when its row holds at least min_pts entries. labels_dev (n
 * int32, device, caller-owned) receives for a core point the smallest index
 * of the core points of its cluster (clusters are the connected components
 * of core points joined by table entries), for a border point (not core,
 * with a core point in its row) the label of the smallest-index core point
 * in its row, and -1 for noise. *nclusters receives the number of clusters.
 * The order of j within a row does not matter. n < 2^31, min_pts >= 1.
 */
int sj_dbscan_csr(const uint64_t *row_off_dev, const uint32_t *cols_dev, uint64_t n, uint32_t min_pts,
                  int32_t *labels_dev, void *stream, uint64_t *nclusters);

/*
 * DBSCAN of n points in one call: the grid index and count pass (unicomp),
 * the CSR fill with unsorted rows into library scratch (4 bytes per pair),
 * then sj_dbscan_csr's labelling into labels_dev. Arguments as for
 * sj_build_index and sj_dbscan_csr.
 */
int sj_dbscan(const double *pts, uint64_t n, uint32_t d, double eps, uint32_t min_pts, int pts_on_device,
              int32_t *labels_dev, void *stream, uint64_t *nclusters);

/*
 * Distance join of a query set R with the indexed set S (Section II: the
 * self-join is the case R = S; the pair test is Section III's, as for the
 * self-join). R is nr x d row-major FP64 with the index's d, in device
 * memory if r_on_device else host memory, owned by the caller and not
 * retained. Result: every (i, j) with i a row of R and j a row of S within
 * eps (the index's), as interleaved uint32 pairs sorted by (i, j).
 * *total_pairs receives P. If pairs_dev is NULL only P is computed;
 * otherwise capacity_pairs must be at least P (else SJ_ECAPACITY, with
 * *total_pairs set and nothing written). Queries outside S's bounding box
 * are allowed (they probe only the cells that exist); a query with a NaN or
 * infinite coordinate has no neighbours. The queries are sorted into S's
 * grid and joined by the self-join's grid-row tiled kernel (full search);
 * SJ_JOIN_KERNEL=ranges in the environment selects a one-query-per-thread
 * kernel instead (same result). Independent of the self-join state of the
 * index (count/fill).
 */
int sj_join_rs(sj_index *idx, const double *R, uint64_t nr, int r_on_device, uint32_t *pairs_dev,
               uint64_t capacity_pairs, void *stream, uint64_t *total_pairs);

/*
 * The same two-set join in two calls, for callers that size the output
 * from P: sj_join_rs_count runs the query sort and the count pass and
 * returns P; sj_join_rs_fill then writes the pairs (capacity_pairs >= P, else
 * SJ_ECAPACITY and nothing written) without repeating either. Between the
 * two calls device queries must stay valid and unchanged (host queries are
 * copied to the device by the count call). A later count replaces the
 * state; the self-join's count/fill state is separate.
 */
int sj_join_rs_count(sj_index *idx, const double *R, uint64_t nr, int r_on_device, void *stream,
                     uint64_t *total_pairs);
int sj_join_rs_fill(sj_index *idx, uint32_t *pairs_dev, uint64_t capacity_pairs, void *stream);

/*
 * Batched join (Section V-A): the result is delivered in at least
 * opts->min_batches runs of at most opts->batch_capacity_pairs pairs each,
 * sized from the exact row lengths of the count pass. Run b holds every
 * result row of the points at positions [row_begin, row_end) of the index's
 * cell order (SJ_EXPORT_PERM maps a position to its point id), sorted by
 * (i, j) within the run; the runs partition the result, and merging them
 * gives the sorted result. A run is passed to cb(user, pairs_dev, npairs,
 * batch_id, row_begin, row_end) as a device buffer that stays valid until
 * cb returns; while cb runs, the next run is already being computed. A
 * non-zero return from cb stops the join and is returned. The library owns
 * the buffers. SJ_ECAPACITY if one result row alone exceeds the capacity.
 * Runs are whole grid-row chunks of the tiled join when the capacity holds
 * 128 times the longest row, else ranges of single points.
 */
typedef int (*sj_run_cb)(void *user, const uint32_t *pairs_dev, uint64_t npairs,
                         uint32_t batch_id, uint64_t row_begin, uint64_t row_end);

int sj_selfjoin_index(sj_index *idx, const sj_join_opts *opts, sj_run_cb cb,
                      void *user, void *stream, uint64_t *total_pairs);

/*
 * Convenience: the whole self-join of Section III in one call -- the index
 * of Section IV-B/IV-C, the count and fill passes of Algorithm 1 (unicomp of
 * Section V-B per opts) -- returning all pairs sorted by (i, j) in a buffer
 * allocated by the library: device memory if out_on_device, else pinned
 * host memory filled batch by batch while later batches compute (the
 * result transfer overlapped with computation, Section V-A). Release it
 * with sj_free. *pairs_out is NULL when *npairs is 0.
 *   pts, n, d, eps   as for sj_build_index (pts_on_device selects device or
 *                    host memory); opts as for sj_join_count (NULL:
 *                    sj_default_opts).
 * Statistics of the run: sj_last_run_stats on the same thread.
 */
int sj_selfjoin(const double *pts, uint64_t n, uint32_t d, double eps,
                const sj_join_opts *opts, int pts_on_device, int out_on_device,
                void *stream, uint32_t **pairs_out, uint64_t *npairs);

/*
 * sj_bruteforce for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same all-pairs join and the same result, with every temporary in a fixed
 * device array that the library holds on each GPU it runs on until the
 * process ends (about 24 MiB), so the call makes no hipMalloc, hipFree or
 * other allocating call. pts_dev must be device memory (no host staging).
 * At most 2^21 points (SJ_EINVAL beyond, before any device work); other
 * arguments and errors as for sj_bruteforce. Calls that overlap on one GPU
 * share that array and race: serialise them.
 */
int sj_bruteforce_noalloc(const double *pts_dev, uint64_t n, uint32_t d, double eps, uint32_t *pairs_dev,
                          uint64_t capacity_pairs, void *stream, uint64_t *total_pairs);

/* Frees a result buffer that sj_selfjoin allocated (device or pinned host
 * memory, the two placements of a Section V-A result). NULL and pointers the
 * library did not hand out are ignored. */
void sj_free(void *ptr);

/*
 * Statistics of the index (|G| of Section IV-C, the grid |g_j| of Section
 * IV-B, the largest cell) and of the last join run on it (evaluations, band
 * re-decisions, pairs, batches, times). Host-side state only: no device
 * work, and it may be called while no call on the index runs.
 */
int sj_index_stats(const sj_index *idx, sj_stats *out);

/*
 * Statistics of the last join run on the calling thread, whatever produced
 * it: a count or fill pass, the batched join (Section V-A), the convenience
 * sj_selfjoin (whose index is gone when it returns), the two-set join (n is
 * then the number of query rows, the grid fields are S's, and evals is
 * counted by the tiled kernel only) or the brute force (whose evals is n^2).
 * Fields a run does not produce are 0.
 * SJ_ESTATE if no join has run on this thread.
 */
int sj_last_run_stats(sj_stats *out);

/*
 * All-pairs join, the GPU brute-force comparison of Section VI-B: every
 * point is compared with every point (n^2 evaluations of the Section III
 * pair test, with no index), giving the same result as the grid join: every
 * ordered pair (i, j) with d2 <= fl(eps * eps), sorted by (i, j).
 *   pts             n x d row-major binary64, device memory if pts_on_device,
 *                   else host memory (copied to the device); not retained.
 *   pairs_dev       device buffer for the pairs (2 * capacity_pairs uint32),
 *                   owned by the caller, or NULL to compute only P.
 *   *total_pairs    receives P (also when SJ_ECAPACITY is returned, in which
 *                   case nothing is written to pairs_dev).
 * Non-finite coordinates are not rejected: a point with a NaN or infinite
 * coordinate has a NaN or infinite distance to every point, itself included,
 * so it takes part in no pair. The cost is n^2 evaluations whatever eps is.
 */
int sj_bruteforce(const double *pts, uint64_t n, uint32_t d, double eps, int pts_on_device,
                  uint32_t *pairs_dev, uint64_t capacity_pairs, void *stream, uint64_t *total_pairs);

/*
 * Copies an internal array of the index to host memory (tests, debugging).
 * `bytes` must equal the array's size, which sj_index_export_size reports.
 *   SJ_EXPORT_CELL_IDS    uint64[|G|]   B: linear ids of non-empty cells, ascending
 *   SJ_EXPORT_CELL_START  uint32[|G|+1] G: cell h holds A[start[h] .. start[h+1]-1]
 *   SJ_EXPORT_PERM        uint32[n]     A: point ids in cell order (inside a cell by the
 *                                       dimension-0 sub-cell floor(t * s), t = (x_0 - g_0^min) / w,
 *                                       s from SJ_EXPORT_GRID, then by id)
 *   SJ_EXPORT_MASKS       uint32[sum_j ceil(|g_j|/32)]  M_j occupancy bitmaps, dimension 0 first
 *   SJ_EXPORT_RANGE_OFF   uint32[|G|+1] candidate ranges of cell h are rng[off[h] .. off[h+1]-1]
 *   SJ_EXPORT_RANGES      uint32[2*R]   (start, end) point ranges in cell order
 *   SJ_EXPORT_GRID        double[2*8+2] g_min[8], |g_j| as doubles [8], w, s (dimension-0
 *                                       sub-cells per cell, a power of two <= 8)
 *   SJ_EXPORT_ROW_OFFSETS uint64[n+1]   result row i holds pairs [off[i], off[i+1]) (after sj_join_count)
 * The two range arrays describe the last join (or the last sj_index_search).
 */
#define SJ_EXPORT_CELL_IDS   1
#define SJ_EXPORT_CELL_START 2
#define SJ_EXPORT_PERM       3
#define SJ_EXPORT_MASKS      4
#define SJ_EXPORT_RANGE_OFF  5
#define SJ_EXPORT_RANGES     6
#define SJ_EXPORT_GRID       7
#define SJ_EXPORT_ROW_OFFSETS 8
int sj_index_export_size(const sj_index *idx, int what, uint64_t *bytes);
int sj_index_export(const sj_index *idx, int what, void *host_dst, uint64_t bytes);

/* Runs only the adjacent-cell search (Section IV-D, or the unicomp subset)
 * so its ranges can be exported without a join. */
int sj_index_search(sj_index *idx, int unicomp, void *stream);

/*
 * The FP32 pre-test thresholds (lo, hi) used by SJ_FP32_BAND for dimension
 * d, distance eps and coordinate extent X = max |x - shift| over the data:
 * an FP32 squared distance S < lo is accepted, S > hi rejected, anything
 * else is re-decided in FP64. Returns SJ_EINVAL when the pre-test is not
 * usable (eps too small relative to X); the join then falls back to FP64.
 */
int sj_band_thresholds(uint32_t d, double eps, double extent, float *lo, float *hi);

/* ---- continuous-batching request server ------------------------------- */
/*
 * A server runs self-join requests as they arrive. `slots` worker threads,
 * each with its own HIP stream, take queued requests in arrival order when
 * the request's estimated device memory fits in what `mem_budget_bytes` has
 * left: the index bytes plus 12 bytes for each of expected_pairs and a
 * quarter more (a caller's expected mean is exceeded by about half the
 * requests), or the index bytes alone when expected_pairs is 0. The first
 * request is admitted whenever nothing else holds memory. After the count
 * pass the exact result size replaces the estimate (waiting for memory if
 * it grew). Requests on
 * different slots overlap on the device. Results stay in device memory,
 * counted against the budget, until sj_server_release.
 *
 * Points passed to sj_server_submit must stay valid (and unchanged) until
 * the request completes; they may be device or host memory. The request is
 * read on the server's own worker stream, which is not ordered after any of
 * the caller's streams: device points must be complete when sj_server_submit
 * is called (the stream that wrote them synchronised, or an event on it
 * waited for).
 */
typedef struct sj_server sj_server;

#define SJ_SERVER_DRY_RUN 1  /* flags: no device work (scheduler tests without a GPU):
                                 a request takes n/1e6 ms twice and its count pass
                                 reports expected_pairs pairs (twice that for even ids;
                                 n when expected_pairs is 0) */

typedef struct sj_server_opts {
    uint32_t slots;             /* concurrent requests (worker threads/streams), 1..64 */
    uint32_t flags;             /* 0 or SJ_SERVER_DRY_RUN */
    uint64_t mem_budget_bytes;  /* soft device-memory budget for admission */
} sj_server_opts;

typedef struct sj_completion {
    uint64_t        req_id;
    int32_t         status;       /* SJ_OK or an SJ_E* code */
    uint32_t        slot;         /* slot that ran the request */
    const uint32_t *pairs_dev;    /* npairs sorted (i, j) pairs, valid until release */
    uint64_t        npairs;
    double          queue_ms;     /* submit -> admitted */
    double          service_ms;   /* admitted -> result ready */
    double          latency_ms;   /* submit -> result ready */
    uint64_t        evals;        /* distance evaluations of the count pass */
    uint64_t        band_rechecks;
} sj_completion;

typedef struct sj_server_info_t {
    uint64_t queued;
    uint64_t running;
    uint64_t mem_used_bytes;
    uint64_t peak_mem_bytes;
    uint64_t over_estimate;      /* requests with expected_pairs > 0 whose result
                                    outgrew the reservation */
    uint64_t completed;
} sj_server_info_t;

int  sj_server_create(const sj_server_opts *opts, sj_server **out);
/* Queues a self-join request (the join of Section III with the method of
 * Sections IV-V; opts as for sj_join_count); *req_id identifies it. opts may
 * be NULL (defaults); expected_pairs 0 means no estimate (the result's
 * memory is reserved after the count pass). Never blocks on
 * device work; see above for the ordering of device points. */
int  sj_server_submit(sj_server *srv, const double *pts, uint64_t n, uint32_t d, double eps,
                      int pts_on_device, const sj_join_opts *opts, uint64_t expected_pairs,
                      uint64_t *req_id);
/* Up to cap completed requests (each reported once); waits up to timeout_ms
 * (0: do not wait, < 0: wait until one completes). */
int  sj_server_poll(sj_server *srv, sj_completion *out, uint32_t cap, uint32_t *count,
                    int32_t timeout_ms);
/* Frees a completed request's result and its memory reservation. */
int  sj_server_release(sj_server *srv, uint64_t req_id);
int  sj_server_info(sj_server *srv, sj_server_info_t *info);
/* Drops queued requests, waits for running ones, frees everything. */
void sj_server_destroy(sj_server *srv);

/*
 * Per-kernel timing with HIP events recorded on the stream each kernel is
 * launched on (off by default; enabling resets the totals). Records are
 * {char name[48]; uint64_t launches; double total_ms;}; *count receives the
 * number of kernels seen (records beyond cap are not written).
 */
typedef struct sj_kernel_time {
    char     name[48];
    uint64_t launches;
    double   total_ms;
} sj_kernel_time;
int sj_profile_enable(int on);
int sj_profile_read(sj_kernel_time *out, uint32_t cap, uint32_t *count);
/* Restricts timing to kernels whose name starts with prefix (NULL or "":
 * every kernel), so a timed region pays for two event records only around
 * the kernels it reports. The string is copied. */
int sj_profile_select(const char *prefix);

/*
 * Device memory held by the library outside the caller's buffers: blocks
 * that calls have handed back and that are kept for reuse (cached_bytes;
 * a later call takes the smallest cached block of at least its size and at
 * most a quarter larger) and blocks in use by indexes, batches and served
 * results (live_bytes). Either pointer may be NULL.
 */
int sj_memory_info(uint64_t *cached_bytes, uint64_t *live_bytes);

/*
 * Waits for the device to be idle and frees every cached block (a process
 * that ran large joins and now needs the memory elsewhere). Live blocks
 * are kept. A failed device allocation does the same by itself before it
 * retries.
 */
int sj_release_cached_memory(void);

/* Thread-local description of the last failure ("" if none). */
const char *sj_last_error(void);

/* Library version string. */
const char *sj_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SJ_H */
