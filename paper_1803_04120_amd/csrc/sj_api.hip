// C ABI of libsj: the index object, the count/fill join, batching and the
// convenience entry point. Every entry point runs inside guarded(), which
// turns internal errors into return codes, synchronises the call's stream
// and only then hands the call's temporaries back to the memory pool.
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "sj.h"
#include "sj_internal.h"
#include "sj_device.h"

using sj::DevBuf;
using sj::Error;

// ------------------------------------------------ allocation-free brute force
// Device scratch of sj_bruteforce_noalloc, a file-scope array that every GPU
// the library runs on holds until the process ends: the count, offset and
// scan tile-sum arrays of at most kNoAllocCells (row, candidate range)
// cells and the fill's overflow word, each region 256-byte aligned. It has
// external linkage, so the device code object keeps it although no kernel
// names it (kernels get its address as an argument).
namespace sj {
constexpr size_t kNoAllocCells = size_t(1) << 21;
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kNaCountOff = 0;
constexpr size_t kNaOffOff = align256(kNaCountOff + kNoAllocCells * sizeof(uint32_t));
constexpr size_t kNaPartOff = align256(kNaOffOff + (kNoAllocCells + 1) * sizeof(uint64_t));
constexpr size_t kNaPartWords = kNoAllocCells / 2048 + 2;  // >= scan_partials(kNoAllocCells)
constexpr size_t kNaFlagOff = align256(kNaPartOff + kNaPartWords * sizeof(uint64_t));
constexpr size_t kNoAllocBytes = align256(kNaFlagOff + sizeof(uint32_t));

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
}  // namespace sj


namespace {

thread_local std::string t_error;
// Statistics of the last join run on this thread (any index, the two-set
// join, the convenience call or the brute force).
thread_local sj_stats t_last_run{};
thread_local bool t_have_last_run = false;

void set_error(const std::string &m) { t_error = m; }

void note_run(const sj_stats &st) {
    t_last_run = st;
    t_have_last_run = true;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <typename F>
int guarded(hipStream_t s, F &&f) {
    sj::pool_enter();
    int rc = SJ_OK;
    try {
        f();
    } catch (const Error &e) {
        set_error(e.what());
        rc = e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        rc = SJ_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        rc = SJ_EDEVICE;
    } catch (...) {
        set_error("unknown error");
        rc = SJ_EDEVICE;
    }
    const hipError_t se = hipStreamSynchronize(s);
    if (se != hipSuccess && rc == SJ_OK) {
        set_error(std::string("stream synchronisation failed: ") + hipGetErrorString(se));
        rc = SJ_EDEVICE;
    }
    sj::pool_leave_after_sync();
    if (rc == SJ_OK) t_error.clear();
    return rc;
}

// Buffers handed to the caller by sj_selfjoin: remembered so sj_free knows
// how to release them.
std::mutex g_out_mu;
std::map<void *, bool> g_out_bufs;  // ptr -> on device

// Band of the FP64 fused-square filter. With d_j the rounded differences and
// T = sum d_j^2 exactly, both the definition's sum S (rounded squares added
// left to right) and the fused sum F (F_1 = fl(d_1^2), F_j = fma(d_j, d_j,
// F_{j-1})) put at most d roundings on every term, so |S - T| and |F - T|
// are at most gamma_d T (gamma_d = d u / (1 - d u), u = 2^-53) and
// |F - S| <= 2 gamma_d / (1 - gamma_d) F. F < eps2 (1 - delta) then implies
// S < eps2 and F > eps2 (1 + delta) implies S > eps2 for any
// delta >= 2 gamma_d / (1 - gamma_d) (1.8e-15 at d = 8); delta = 2^-45 is
// 15 times that at d = 8, twice at d = 64. The bounds hold without underflow; for eps2 below 2^-900 the
// absolute error of subnormal results (a few 2^-1074) is no longer small
// next to delta eps2, and for eps2 above 2^1000 F may overflow: then every
// finite F goes to the exact sum. eps2 = 0: F > 0 exactly when S > 0
// (rounding is monotone and each term enters both sums the same way while
// the partial sums are zero), so lo = hi = 0 is exact.
void fused_band(double eps2, double *lo, double *hi) {
    const double delta = std::ldexp(1.0, -45);
    static_assert(sj::kMaxDim <= 64, "delta covers 2 gamma_d / (1 - gamma_d) up to d = 64");
    if (eps2 == 0.0) {
        *lo = *hi = 0.0;
    } else if (eps2 >= std::ldexp(1.0, -900) && eps2 <= std::ldexp(1.0, 1000)) {
        *lo = eps2 * (1.0 - delta);
        *hi = eps2 * (1.0 + delta);
    } else {
        *lo = -1.0;
        *hi = std::numeric_limits<double>::infinity();
    }
}

// FP32 pre-test thresholds (the reading documented with the band kernel):
// gamma(k, u) = k u / (1 - k u); tau = X 2^-24 (1 + 2^-28) + 2^-126;
// Delta(E) = 4 tau sqrt(dE) + 4 d tau^2 + gamma(d+2, 2^-24)(sqrt E + 2 tau sqrt d)^2
//            + (2d + 2) 2^-126;
// lo = down32(E_a - 2 Delta(E_a)), hi = up32(E_r + 2 Delta(E_r)),
// E_a = eps^2 / (1 + g64), E_r = eps^2 / (1 - g64), g64 = gamma(d+2, 2^-53).
bool band_thresholds(uint32_t d, double eps, double extent, float *lo, float *hi) {
    const double u32 = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53);
    const double tiny = std::ldexp(1.0, -126);
    auto gamma = [](double k, double u) { return k * u / (1.0 - k * u); };
    const double tau = extent * u32 * (1.0 + std::ldexp(1.0, -28)) + tiny;
    if (!(eps >= 64.0 * tau * std::sqrt(static_cast<double>(d)))) return false;
    const double dd = static_cast<double>(d);
    auto delta = [&](double E) {
        const double rE = std::sqrt(E > 0 ? E : 0.0);
        const double a = rE + 2.0 * tau * std::sqrt(dd);
        return 4.0 * tau * std::sqrt(dd * E) + 4.0 * dd * tau * tau + gamma(dd + 2.0, u32) * a * a +
               (2.0 * dd + 2.0) * tiny;
    };
    const double eps2 = eps * eps;
    const double g64 = gamma(dd + 2.0, u64);
    const double Ea = eps2 / (1.0 + g64), Er = eps2 / (1.0 - g64);
    const double l = Ea - 2.0 * delta(Ea), h = Er + 2.0 * delta(Er);
    float lf = static_cast<float>(l);
    if (static_cast<double>(lf) > l) lf = std::nextafter(lf, -std::numeric_limits<float>::infinity());
    float hf = static_cast<float>(h);
    if (static_cast<double>(hf) < h) hf = std::nextafter(hf, std::numeric_limits<float>::infinity());
    *lo = lf;
    *hi = hf;
    return true;
}

}  // namespace

struct sj_index {
    uint64_t n = 0;
    uint32_t d = 0;
    double eps = 0.0;
    sj::GridParams grid{};
    int key_bits = 0;
    uint64_t ncells = 0;
    uint32_t max_cell = 0;
    double bmin[sj::kMaxDim] = {}, bmax[sj::kMaxDim] = {};
    // resident arrays
    DevBuf<double> X;        // d x n, cell order
    DevBuf<float> Y;         // d x n, cell order, shifted FP32 copy (built on demand)
    bool y_ready = false;
    double shift[sj::kMaxDim] = {};
    double extent = 0.0;
    DevBuf<uint32_t> perm;   // A
    DevBuf<uint32_t> cell_of;
    DevBuf<uint64_t> B;
    DevBuf<uint32_t> starts;
    DevBuf<uint32_t> coords;
    DevBuf<uint32_t> masks;
    DevBuf<uint32_t> max_cell_dev;
    uint32_t mask_off[sj::kMaxDim] = {};
    uint32_t mask_words = 0;
    // adjacent-cell search, cached per setting: [0] all adjacent cells,
    // [1] the unicomp subset
    struct Ranges {
        bool ready = false;
        DevBuf<uint64_t> roff;
        uint32_t *rng = nullptr;
        size_t cap = 0;
        uint64_t count = 0;
    } ranges[2];
    int last_ranges = -1;
    // grid-row chunks of the tiled join
    DevBuf<uint32_t> cx;
    uint2 *chunks = nullptr;
    size_t chunks_cap = 0;
    uint32_t nchunks = 0;               // upper bound (launch size)
    DevBuf<uint32_t> nchunks_dev;       // exact count
    uint32_t rows_per_chunk = 0;
    DevBuf<uint2> segs;
    bool chunks_ready = false;
    // hit bits of the last count pass (grid-row kernel, FP64, 5-D and up):
    // word rows per chunk, their exclusive scan, the bits; bits_uni is the
    // search (1 unicomp, 0 full) they were recorded for, -1 when none
    DevBuf<uint32_t> cwords;
    DevBuf<uint64_t> cbase;
    DevBuf<uint32_t> hitbits;
    int bits_uni = -1;
    // join state
    bool counted = false;
    sj_join_opts opts{};
    int band_used = 0;
    float lo = 0.f, hi = 0.f;
    DevBuf<uint32_t> own_cnt, in_cnt, len_orig, len_cell, cur;
    DevBuf<uint64_t> off_orig;   // row offsets in order of i (n + 1)
    DevBuf<uint64_t> off_cell;   // row offsets in cell order (n + 1): whole-result fill layout
    DevBuf<uint64_t> offc;       // off_orig gathered to cell order (batched fills)
    bool offc_ready = false;
    DevBuf<unsigned long long> counters;  // evals, band rechecks
    DevBuf<uint32_t> max_len;
    DevBuf<uint32_t> overflow;
    bool overflow_clear = false;  // the device flag is known to be 0
    DevBuf<uint64_t> summary;  // count pass results read back together
    uint64_t pairs = 0;
    uint32_t max_row = 0;
    uint64_t rows_longer[3] = {0, 0, 0};  // rows longer than 16, 24, 32
    sj_stats stats{};
    // two-set join state between its count and fill (sj_join_rs_count /
    // sj_join_rs_fill): the queries (staged copy if they came from the host),
    // their order, row offsets by query row and by probe position
    struct RsState {
        bool counted = false;
        bool tiled = false;  // which kernel the count ran on
        const double *R = nullptr;
        DevBuf<double> staged;
        uint64_t nr = 0, P = 0;
        uint32_t max_len = 0;
        DevBuf<uint32_t> qperm, words;
        // per-query kernel: counts and offsets by query row and by probe position
        DevBuf<uint32_t> cnt, cnt_k;
        DevBuf<uint64_t> off, off_k;
        // tiled kernel: the nv queries with adjacent cells, in S's grid and
        // sorted by cell (qperm's first nv entries): coordinates (d x nv),
        // dimension-0 cells, their cells and grid-row chunks; row lengths and
        // offsets by query row (nr) and in cell order (nr, zero past nv)
        uint32_t nv = 0, nchunks = 0, rows_per_chunk = 0;
        DevBuf<double> Xq;
        DevBuf<uint32_t> cxq, cell_of, starts, coords, own_cnt, len_orig, len_cell, nchunks_dev, row_stats;
        DevBuf<uint64_t> B, off_orig, off_cell, summary;
        DevBuf<unsigned long long> counters;
        uint2 *chunks = nullptr;
        size_t chunks_cap = 0;
        DevBuf<uint2> segs;
        uint64_t rows_longer[3] = {0, 0, 0};
        uint64_t evals = 0;
        sj_stats stats{};  // of the last two-set join (sj_last_run_stats)
    } rs;
    // second stream of the batched join (default priority), created on first use
    hipStream_t side_stream = nullptr;

    ~sj_index() {
        for (auto &r : ranges)
            if (r.rng) sj::dev_free(r.rng);
        if (chunks) sj::dev_free(chunks);
        if (rs.chunks) sj::dev_free(rs.chunks);
        if (side_stream) (void)hipStreamDestroy(side_stream);
    }
};

namespace {

// Index and last-join statistics, from host-side state only.
sj_stats stats_of(const sj_index &ix) {
    sj_stats st = ix.stats;
    st.n = ix.n;
    st.d = ix.d;
    st.key_bits = static_cast<uint32_t>(ix.key_bits);
    st.cells = ix.ncells;
    for (int j = 0; j < sj::kMaxDim; ++j) st.grid_dims[j] = j < static_cast<int>(ix.d) ? ix.grid.dims[j] : 0;
    st.eps = ix.eps;
    st.cell_width = ix.grid.w;
    st.max_cell_points = ix.max_cell;
    return st;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

void compute_grid(sj_index &ix) {
    const uint32_t d = ix.d;
    double w = std::nextafter(ix.eps * (1.0 + std::ldexp(1.0, -16)),
                              std::numeric_limits<double>::infinity());
    const unsigned __int128 limit = static_cast<unsigned __int128>(1) << 63;
    for (int attempt = 0; attempt < 2100; ++attempt) {
        bool ok = std::isfinite(w);
        unsigned __int128 prod = 1;
        for (uint32_t j = 0; j < d && ok; ++j) {
            const double gmin = ix.bmin[j] - w;
            const double cells = std::floor((ix.bmax[j] - gmin) / w) + 2.0;
            if (!std::isfinite(gmin) || !(cells < 2147483648.0)) {
                ok = false;
                break;
            }
            ix.grid.gmin[j] = gmin;
            ix.grid.dims[j] = static_cast<uint64_t>(cells);
            prod *= static_cast<unsigned __int128>(ix.grid.dims[j]);
            if (prod >= limit) ok = false;
        }
        if (ok) {
            ix.grid.w = w;
            ix.grid.d = d;
            uint64_t stride = 1;
            for (uint32_t j = 0; j < d; ++j) {
                ix.grid.stride[j] = stride;
                stride *= ix.grid.dims[j];
            }
            const uint64_t maxid = stride - 1;
            int bits = 0;
            while (bits < 64 && (maxid >> bits) != 0) ++bits;
            ix.key_bits = bits;
            // dimension-0 sub-cells per cell: 8, fewer when the sub-cell
            // coordinate or the sort key would not fit (SJ_SUBCELL_SHIFT=0..3
            // overrides)
            uint32_t sh = 3;
            if (const char *e = std::getenv("SJ_SUBCELL_SHIFT")) {
                const int v = std::atoi(e);
                if (v >= 0 && v <= 3) sh = static_cast<uint32_t>(v);
            }
            // (sub-cell coordinates plus the window's S stay below 2^32)
            while (sh > 0 && ((ix.grid.dims[0] << sh) >= 0xfffffff0ULL || bits + static_cast<int>(sh) > 64)) --sh;
            ix.grid.sub_shift = sh;
            return;
        }
        w = w * 2.0;
    }
    throw Error(SJ_EGRID, "grid cannot be represented (coordinate range too large for eps)");
}

void validate_points_args(const double *pts, uint64_t n, uint32_t d, double eps) {
    if (d < 1 || d > static_cast<uint32_t>(sj::kMaxDim)) throw Error(SJ_EINVAL, "d must be in [1, 8]");
    if (!(eps > 0.0) || !std::isfinite(eps)) throw Error(SJ_EINVAL, "eps must be finite and > 0");
    if (n >= 0xffffffffULL) throw Error(SJ_EINVAL, "n must be below 2^32 - 1");
    if (n > 0 && !pts) throw Error(SJ_EINVAL, "pts is NULL");
}

void validate_opts(const sj_join_opts *o) {
    if (!o) return;
    if (o->precision != SJ_FP64 && o->precision != SJ_FP32_BAND)
        throw Error(SJ_EINVAL, "precision must be SJ_FP64 or SJ_FP32_BAND");
    if (o->sort_output != 0 && o->sort_output != 1) throw Error(SJ_EINVAL, "opts.sort_output must be 0 or 1");
}

sj_join_opts resolve_opts(const sj_join_opts *o) {
    sj_join_opts r;
    sj_default_opts(&r);
    if (o) r = *o;
    if (r.min_batches == 0) r.min_batches = 1;
    return r;
}

void build(sj_index &ix, const double *pts, int on_device, hipStream_t s) {
    const double t0 = now_ms();
    const uint64_t n = ix.n;
    const uint32_t d = ix.d;
    DevBuf<double> staged;
    const double *dp = pts;
    if (!on_device) {
        staged.reset(n * d);
        SJ_HIP(hipMemcpyAsync(staged.ptr, pts, n * d * sizeof(double), hipMemcpyHostToDevice, s));
        dp = staged.ptr;
    }
    // bounding box (Section IV-B)
    // [0, 2 kMaxDim): min and max; the word after them: the NaN/Inf flag
    DevBuf<double> bb(2 * sj::kMaxDim + 1);
    sj::launch_bbox(dp, n, d, bb.ptr, reinterpret_cast<uint32_t *>(bb.ptr + 2 * sj::kMaxDim), s);
    sj::HostStage hs;
    SJ_HIP(hipMemcpyAsync(hs.p, bb.ptr, bb.bytes(), hipMemcpyDeviceToHost, s));
    // the buffers whose sizes depend only on n and d are taken from the pool
    // while the bounding box runs (32-bit cell ids use the first half of the
    // 64-bit key buffers)
    ix.perm.reset(n);
    DevBuf<uint32_t> ids_alt(n);
    ix.cell_of.reset(n);
    ix.B.reset(n);
    ix.starts.reset(n + 1);
    DevBuf<uint64_t> keys64(n), keys64_alt(n);
    ix.coords.reset(n * d);
    ix.X.reset(n * d);
    ix.cx.reset(n);
    SJ_HIP(hipStreamSynchronize(s));
    const double *hb = hs.as<double>();
    if (*reinterpret_cast<const uint32_t *>(hb + 2 * sj::kMaxDim)) throw Error(SJ_EINVAL, "coordinates contain NaN or Inf");
    for (uint32_t j = 0; j < d; ++j) {
        ix.bmin[j] = hb[j];
        ix.bmax[j] = hb[sj::kMaxDim + j];
    }
    compute_grid(ix);
    // cell ids and the sort by cell (A), inside a cell by dimension-0 sub-cell
    const int sh = static_cast<int>(ix.grid.sub_shift);
    const int sort_bits = ix.key_bits + sh;
    if (sort_bits <= 32) {
        uint32_t *keys = reinterpret_cast<uint32_t *>(keys64.ptr);
        uint32_t *keys_alt = reinterpret_cast<uint32_t *>(keys64_alt.ptr);
        sj::launch_cell_keys_u32(dp, n, ix.grid, keys, ix.perm.ptr, s);
        if (sj::radix_sort_u32(keys, ix.perm.ptr, keys_alt, ids_alt.ptr, n, sort_bits, s)) {
            std::swap(keys, keys_alt);
            std::swap(ix.perm, ids_alt);
        }
        sj::build_cells<uint32_t>(keys, n, sh, ix.cell_of.ptr, ix.B.ptr, ix.starts.ptr, s);
    } else {
        uint64_t *keys = keys64.ptr, *keys_alt = keys64_alt.ptr;
        sj::launch_cell_keys_u64(dp, n, ix.grid, keys, ix.perm.ptr, s);
        if (sj::radix_sort_u64(keys, ix.perm.ptr, keys_alt, ids_alt.ptr, n, sort_bits, s)) {
            std::swap(keys, keys_alt);
            std::swap(ix.perm, ids_alt);
        }
        sj::build_cells<uint64_t>(keys, n, sh, ix.cell_of.ptr, ix.B.ptr, ix.starts.ptr, s);
    }
    // per-cell coordinates and occupancy masks M_j (Section IV-C)
    uint64_t words = 0;
    for (uint32_t j = 0; j < d; ++j) {
        ix.mask_off[j] = static_cast<uint32_t>(words);
        words += (ix.grid.dims[j] + 31) / 32;
    }
    sj::MaskOffsets moff{};
    for (uint32_t j = 0; j < d; ++j) moff.off[j] = ix.mask_off[j];
    if (words <= (1ull << 26)) {
        ix.mask_words = static_cast<uint32_t>(words);
        ix.masks.reset(words);
    } else {
        ix.mask_words = 0;  // masks only prune; a grid this wide goes without
    }
    // |G| stays on the device until the end of the build: tables that depend
    // on it are sized by n (an upper bound)
    ix.max_cell_dev.ensure(1);
    sj::launch_cell_coords_masks(ix.B.ptr, ix.starts.ptr, n, ix.cell_of.ptr + (n - 1), ix.grid, ix.coords.ptr,
                                 ix.masks.ptr, moff, ix.mask_words, ix.max_cell_dev.ptr, s);
    // cell-ordered structure of arrays
    sj::launch_gather_soa(dp, ix.perm.ptr, n, d, ix.X.ptr, ix.grid, ix.cx.ptr, s);
    for (uint32_t j = 0; j < d; ++j) {
        ix.shift[j] = 0.5 * (ix.bmin[j] + ix.bmax[j]);
        ix.extent = std::max(ix.extent, std::max(std::fabs(ix.bmax[j] - ix.shift[j]),
                                                 std::fabs(ix.bmin[j] - ix.shift[j])));
    }
    SJ_HIP(hipMemcpyAsync(hs.p, ix.cell_of.ptr + (n - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipMemcpyAsync(hs.as<uint32_t>() + 1, ix.max_cell_dev.ptr, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    ix.ncells = static_cast<uint64_t>(*hs.as<uint32_t>()) + 1;
    ix.max_cell = hs.as<uint32_t>()[1];
    ix.stats.ms_build = now_ms() - t0;
}

void ensure_ranges(sj_index &ix, int unicomp, hipStream_t s) {
    ix.last_ranges = unicomp;
    auto &R = ix.ranges[unicomp];
    if (R.ready) return;
    sj::SearchArgs a{};
    a.B = ix.B.ptr;
    a.starts = ix.starts.ptr;
    a.coords = ix.coords.ptr;
    a.masks = ix.mask_words ? ix.masks.ptr : nullptr;
    for (uint32_t j = 0; j < ix.d; ++j) {
        a.mask_off[j] = ix.mask_off[j];
        a.dims[j] = ix.grid.dims[j];
        a.stride[j] = ix.grid.stride[j];
    }
    a.ncells = static_cast<uint32_t>(ix.ncells);
    a.d = ix.d;
    R.roff.ensure(ix.ncells + 1);
    R.count = sj::build_ranges(a, unicomp, R.roff.ptr, &R.rng, &R.cap, s);
    R.ready = true;
}

// Which refine kernel runs whole-result passes: the grid-row tiled kernel
// (default) or the per-point range kernel (SJ_JOIN_KERNEL=ranges).
bool use_tiled() {
    const char *e = std::getenv("SJ_JOIN_KERNEL");
    return !(e && std::strcmp(e, "ranges") == 0);
}

sj::TileArgs tile_args(sj_index &ix) {
    sj::TileArgs t{};
    t.B = ix.B.ptr;
    t.ncells = static_cast<uint32_t>(ix.ncells);
    t.coords = ix.coords.ptr;
    t.masks = ix.mask_words ? ix.masks.ptr : nullptr;
    for (uint32_t j = 0; j < ix.d; ++j) {
        t.mask_off[j] = ix.mask_off[j];
        t.dims[j] = ix.grid.dims[j];
        t.stride[j] = ix.grid.stride[j];
    }
    t.cx = ix.cx.ptr;
    t.cxq = ix.cx.ptr;
    t.sub_shift = ix.grid.sub_shift;
    t.chunks = ix.chunks;
    t.nchunks = ix.nchunks;
    t.nchunks_dev = ix.nchunks_dev.ptr;
    t.chunk0 = 0;
    t.chunk_end = 0xffffffffu;
    t.rows_per_chunk = ix.rows_per_chunk;
    t.segs = ix.segs.ptr;
    return t;
}

// Row sort fused into the full fill, or run as its own kernels after it.
// Fused in 1..3-D: the rows stay in LDS and are written once, sorted. From
// 4-D on the fill evaluates 27..2187 candidate rows per chunk and needs every
// wave it can hold; the LDS row slots would cut that to 3..4 waves per SIMD
// (measured on a mixed 2..6-D request stream: 137 ms fused vs 74 ms + 6 ms of
// row sorts unfused). SJ_FUSED_SORT=0|1 overrides.
bool use_fused_sort(uint32_t d) {
    const char *e = std::getenv("SJ_FUSED_SORT");
    if (e && std::strcmp(e, "0") == 0) return false;
    if (e && std::strcmp(e, "1") == 0) return true;
    return d <= 3;
}

// Entries per lane in the fused fill's LDS row slot (SJ_FUSED_NS=16|24|32
// overrides). A larger slot keeps more rows out of out_j (a longer row costs
// the wave a sort of its own) but holds more LDS per wave, so fewer waves fit
// on a CU (5, 4, 3 for 16, 24, 32 in 2-D). The smallest slot that at most 5%
// of the rows exceed; 32 otherwise.
uint32_t fused_slot(const sj_index &ix) {
    const char *e = std::getenv("SJ_FUSED_NS");
    if (e) {
        const int v = std::atoi(e);
        if (v == 16 || v == 24 || v == 32) return static_cast<uint32_t>(v);
    }
    const double lim = 0.05 * static_cast<double>(ix.n);
    if (static_cast<double>(ix.rows_longer[0]) <= lim) return 16u;
    if (static_cast<double>(ix.rows_longer[1]) <= lim) return 24u;
    return 32u;
}

void ensure_chunks(sj_index &ix, hipStream_t s) {
    if (ix.chunks_ready) return;
    ix.nchunks_dev.ensure(1);
    // grid rows: one per occupied combination of the dimension-1..d-1 cells
    uint64_t rows_bound = 1;
    for (uint32_t j = 1; j < ix.d; ++j)
        rows_bound = ix.grid.dims[j] > (UINT64_MAX / 2) / rows_bound ? UINT64_MAX / 2 : rows_bound * ix.grid.dims[j];
    ix.nchunks = sj::build_chunks(ix.coords.ptr, ix.starts.ptr, static_cast<uint32_t>(ix.ncells),
                                  static_cast<uint32_t>(ix.n), ix.d, rows_bound, &ix.chunks, &ix.chunks_cap,
                                  ix.nchunks_dev.ptr, s);
    uint32_t r3 = 1;
    for (uint32_t j = 1; j < ix.d; ++j) r3 *= 3;
    ix.rows_per_chunk = r3;
    ix.segs.reset(static_cast<size_t>(ix.nchunks) * r3);
    sj::build_chunk_segments(tile_args(ix), ix.cell_of.ptr, ix.starts.ptr, ix.d, ix.segs.ptr, s);
    ix.chunks_ready = true;
}

void ensure_f32(sj_index &ix, hipStream_t s) {
    if (ix.y_ready) return;
    ix.Y.reset(ix.n * ix.d);
    sj::launch_make_f32(ix.X.ptr, ix.n, ix.d, ix.shift, ix.Y.ptr, s);
    ix.y_ready = true;
}

// Hit bits for the fill pass (grid-row kernel, FP64, 5-D and up): the count
// pass records each tested candidate's outcome so that the fill of the same
// search reads them instead of testing again. Sized exactly from the chunks'
// segments (one read-back); taken only when they fit in 40% of the device
// memory that is free or cached by the pool (SJ_HIT_BITS=0: never).
void prepare_hit_bits(sj_index &ix, int uni, sj::TileArgs &tt, hipStream_t s) {
    ix.bits_uni = -1;
    ix.stats.hit_bit_bytes = 0;
    ix.hitbits.release();
    if (ix.band_used || ix.d < sj::kHitBitsMinDim) return;
    const char *e = std::getenv("SJ_HIT_BITS");
    if (e && std::strcmp(e, "0") == 0) return;
    const uint32_t nslots = ix.nchunks + 1;
    ix.cwords.ensure(nslots + 1);  // the last word: the overflow flag
    ix.cbase.ensure(nslots);
    uint32_t *big = ix.cwords.ptr + nslots;
    sj::launch_fill_u32(big, 1, 0u, s);
    sj::launch_chunk_words(tt, ix.cell_of.ptr, ix.d, uni, nslots, ix.cwords.ptr, big, s);
    sj::scan_exclusive_u32_to_u64(ix.cwords.ptr, ix.cbase.ptr, nslots, s);
    sj::HostStage hs;
    SJ_HIP(hipMemcpyAsync(hs.p, ix.cbase.ptr + (nslots - 1), sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipMemcpyAsync(hs.as<uint32_t>() + 2, big, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    const uint64_t rows = *hs.as<uint64_t>();
    if (hs.as<uint32_t>()[2] || rows == 0) return;
    const uint64_t bytes = rows * 64 * sizeof(uint32_t);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    uint64_t cached = 0;
    sj::pool_info(&cached, nullptr);
    if (static_cast<double>(bytes) > 0.4 * static_cast<double>(free_b + cached)) return;
    try {
        ix.hitbits.reset(rows * 64);
    } catch (const Error &err) {
        if (err.code != SJ_ENOMEM) throw;
        return;
    }
    tt.bits = ix.hitbits.ptr;
    tt.cbase = ix.cbase.ptr;
    ix.bits_uni = uni;
    ix.stats.hit_bit_bytes = bytes;
}

sj::JoinArgs base_args(sj_index &ix, int mode) {
    sj::JoinArgs a{};
    const auto &R = ix.ranges[mode];
    a.X = ix.X.ptr;
    a.Y = ix.band_used ? ix.Y.ptr : nullptr;
    a.n = static_cast<uint32_t>(ix.n);
    a.Xq = a.X;
    a.Yq = a.Y;
    a.nqs = a.n;
    a.permq = ix.perm.ptr;
    a.cell_of = ix.cell_of.ptr;
    a.starts = ix.starts.ptr;
    a.roff = R.roff.ptr;
    a.rng = reinterpret_cast<const uint2 *>(R.rng);
    a.qlist = nullptr;
    a.nq = static_cast<uint32_t>(ix.n);
    a.eps2 = ix.eps * ix.eps;
    a.lo = ix.lo;
    a.hi = ix.hi;
    fused_band(a.eps2, &a.flo, &a.fhi);
    a.own_cnt = ix.own_cnt.ptr;
    a.in_cnt = ix.in_cnt.ptr;
    a.offc = nullptr;
    a.perm = ix.perm.ptr;
    a.evals = ix.counters.ptr;
    a.band_rechecks = ix.counters.ptr + sj::kCounterSlots * sj::kCounterStride;
    return a;
}

void join_count(sj_index &ix, const sj_join_opts &o, hipStream_t s) {
    const double t0 = now_ms();
    ix.counted = false;
    ix.opts = o;
    ix.pairs = 0;
    ix.max_row = 0;
    ix.stats.evals = ix.stats.band_rechecks = 0;
    ix.stats.hit_bit_bytes = 0;
    ix.stats.pairs = 0;
    ix.stats.max_row_pairs = 0;
    ix.stats.unicomp_used = o.unicomp ? 1u : 0u;
    ix.band_used = 0;
    // The FP32 pre-test runs up to 5-D. From 6-D on the grid-row kernel's FP64
    // path (fused-square filter, hit bits) is the faster one and runs instead
    // (same pairs; precision_used says which ran): 10M uniform points,
    // count + fill, 6-D at 32 and 256 neighbours 52.4 / 170.0 ms with the
    // pre-test against 45.8 / 133.3 ms without; at 3..5-D the pre-test is
    // 2-7% faster.
    constexpr uint32_t kBandMaxDimTiled = 5;
    if (o.precision == SJ_FP32_BAND && ix.n > 0 && !(use_tiled() && ix.d > kBandMaxDimTiled))
        ix.band_used = band_thresholds(ix.d, ix.eps, ix.extent, &ix.lo, &ix.hi) ? 1 : 0;
    ix.stats.precision_used = ix.band_used ? SJ_FP32_BAND : SJ_FP64;
    if (ix.n == 0) {
        ix.counted = true;
        ix.stats.ms_count = now_ms() - t0;
        note_run(stats_of(ix));
        return;
    }
    const int uni = o.unicomp ? 1 : 0;
    const bool tiled = use_tiled();
    if (tiled)
        ensure_chunks(ix, s);
    else
        ensure_ranges(ix, uni, s);
    if (ix.band_used) ensure_f32(ix, s);
    const uint64_t n = ix.n;
    ix.own_cnt.ensure(n);
    ix.in_cnt.ensure(n);
    ix.len_orig.ensure(n);
    ix.off_orig.ensure(n + 1);
    ix.off_cell.ensure(n + 1);
    ix.len_cell.ensure(n);
    ix.offc_ready = false;
    const size_t nctr = 2 * sj::kCounterSlots * sj::kCounterStride;
    ix.counters.ensure(nctr);
    ix.max_len.ensure(sj::kRowStatWords);
    sj::ZeroSpans z{};
    if (uni) z.add(ix.in_cnt.ptr, n);
    z.add(ix.counters.ptr, 2 * nctr);
    sj::launch_zero_spans(z, s);
    sj::JoinArgs a = base_args(ix, uni);
    sj::TileArgs tt{};
    if (tiled) {
        tt = tile_args(ix);
        prepare_hit_bits(ix, uni, tt, s);
    }
    if (tiled)
        sj::launch_join_tiled(a, tt, ix.d, uni, sj::kCount, ix.band_used, s);
    else
        sj::launch_join(a, ix.d, uni, sj::kCount, ix.band_used, s);
    sj::launch_row_lengths(ix.own_cnt.ptr, uni ? ix.in_cnt.ptr : nullptr, ix.perm.ptr, n,
                           ix.len_orig.ptr, ix.len_cell.ptr, ix.max_len.ptr, s);
    sj::scan_exclusive_u32_to_u64_x2(ix.len_orig.ptr, ix.off_orig.ptr, ix.len_cell.ptr, ix.off_cell.ptr, n, s);
    ix.summary.ensure(8);
    ix.overflow.ensure(1);
    sj::launch_count_summary(ix.off_orig.ptr, n, ix.max_len.ptr, ix.counters.ptr,
                             tiled ? ix.nchunks_dev.ptr : nullptr, ix.summary.ptr, ix.overflow.ptr, s);
    sj::HostStage hs;
    SJ_HIP(hipMemcpyAsync(hs.p, ix.summary.ptr, 8 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    const uint64_t *sm = hs.as<uint64_t>();
    ix.pairs = sm[0];
    ix.max_row = static_cast<uint32_t>(sm[1]);
    ix.stats.evals = sm[2];
    ix.stats.band_rechecks = sm[3];
    if (tiled) ix.stats.chunks = static_cast<uint32_t>(sm[4]);
    for (int k = 0; k < 3; ++k) ix.rows_longer[k] = sm[5 + k];
    ix.stats.pairs = ix.pairs;
    ix.stats.max_row_pairs = ix.max_row;
    ix.stats.ranges = tiled ? 0 : ix.ranges[uni].count;
    ix.overflow_clear = true;
    ix.counted = true;
    ix.stats.ms_count = now_ms() - t0;
    note_run(stats_of(ix));
}

void check_overflow(sj_index &ix, hipStream_t s) {
    sj::HostStage hs;
    SJ_HIP(hipMemcpyAsync(hs.p, ix.overflow.ptr, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    if (*hs.as<uint32_t>()) throw Error(SJ_EDEVICE, "internal: the fill pass disagreed with the count pass");
    ix.overflow_clear = true;
}

// Fill + row sort of result rows [i0, i1) into out_j / pairs (batch-relative).
// unicomp_fill: evaluate the unicomp subset over all points (valid only for
// the single batch holding every row); otherwise the batch's own query
// points scan all adjacent cells and write only their own rows.
struct Scratch {
    DevBuf<uint32_t> qlist, flags;
};

void fill_rows(sj_index &ix, uint64_t i0, uint64_t i1, uint64_t base, uint64_t cap,
               bool unicomp_fill, uint32_t *out_j, uint32_t *pairs, Scratch &sc, hipStream_t s,
               uint32_t *cols = nullptr, bool sort_rows = true) {
    const uint64_t n = ix.n;
    const int mode = unicomp_fill ? 1 : 0;
    const bool whole = (i0 == 0 && i1 == n);
    const bool tiled = whole && use_tiled();
    if (tiled)
        ensure_chunks(ix, s);
    else
        ensure_ranges(ix, mode, s);
    sj::JoinArgs a = base_args(ix, tiled ? 0 : mode);
    a.out_j = out_j;
    a.out_base = base;
    a.out_cap = cap;
    ix.overflow.ensure(1);
    a.overflow = ix.overflow.ptr;
    if (whole) {
        // whole result: rows laid out in cell order, scattered to order of i
        // by the row sort
        a.offc = ix.off_cell.ptr;
    } else {
        if (!ix.offc_ready) {
            ix.offc.ensure(n);
            sj::launch_gather_offsets(ix.off_orig.ptr, ix.perm.ptr, n, ix.offc.ptr, s);
            ix.offc_ready = true;
        }
        a.offc = ix.offc.ptr;
    }
    if (unicomp_fill) {
        ix.cur.ensure(n);
        sj::launch_fill_u32(ix.cur.ptr, n, 0u, s);
        a.cur = ix.cur.ptr;
    }
    // whole result, full fill: each point's row is complete when its own
    // evaluation ends, so the row sort runs inside the fill kernel
    const bool fused = tiled && !unicomp_fill && whole && !cols && use_fused_sort(ix.d);
    if (tiled) {
        uint32_t ns = 0;
        if (fused) {
            ns = fused_slot(ix);
            a.off_orig = ix.off_orig.ptr;
            a.pairs = reinterpret_cast<uint2 *>(pairs);
        }
        if (whole && !ix.overflow_clear) sj::launch_fill_u32(a.overflow, 1, 0u, s);
        ix.overflow_clear = false;
        // the count's hit bits when they were recorded for this search
        sj::TileArgs tt = tile_args(ix);
        const bool replay = !fused && ix.bits_uni == mode && ix.hitbits.ptr;
        if (replay) {
            tt.bits = ix.hitbits.ptr;
            tt.cbase = ix.cbase.ptr;
        }
        sj::launch_join_tiled(a, tt, ix.d, mode, replay ? sj::kReplay : sj::kFill, ix.band_used, s, ns);
        if (replay) {
            // read once: the memory goes back to the pool when the call ends
            ix.hitbits.release();
            ix.bits_uni = -1;
        }
        if (fused) {
            // the fused fill sorts rows of up to 64 itself
            sj::launch_rowsort_long(ix.off_cell.ptr, ix.off_orig.ptr, ix.perm.ptr, n, out_j, pairs,
                                    ix.max_row, 64, s, nullptr, ix.opts.sort_output != 0);
            return;
        }
    } else if (unicomp_fill) {
        if (whole && !ix.overflow_clear) sj::launch_fill_u32(a.overflow, 1, 0u, s);
        ix.overflow_clear = false;
        sj::launch_join(a, ix.d, 1, sj::kFill, ix.band_used, s);
    } else {
        if (whole) {
            if (!ix.overflow_clear) sj::launch_fill_u32(a.overflow, 1, 0u, s);
            a.qlist = nullptr;
            a.nq = static_cast<uint32_t>(n);
        } else {
            sc.qlist.ensure(n);
            sc.flags.ensure(n);
            a.nq = sj::build_query_list(ix.perm.ptr, n, i0, i1, sc.flags.ptr, sc.qlist.ptr, s);
            a.qlist = sc.qlist.ptr;
        }
        ix.overflow_clear = false;
        sj::launch_join(a, ix.d, 0, sj::kFill, ix.band_used, s);
    }
    if (!sort_rows) return;  // the rows stay in out_j (cell order) for the caller
    if (whole)
        sj::launch_rowsort_cells(ix.off_cell.ptr, ix.off_orig.ptr, ix.perm.ptr, n, out_j, pairs,
                                 ix.max_row, s, cols, ix.opts.sort_output != 0);
    else
        sj::launch_rowsort(ix.off_orig.ptr, i0, i1, base, out_j, pairs, ix.max_row, s, cols,
                           ix.opts.sort_output != 0);
}

// The fill pass may evaluate the unicomp subset (every candidate's mirrored
// entries then take a slot in its row with one atomic per tile) or all
// adjacent cells (each point writes only its own row, no atomics, twice the
// distance evaluations; in 1..3-D its rows are sorted inside the fill).
// Both fill the same rows. Measured on the 10M-point joins: from 4-D on the
// unicomp fill is faster at every density (4-D: 4.1 against 4.6 ms at 32
// neighbours, 19.2 against 24.2 ms at 256; 5-D: 45 against 72 ms); in 3-D
// the full fill with its fused row sort is as fast or faster (4.4 against
// 2.5 + 2.3 ms of row sorts at 32 neighbours), so there the unicomp fill is
// taken only when pairs are under 8% of the unicomp evaluations.
// SJ_FILL_MODE=full|unicomp overrides the choice.
bool choose_unicomp_fill(const sj_index &ix) {
    if (!ix.opts.unicomp) return false;
    const char *e = std::getenv("SJ_FILL_MODE");
    if (e && std::strcmp(e, "full") == 0) return false;
    if (e && std::strcmp(e, "unicomp") == 0) return true;
    if (ix.d >= 4) return true;
    return static_cast<double>(ix.pairs) < 0.08 * static_cast<double>(ix.stats.evals);
}

void join_fill_all(sj_index &ix, uint32_t *pairs_dev, hipStream_t s, uint32_t *cols_dev = nullptr) {
    const double t0 = now_ms();
    if (ix.n == 0 || ix.pairs == 0) return;
    DevBuf<uint32_t> out_j(ix.pairs);
    Scratch sc;
    ix.overflow.ensure(1);
    const bool uni_fill = choose_unicomp_fill(ix);
    ix.stats.fill_unicomp = uni_fill ? 1u : 0u;
    // (a whole-result fill clears the overflow flag itself)
    fill_rows(ix, 0, ix.n, 0, ix.pairs, uni_fill, out_j.ptr, pairs_dev, sc, s, cols_dev);
    check_overflow(ix, s);
    ix.stats.batches = 1;
    ix.stats.ms_fill = now_ms() - t0;
    note_run(stats_of(ix));
}

// Batched delivery (Section V-A) in runs of cell order: batch b holds the
// rows of the cell-ordered points [pos[b], pos[b+1]), a range of whole
// grid-row chunks (so the fill is the tiled kernel, with its row sort fused
// in 1..3-D) or, when the capacity is below what one chunk can hold, of
// single points (the per-point kernel). Batches are sized from the exact
// row lengths of the count pass, at least min_batches, and each is sorted
// by (i, j) within itself: its row lengths are scattered to order of i and
// scanned, and the fill writes every row at that batch-local offset.
// Double-buffered, so batch b+1 computes while the callback consumes b.
int join_batched_cells(sj_index &ix, sj_run_cb cb, void *user, hipStream_t s) {
    const double t0 = now_ms();
    const uint64_t n = ix.n, P = ix.pairs;
    if (n == 0 || P == 0) {
        ix.stats.batches = 0;
        note_run(stats_of(ix));
        return 0;
    }
    const uint64_t cap = ix.opts.batch_capacity_pairs ? ix.opts.batch_capacity_pairs : P;
    if (ix.max_row > cap)
        throw Error(SJ_ECAPACITY, "batch capacity is smaller than the longest result row (" +
                                      std::to_string(ix.max_row) + " pairs)");
    // work units: grid-row chunks (at most 64 rows each) when the capacity
    // leaves room for one, else single points
    const bool tiled = use_tiled() && static_cast<double>(cap) >= 128.0 * ix.max_row;
    if (tiled) ensure_chunks(ix, s);
    const uint32_t units = tiled ? static_cast<uint32_t>(ix.stats.chunks) : static_cast<uint32_t>(n);
    const uint64_t gran = tiled ? 64ull * ix.max_row : ix.max_row;
    const uint64_t per = cap > gran ? cap - gran : 1;
    uint64_t nb64 = std::max<uint64_t>(ix.opts.min_batches, (P + per - 1) / per);
    if (cap >= P && ix.opts.min_batches <= 1) nb64 = 1;
    nb64 = std::min<uint64_t>(nb64, units);
    const uint32_t nb = static_cast<uint32_t>(std::max<uint64_t>(nb64, 1));
    std::vector<uint32_t> unit(nb + 1);
    std::vector<uint64_t> pos(nb + 1), boff(nb + 1);
    {
        DevBuf<uint32_t> du(nb + 1);
        DevBuf<uint64_t> dp(nb + 1), dof(nb + 1);
        sj::launch_batch_units(tiled ? ix.chunks : nullptr, ix.off_cell.ptr, n, units, P, nb, du.ptr, dp.ptr,
                               dof.ptr, s);
        SJ_HIP(hipMemcpyAsync(unit.data(), du.ptr, (nb + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        SJ_HIP(hipMemcpyAsync(pos.data(), dp.ptr, (nb + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        SJ_HIP(hipMemcpyAsync(boff.data(), dof.ptr, (nb + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        SJ_HIP(hipStreamSynchronize(s));
    }
    uint64_t maxbatch = 0;
    for (uint32_t b = 0; b < nb; ++b) maxbatch = std::max(maxbatch, boff[b + 1] - boff[b]);
    if (maxbatch > cap) throw Error(SJ_EDEVICE, "internal: a planned batch exceeds the capacity");
    // Where the unicomp fill is the faster one and the neighbour ids of the
    // whole result (4 bytes per pair, half the pairs' size) fit in half the
    // free device memory, every row is filled once, unicomp, in cell order,
    // and each run only sorts its rows out of that table. Otherwise each run
    // fills its own rows with the full search (unicomp's mirrored entries
    // would land in other runs' rows). SJ_BATCH_FILL=whole|runs overrides.
    bool whole_fill = false;
    if (tiled && choose_unicomp_fill(ix)) {
        size_t free_b = 0, total_b = 0;
        whole_fill = hipMemGetInfo(&free_b, &total_b) == hipSuccess && 4 * P <= free_b / 2;
    }
    if (const char *e = std::getenv("SJ_BATCH_FILL")) {
        if (std::strcmp(e, "runs") == 0) whole_fill = false;
        if (std::strcmp(e, "whole") == 0) whole_fill = tiled && ix.opts.unicomp;
    }
    // per-run fills test again (the hit bits serve the whole fill only):
    // their memory goes back to the pool before the runs' buffers are taken
    if (!whole_fill) {
        ix.hitbits.release();
        ix.bits_uni = -1;
    }
    ix.stats.fill_unicomp = whole_fill ? 1u : 0u;  // else every point writes its own row
    const bool fused = tiled && !whole_fill && use_fused_sort(ix.d);
    const uint32_t ns = fused ? fused_slot(ix) : 0;
    const int nsets = nb > 1 ? 2 : 1;
    DevBuf<uint32_t> out_j[2], pairs[2], len_b[2], out_all;
    DevBuf<uint64_t> off_b[2];
    for (int k = 0; k < nsets; ++k) {
        if (!whole_fill) out_j[k].reset(std::max<uint64_t>(1, maxbatch));
        pairs[k].reset(2 * std::max<uint64_t>(1, maxbatch));
        len_b[k].reset(n);
        off_b[k].reset(n + 1);
    }
    if (!tiled) ensure_ranges(ix, 0, s);
    // Batches alternate between the caller's stream and a second one, each
    // with its own buffers: a batch's fill launch holds few rounds of
    // long-running waves, and its tail overlaps the next batch's start.
    // Batch b reuses the buffers of batch b - 2, which ran on the same
    // stream and was delivered before b is enqueued.
    hipStream_t ss[2] = {s, s};
    if (nsets > 1) {
        if (!ix.side_stream) SJ_HIP(hipStreamCreateWithFlags(&ix.side_stream, hipStreamNonBlocking));
        ss[1] = ix.side_stream;
    }
    hipEvent_t ev[3];
    SJ_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    SJ_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    SJ_HIP(hipEventCreateWithFlags(&ev[2], hipEventDisableTiming));
    struct EvGuard {
        hipEvent_t *e;
        hipStream_t side;
        ~EvGuard() {
            // no work of this call may outlive it on the second stream (its
            // freed blocks are released once the caller's stream is synchronised)
            if (side) (void)hipStreamSynchronize(side);
            (void)hipEventDestroy(e[0]);
            (void)hipEventDestroy(e[1]);
            (void)hipEventDestroy(e[2]);
        }
    } evg{ev, nsets > 1 ? ss[1] : nullptr};
    int rc = 0;
    auto deliver = [&](uint32_t b) {
        const int k = b & 1;
        SJ_HIP(hipEventSynchronize(ev[k]));
        if (rc == 0 && cb) rc = cb(user, pairs[k].ptr, boff[b + 1] - boff[b], b, pos[b], pos[b + 1]);
    };
    ix.overflow.ensure(1);
    sj::launch_fill_u32(ix.overflow.ptr, 1, 0u, s);
    ix.overflow_clear = true;
    if (whole_fill) {
        out_all.reset(P);
        Scratch sc;
        fill_rows(ix, 0, n, 0, P, true, out_all.ptr, nullptr, sc, s, nullptr, false);
    }
    ix.overflow_clear = false;
    if (nsets > 1) {
        // the second stream starts after everything before on the caller's
        SJ_HIP(hipEventRecord(ev[2], s));
        SJ_HIP(hipStreamWaitEvent(ss[1], ev[2], 0));
    }
    for (uint32_t b = 0; b < nb && rc == 0; ++b) {
        const int k = b & 1;
        hipStream_t st = ss[k];
        const uint64_t r0 = pos[b], r1 = pos[b + 1], bp = boff[b + 1] - boff[b];
        if (bp > 0) {
            // the batch's row offsets in order of i
            sj::launch_fill_u32(len_b[k].ptr, n, 0u, st);
            sj::launch_batch_lengths(ix.len_cell.ptr, ix.perm.ptr, r0, r1, len_b[k].ptr, st);
            sj::scan_exclusive_u32_to_u64(len_b[k].ptr, off_b[k].ptr, n, st);
            sj::JoinArgs a = base_args(ix, 0);
            a.out_j = out_j[k].ptr;
            a.offc = ix.off_cell.ptr;
            a.out_base = boff[b];
            a.out_cap = bp;
            a.overflow = ix.overflow.ptr;
            if (whole_fill) {
                // the run's rows from the whole table (rows in cell order at
                // off_cell), sorted into the run's buffer
                sj::launch_rowsort_range(ix.off_cell.ptr, r0, r1, 0, off_b[k].ptr, ix.perm.ptr, out_all.ptr,
                                         pairs[k].ptr, ix.max_row, 0u, st, nullptr, ix.opts.sort_output != 0);
            } else if (tiled) {
                sj::TileArgs t = tile_args(ix);
                t.chunk0 = unit[b];
                t.chunk_end = unit[b + 1];
                if (fused) {
                    a.off_orig = off_b[k].ptr;
                    a.pairs = reinterpret_cast<uint2 *>(pairs[k].ptr);
                }
                sj::launch_join_tiled(a, t, ix.d, 0, sj::kFill, ix.band_used, st, ns);
            } else {
                a = base_args(ix, 0);
                a.out_j = out_j[k].ptr;
                a.offc = ix.off_cell.ptr;
                a.out_base = boff[b];
                a.out_cap = bp;
                a.overflow = ix.overflow.ptr;
                a.qlist = nullptr;
                a.qbase = static_cast<uint32_t>(r0);
                a.nq = static_cast<uint32_t>(r1 - r0);
                sj::launch_join(a, ix.d, 0, sj::kFill, ix.band_used, st);
            }
            if (!whole_fill)
                sj::launch_rowsort_range(ix.off_cell.ptr, r0, r1, boff[b], off_b[k].ptr, ix.perm.ptr, out_j[k].ptr,
                                         pairs[k].ptr, ix.max_row, fused ? 64u : 0u, st, nullptr,
                                         ix.opts.sort_output != 0);
        }
        SJ_HIP(hipEventRecord(ev[k], st));
        if (b >= 1) deliver(b - 1);
    }
    if (rc == 0) deliver(nb - 1);
    if (nsets > 1) {
        // the caller's stream continues after the second stream's batches
        SJ_HIP(hipEventRecord(ev[2], ss[1]));
        SJ_HIP(hipStreamWaitEvent(s, ev[2], 0));
    }
    check_overflow(ix, s);
    ix.stats.batches = nb;
    ix.stats.ms_fill = now_ms() - t0;
    note_run(stats_of(ix));
    return rc;
}

// Batched delivery in consecutive ranges of i (the convenience call's
// pinned-host result, whose batches are concatenated in place): each batch's
// query points scan all adjacent cells with the per-point kernel and write
// only their own rows; double-buffered like the cell-ordered runs.
int join_batched_rows(sj_index &ix, sj_run_cb cb, void *user, hipStream_t s) {
    const double t0 = now_ms();
    const uint64_t n = ix.n, P = ix.pairs;
    ix.hitbits.release();  // ranges of i test again; the bits serve only the whole fill
    ix.bits_uni = -1;
    if (n == 0 || P == 0) {
        ix.stats.batches = 0;
        return 0;
    }
    const uint64_t cap = ix.opts.batch_capacity_pairs ? ix.opts.batch_capacity_pairs : P;
    if (ix.max_row > cap)
        throw Error(SJ_ECAPACITY, "batch capacity is smaller than the longest result row (" +
                                      std::to_string(ix.max_row) + " pairs)");
    const uint64_t per = cap > ix.max_row ? cap - ix.max_row : 1;
    uint64_t nb64 = std::max<uint64_t>(ix.opts.min_batches, (P + per - 1) / per);
    if (cap >= P && ix.opts.min_batches <= 1) nb64 = 1;
    nb64 = std::min<uint64_t>(nb64, n);
    const uint32_t nb = static_cast<uint32_t>(nb64);
    std::vector<uint64_t> rows(nb + 1);
    {
        DevBuf<uint64_t> drows(nb + 1);
        sj::launch_batch_bounds(ix.off_orig.ptr, n, P, nb, drows.ptr, s);
        SJ_HIP(hipMemcpyAsync(rows.data(), drows.ptr, (nb + 1) * sizeof(uint64_t),
                              hipMemcpyDeviceToHost, s));
        SJ_HIP(hipStreamSynchronize(s));
    }
    std::vector<uint64_t> offs(nb + 1);
    for (uint32_t b = 0; b <= nb; ++b)
        SJ_HIP(hipMemcpyAsync(&offs[b], ix.off_orig.ptr + rows[b], sizeof(uint64_t),
                              hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    uint64_t maxbatch = 0;
    for (uint32_t b = 0; b < nb; ++b) maxbatch = std::max(maxbatch, offs[b + 1] - offs[b]);
    const bool uni_fill = (nb == 1) && choose_unicomp_fill(ix);
    ix.stats.fill_unicomp = uni_fill ? 1u : 0u;
    const int nsets = nb > 1 ? 2 : 1;
    DevBuf<uint32_t> out_j[2], pairs[2];
    for (int k = 0; k < nsets; ++k) {
        out_j[k].reset(std::max<uint64_t>(1, maxbatch));
        pairs[k].reset(2 * std::max<uint64_t>(1, maxbatch));
    }
    hipEvent_t ev[2];
    SJ_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    SJ_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            (void)hipEventDestroy(e[0]);
            (void)hipEventDestroy(e[1]);
        }
    } evg{ev};
    Scratch sc;
    int rc = 0;
    uint32_t delivered = 0;
    auto deliver = [&](uint32_t b) {
        const int k = b & 1;
        SJ_HIP(hipEventSynchronize(ev[k]));
        if (rc == 0 && cb)
            rc = cb(user, pairs[k].ptr, offs[b + 1] - offs[b], b, rows[b], rows[b + 1]);
        ++delivered;
    };
    ix.overflow.ensure(1);
    sj::launch_fill_u32(ix.overflow.ptr, 1, 0u, s);
    ix.overflow_clear = false;
    for (uint32_t b = 0; b < nb && rc == 0; ++b) {
        const int k = b & 1;
        if (offs[b + 1] > offs[b])
            fill_rows(ix, rows[b], rows[b + 1], offs[b], offs[b + 1] - offs[b], uni_fill,
                      out_j[k].ptr, pairs[k].ptr, sc, s);
        SJ_HIP(hipEventRecord(ev[k], s));
        if (b >= 1) deliver(b - 1);
    }
    if (rc == 0) deliver(nb - 1);
    check_overflow(ix, s);
    ix.stats.batches = nb;
    ix.stats.ms_fill = now_ms() - t0;
    note_run(stats_of(ix));
    return rc;
}

// ---------------------------------------------------------------- brute force
// Candidate ranges per query row: enough workgroups (query blocks x ranges)
// to fill the chip, each range a whole number of LDS tiles.
struct BrutePlan {
    uint32_t splits;
    uint64_t span;
};

BrutePlan brute_plan(uint64_t n, uint32_t d) {
    constexpr uint64_t kTargetBlocks = 1024;
    const uint64_t rows_blk = sj::brute_rows_per_block(d);
    const uint64_t tile = sj::brute_tile();
    const uint64_t qblocks = (n + rows_blk - 1) / rows_blk;
    const uint64_t tiles = (n + tile - 1) / tile;
    uint64_t S = qblocks ? (kTargetBlocks + qblocks - 1) / qblocks : 1;
    S = std::max<uint64_t>(1, std::min<uint64_t>(S, tiles));
    const uint64_t span = ((n + S - 1) / S + tile - 1) / tile * tile;
    BrutePlan p;
    p.span = std::max<uint64_t>(span, tile);
    p.splits = static_cast<uint32_t>(n ? (n + p.span - 1) / p.span : 1);
    return p;
}

// Count pass, offsets and (when pairs_dev is set and holds the result) fill
// pass of the all-pairs join over device points dp. count, off and part
// hold n * splits, n * splits + 1 and scan_partials(n * splits) entries;
// flag is one word; readback is a host word for P (page-locked or not).
// Allocates nothing.
void brute_join(const double *dp, uint64_t n, uint32_t d, double eps, const BrutePlan &pl, uint32_t *count,
                uint64_t *off, uint64_t *part, uint32_t *flag, uint64_t *readback, uint32_t *pairs_dev,
                uint64_t cap, hipStream_t s, uint64_t *P_out) {
    sj::BruteArgs a{};
    a.pts = dp;
    a.n = n;
    a.splits = pl.splits;
    a.span = pl.span;
    a.eps2 = eps * eps;
    a.count = count;
    const double t0 = now_ms();
    sj::launch_brute(a, d, sj::kCount, s);
    const size_t cells = static_cast<size_t>(n) * pl.splits;
    sj::scan_exclusive_u32_to_u64_ws(count, off, cells, part, s);
    sj::launch_fill_u32(flag, 1, 0u, s);
    SJ_HIP(hipMemcpyAsync(readback, off + cells, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    const uint64_t P = *readback;
    if (P_out) *P_out = P;
    sj_stats st{};
    st.n = n;
    st.d = d;
    st.eps = eps;
    st.precision_used = SJ_FP64;
    st.evals = n * n;
    st.pairs = P;
    st.ms_count = now_ms() - t0;
    note_run(st);
    if (!pairs_dev || P == 0) return;
    if (cap < P)
        throw Error(SJ_ECAPACITY, "output buffer holds " + std::to_string(cap) + " pairs, the result has " +
                                      std::to_string(P));
    const double t1 = now_ms();
    a.off = off;
    a.pairs = reinterpret_cast<uint2 *>(pairs_dev);
    a.overflow = flag;
    sj::launch_brute(a, d, sj::kFill, s);
    uint32_t *fw = reinterpret_cast<uint32_t *>(readback);
    SJ_HIP(hipMemcpyAsync(fw, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    if (*fw) throw Error(SJ_EDEVICE, "internal: the brute-force fill disagreed with its count");
    st.ms_fill = now_ms() - t1;
    st.batches = 1;
    note_run(st);
}

// The array's device address on the current device, looked up once per
// device (in host code the array's name is only a stand-in, not a device
// address).
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
unsigned char *g_scratch_addr[kMaxDevices] = {};

unsigned char *scratch_on_current_device() {
    int dev = -1;
    SJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(SJ_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        SJ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(sj::scratch)));
        if (!p) throw Error(SJ_EDEVICE, "scratch address lookup returned NULL");
        g_scratch_addr[dev] = static_cast<unsigned char *>(p);
    }
    return g_scratch_addr[dev];
}

void validate_brute_args(const double *pts, uint64_t n, uint32_t d, double eps) {
    if (d < 1 || d > static_cast<uint32_t>(sj::kMaxDim)) throw Error(SJ_EINVAL, "d must be in [1, 8]");
    if (!(eps > 0.0) || !std::isfinite(eps)) throw Error(SJ_EINVAL, "eps must be finite and > 0");
    if (n >= 0xffffffffULL) throw Error(SJ_EINVAL, "n must be below 2^32 - 1");
    if (n > 0 && !pts) throw Error(SJ_EINVAL, "pts is NULL");
}

// ---------------------------------------------------------------- two-set join
sj::RsArgs rs_args(sj_index &ix) {
    sj::RsArgs a{};
    a.R = ix.rs.R;
    a.nr = ix.rs.nr;
    a.qperm = ix.rs.qperm.ptr;
    a.X = ix.X.ptr;
    a.ns = ix.n;
    a.perm = ix.perm.ptr;
    a.B = ix.B.ptr;
    a.starts = ix.starts.ptr;
    a.ncells = static_cast<uint32_t>(ix.ncells);
    a.g = ix.grid;
    a.eps2 = ix.eps * ix.eps;
    return a;
}

// Count pass of R x S on the per-query kernel (SJ_JOIN_KERNEL=ranges):
// queries in S's cell order (the index's cell key and radix sort), so that a
// wave's queries share candidate cells; row offsets by query row (output)
// and by probe position (fill layout); P and the longest row.
void rs_count_perquery(sj_index &ix, const double *rp, uint64_t nr, hipStream_t s) {
    auto &st = ix.rs;
    st.qperm.ensure(nr);
    {
        DevBuf<uint32_t> qperm_alt(nr);
        DevBuf<uint64_t> k64(nr), k64_alt(nr);
        sj::GridParams g = ix.grid;
        g.sub_shift = 0;  // plain cell ids
        if (ix.key_bits <= 32) {
            uint32_t *k = reinterpret_cast<uint32_t *>(k64.ptr), *k2 = reinterpret_cast<uint32_t *>(k64_alt.ptr);
            sj::launch_cell_keys_u32(rp, nr, g, k, st.qperm.ptr, s);
            if (sj::radix_sort_u32(k, st.qperm.ptr, k2, qperm_alt.ptr, nr, ix.key_bits, s))
                std::swap(st.qperm, qperm_alt);
        } else {
            sj::launch_cell_keys_u64(rp, nr, g, k64.ptr, st.qperm.ptr, s);
            if (sj::radix_sort_u64(k64.ptr, st.qperm.ptr, k64_alt.ptr, qperm_alt.ptr, nr, ix.key_bits, s))
                std::swap(st.qperm, qperm_alt);
        }
    }
    sj::RsArgs a = rs_args(ix);
    st.cnt.ensure(nr);
    st.cnt_k.ensure(nr);
    st.words.ensure(2);
    st.off.ensure(nr + 1);
    st.off_k.ensure(nr + 1);
    a.count = st.cnt.ptr;
    a.count_k = st.cnt_k.ptr;
    sj::launch_join_rs(a, 0, s);
    sj::scan_exclusive_u32_to_u64_x2(st.cnt.ptr, st.off.ptr, st.cnt_k.ptr, st.off_k.ptr, nr, s);
    sj::launch_fill_u32(st.words.ptr, 2, 0u, s);
    sj::launch_rs_max(st.cnt.ptr, nr, st.words.ptr, s);
    sj::HostStage hs;
    SJ_HIP(hipMemcpyAsync(hs.p, st.off.ptr + nr, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipMemcpyAsync(hs.as<uint32_t>() + 2, st.words.ptr, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    st.P = *hs.as<uint64_t>();
    st.max_len = hs.as<uint32_t>()[2];
}

// Fill pass of the per-query kernel: neighbour ids per query in probe
// order, unsorted, then each row sorted and written as (i, j) pairs at its
// offset in R's order.
void rs_fill_perquery(sj_index &ix, uint32_t *pairs_dev, hipStream_t s) {
    auto &st = ix.rs;
    const uint64_t P = st.P;
    sj::RsArgs a = rs_args(ix);
    DevBuf<uint32_t> out_j(P);
    a.off = st.off_k.ptr;
    a.out_j = out_j.ptr;
    a.out_cap = P;
    a.overflow = st.words.ptr + 1;
    sj::launch_join_rs(a, 1, s);
    sj::launch_rowsort_cells(st.off_k.ptr, st.off.ptr, st.qperm.ptr, st.nr, out_j.ptr, pairs_dev, st.max_len, s);
    sj::HostStage hs;
    SJ_HIP(hipMemcpyAsync(hs.p, st.words.ptr + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    if (*hs.as<uint32_t>()) throw Error(SJ_EDEVICE, "internal: the two-set fill disagreed with its count");
}

// Tile arguments of the two-set join: S's cells, masks and candidate cells,
// the queries' chunks, segments and dimension-0 cells.
sj::TileArgs rs_tile_args(sj_index &ix) {
    auto &st = ix.rs;
    sj::TileArgs t = tile_args(ix);
    t.coords = st.coords.ptr;  // chunk geometry (the segments' search)
    t.cxq = st.cxq.ptr;
    t.chunks = st.chunks;
    t.nchunks = st.nchunks;
    t.nchunks_dev = st.nchunks_dev.ptr;
    t.rows_per_chunk = st.rows_per_chunk;
    t.segs = st.segs.ptr;
    return t;
}

sj::JoinArgs rs_join_args(sj_index &ix) {
    auto &st = ix.rs;
    sj::JoinArgs a = base_args(ix, 0);
    a.Y = nullptr;  // FP64 only
    a.Xq = st.Xq.ptr;
    a.Yq = nullptr;
    a.nqs = static_cast<uint32_t>(st.nr);  // the SoA's stride (all rows gathered; the first nv are joined)
    a.permq = st.qperm.ptr;
    a.cell_of = st.cell_of.ptr;
    a.own_cnt = st.own_cnt.ptr;
    a.in_cnt = nullptr;
    a.evals = st.counters.ptr;
    a.band_rechecks = st.counters.ptr + sj::kCounterSlots * sj::kCounterStride;
    return a;
}

// Count pass of R x S on the grid-row tiled kernel. R's rows take their
// cells in S's grid and are sorted by cell (rows with no adjacent cell
// last, left out); the sorted queries get their own cells, grid-row chunks
// of at most 64 and, per chunk, the 3^(d-1) candidate segments of S's cell
// order. The full search then counts each query's neighbours; row lengths
// and offsets follow as in the self-join.
void rs_count_tiled(sj_index &ix, const double *rp, uint64_t nr, hipStream_t s) {
    auto &st = ix.rs;
    const uint32_t d = ix.d;
    const int bits = ix.key_bits + 1;  // one more: the key of the rows left out
    st.qperm.ensure(nr);
    st.words.ensure(2);  // [0] rows left out, [1] the fill's overflow flag
    sj::launch_fill_u32(st.words.ptr, 2, 0u, s);
    DevBuf<uint32_t> qalt(nr);
    DevBuf<uint64_t> k64(nr), k64_alt(nr);
    const bool k32 = bits <= 32;
    if (k32) {
        uint32_t *k = reinterpret_cast<uint32_t *>(k64.ptr), *k2 = reinterpret_cast<uint32_t *>(k64_alt.ptr);
        sj::launch_rs_query_keys_u32(rp, nr, ix.grid, ix.key_bits, k, st.qperm.ptr, st.words.ptr, s);
        if (sj::radix_sort_u32(k, st.qperm.ptr, k2, qalt.ptr, nr, bits, s)) {
            std::swap(k64, k64_alt);
            std::swap(st.qperm, qalt);
        }
    } else {
        sj::launch_rs_query_keys_u64(rp, nr, ix.grid, ix.key_bits, k64.ptr, st.qperm.ptr, st.words.ptr, s);
        if (sj::radix_sort_u64(k64.ptr, st.qperm.ptr, k64_alt.ptr, qalt.ptr, nr, bits, s)) {
            std::swap(k64, k64_alt);
            std::swap(st.qperm, qalt);
        }
    }
    // cells of all rows (those left out form the last cell, if any), their
    // coordinates and the cell-ordered SoA, before the one readback of the
    // counts they depend on
    st.cell_of.ensure(nr);
    st.B.ensure(nr);
    st.starts.ensure(nr + 1);
    st.coords.ensure(nr * d);
    st.Xq.ensure(nr * d);
    st.cxq.ensure(nr);
    if (k32)
        sj::build_cells<uint32_t>(reinterpret_cast<uint32_t *>(k64.ptr), nr, 0, st.cell_of.ptr, st.B.ptr,
                                  st.starts.ptr, s);
    else
        sj::build_cells<uint64_t>(k64.ptr, nr, 0, st.cell_of.ptr, st.B.ptr, st.starts.ptr, s);
    DevBuf<uint32_t> max_pts(1);
    sj::launch_cell_coords_masks(st.B.ptr, st.starts.ptr, nr, st.cell_of.ptr + (nr - 1), ix.grid, st.coords.ptr,
                                 nullptr, sj::MaskOffsets{}, 0, max_pts.ptr, s);
    sj::launch_gather_soa(rp, st.qperm.ptr, nr, d, st.Xq.ptr, ix.grid, st.cxq.ptr, s);
    st.len_orig.ensure(nr);
    st.len_cell.ensure(nr);
    st.off_orig.ensure(nr + 1);
    st.off_cell.ensure(nr + 1);
    const size_t nctr = 2 * sj::kCounterSlots * sj::kCounterStride;
    st.counters.ensure(nctr);
    st.row_stats.ensure(sj::kRowStatWords);
    st.nchunks_dev.ensure(1);
    st.summary.ensure(8);
    sj::ZeroSpans z{};
    z.add(st.len_orig.ptr, nr);
    z.add(st.len_cell.ptr, nr);
    z.add(st.counters.ptr, 2 * nctr);
    sj::launch_zero_spans(z, s);
    sj::HostStage hs;
    SJ_HIP(hipMemcpyAsync(hs.p, st.words.ptr, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipMemcpyAsync(hs.as<uint32_t>() + 1, st.cell_of.ptr + (nr - 1), sizeof(uint32_t),
                          hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    const uint32_t nleft = hs.as<uint32_t>()[0];
    const uint32_t nv = static_cast<uint32_t>(nr) - nleft;
    const uint32_t ncq = hs.as<uint32_t>()[1] + 1 - (nleft ? 1u : 0u);
    st.nv = nv;
    if (nv > 0) {
        // grid-row chunks of the queries and their candidate segments in S
        uint64_t rows_bound = 1;
        for (uint32_t j = 1; j < d; ++j)
            rows_bound = ix.grid.dims[j] > (UINT64_MAX / 2) / rows_bound ? UINT64_MAX / 2 : rows_bound * ix.grid.dims[j];
        st.nchunks = sj::build_chunks(st.coords.ptr, st.starts.ptr, ncq, nv, d, rows_bound, &st.chunks,
                                      &st.chunks_cap, st.nchunks_dev.ptr, s);
        uint32_t r3 = 1;
        for (uint32_t j = 1; j < d; ++j) r3 *= 3;
        st.rows_per_chunk = r3;
        st.segs.reset(static_cast<size_t>(st.nchunks) * r3);
        sj::build_chunk_segments(rs_tile_args(ix), st.cell_of.ptr, ix.starts.ptr, d, st.segs.ptr, s);
        // count
        st.own_cnt.ensure(nv);
        sj::launch_join_tiled(rs_join_args(ix), rs_tile_args(ix), d, 0, sj::kCount, 0, s);
        sj::launch_row_lengths(st.own_cnt.ptr, nullptr, st.qperm.ptr, nv, st.len_orig.ptr, st.len_cell.ptr,
                               st.row_stats.ptr, s);
    } else {
        st.nchunks = 0;
        sj::launch_fill_u32(st.nchunks_dev.ptr, 1, 0u, s);
        sj::launch_fill_u32(st.row_stats.ptr, sj::kRowStatWords, 0u, s);
    }
    sj::scan_exclusive_u32_to_u64_x2(st.len_orig.ptr, st.off_orig.ptr, st.len_cell.ptr, st.off_cell.ptr, nr, s);
    sj::launch_count_summary(st.off_orig.ptr, nr, st.row_stats.ptr, st.counters.ptr, st.nchunks_dev.ptr,
                             st.summary.ptr, st.words.ptr + 1, s);
    SJ_HIP(hipMemcpyAsync(hs.p, st.summary.ptr, 8 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    const uint64_t *sm = hs.as<uint64_t>();
    st.P = sm[0];
    st.max_len = static_cast<uint32_t>(sm[1]);
    st.evals = sm[2];
    st.stats.chunks = sm[4];
    for (int k = 0; k < 3; ++k) st.rows_longer[k] = sm[5 + k];
}

// Fill pass of the tiled kernel: in 1..3-D with the row sort fused (rows
// that fit the LDS slot are sorted there and written as (i, j) pairs at
// their offset in R's order, longer ones go through out_j to the row-sort
// kernels), from 4-D on into out_j in cell order, then every row sorted.
void rs_fill_tiled(sj_index &ix, uint32_t *pairs_dev, hipStream_t s) {
    auto &st = ix.rs;
    const uint64_t P = st.P;
    DevBuf<uint32_t> out_j(P);
    sj::JoinArgs a = rs_join_args(ix);
    a.out_j = out_j.ptr;
    a.out_base = 0;
    a.out_cap = P;
    a.overflow = st.words.ptr + 1;  // cleared by the count summary
    a.offc = st.off_cell.ptr;
    const bool fused = use_fused_sort(ix.d);
    uint32_t ns = 0;
    if (fused) {
        // the smallest LDS slot that at most 5% of the rows exceed
        const double lim = 0.05 * static_cast<double>(st.nv);
        ns = static_cast<double>(st.rows_longer[0]) <= lim ? 16u
             : (static_cast<double>(st.rows_longer[1]) <= lim ? 24u : 32u);
        a.off_orig = st.off_orig.ptr;
        a.pairs = reinterpret_cast<uint2 *>(pairs_dev);
    }
    sj::launch_join_tiled(a, rs_tile_args(ix), ix.d, 0, sj::kFill, 0, s, ns);
    if (fused)
        sj::launch_rowsort_long(st.off_cell.ptr, st.off_orig.ptr, st.qperm.ptr, st.nv, out_j.ptr, pairs_dev,
                                st.max_len, 64, s);
    else
        sj::launch_rowsort_cells(st.off_cell.ptr, st.off_orig.ptr, st.qperm.ptr, st.nv, out_j.ptr, pairs_dev,
                                 st.max_len, s);
    sj::HostStage hs;
    SJ_HIP(hipMemcpyAsync(hs.p, st.words.ptr + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SJ_HIP(hipStreamSynchronize(s));
    if (*hs.as<uint32_t>()) throw Error(SJ_EDEVICE, "internal: the two-set fill disagreed with its count");
}

// Count pass of R x S; the state is kept in ix.rs for rs_fill.
void rs_count(sj_index &ix, const double *R, uint64_t nr, int r_on_device, hipStream_t s) {
    auto &st = ix.rs;
    st.counted = false;
    st.P = 0;
    st.nr = nr;
    st.nv = 0;
    st.evals = 0;
    if (nr && !R) throw Error(SJ_EINVAL, "R is NULL");
    if (nr >= 0x7fffffffULL) throw Error(SJ_EINVAL, "too many query rows");
    if (nr == 0 || ix.n == 0) {
        st.counted = true;
        return;
    }
    const double *rp = R;
    if (!r_on_device) {
        st.staged.ensure(nr * ix.d);
        SJ_HIP(hipMemcpyAsync(st.staged.ptr, R, nr * ix.d * sizeof(double), hipMemcpyHostToDevice, s));
        rp = st.staged.ptr;
    }
    st.R = rp;
    st.tiled = use_tiled();
    const double t0 = now_ms();
    st.stats = sj_stats{};
    if (st.tiled)
        rs_count_tiled(ix, rp, nr, s);
    else
        rs_count_perquery(ix, rp, nr, s);
    st.counted = true;
    // statistics of the run: the queries as n, S's grid
    sj_stats &r = st.stats;
    r.n = nr;
    r.d = ix.d;
    r.key_bits = static_cast<uint32_t>(ix.key_bits);
    r.cells = ix.ncells;
    for (uint32_t j = 0; j < ix.d; ++j) r.grid_dims[j] = ix.grid.dims[j];
    r.eps = ix.eps;
    r.cell_width = ix.grid.w;
    r.max_cell_points = ix.max_cell;
    r.precision_used = SJ_FP64;
    r.evals = st.evals;  // counted by the tiled kernel only
    r.pairs = st.P;
    r.max_row_pairs = st.max_len;
    r.ms_count = now_ms() - t0;
    note_run(r);
}

void rs_fill(sj_index &ix, uint32_t *pairs_dev, uint64_t cap, hipStream_t s) {
    auto &st = ix.rs;
    if (st.P == 0) return;
    if (!pairs_dev) throw Error(SJ_EINVAL, "pairs_dev is NULL");
    if (cap < st.P)
        throw Error(SJ_ECAPACITY, "output buffer holds " + std::to_string(cap) + " pairs, the result has " +
                                      std::to_string(st.P));
    const double t0 = now_ms();
    if (st.tiled)
        rs_fill_tiled(ix, pairs_dev, s);
    else
        rs_fill_perquery(ix, pairs_dev, s);
    st.stats.ms_fill = now_ms() - t0;
    st.stats.batches = 1;
    note_run(st.stats);
}

}  // namespace

// ====================================================================== ABI
extern "C" {

void sj_default_opts(sj_join_opts *o) {
    if (!o) return;
    o->unicomp = 1;
    o->precision = SJ_FP64;
    o->batch_capacity_pairs = 0;
    o->min_batches = 1;
    o->sort_output = 1;
}

const char *sj_last_error(void) { return t_error.c_str(); }

const char *sj_version(void) { return "sj 0.1 (gfx950)"; }

int sj_build_index(const double *pts, uint64_t n, uint32_t d, double eps, int pts_on_device,
                   void *stream, sj_index **out) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        if (!out) throw Error(SJ_EINVAL, "out is NULL");
        *out = nullptr;
        validate_points_args(pts, n, d, eps);
        auto *ix = new sj_index;
        ix->n = n;
        ix->d = d;
        ix->eps = eps;
        ix->grid.d = d;
        try {
            if (n > 0) build(*ix, pts, pts_on_device, s);
        } catch (...) {
            (void)hipStreamSynchronize(s);
            delete ix;
            throw;
        }
        ix->stats.n = n;
        ix->stats.d = d;
        ix->stats.eps = eps;
        *out = ix;
    });
}

void sj_destroy_index(sj_index *idx) {
    if (!idx) return;
    (void)guarded(nullptr, [&] { delete idx; });
}

int sj_join_count(sj_index *idx, const sj_join_opts *opts, void *stream, uint64_t *total_pairs) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        if (!idx) throw Error(SJ_EINVAL, "index is NULL");
        validate_opts(opts);
        join_count(*idx, resolve_opts(opts), s);
        if (total_pairs) *total_pairs = idx->pairs;
    });
}

int sj_join_fill(sj_index *idx, uint32_t *pairs_dev, uint64_t capacity_pairs, void *stream) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        if (!idx) throw Error(SJ_EINVAL, "index is NULL");
        if (!idx->counted) throw Error(SJ_ESTATE, "sj_join_fill needs a preceding sj_join_count");
        if (capacity_pairs < idx->pairs)
            throw Error(SJ_ECAPACITY, "output buffer holds " + std::to_string(capacity_pairs) +
                                          " pairs, the result has " + std::to_string(idx->pairs));
        if (idx->pairs && !pairs_dev) throw Error(SJ_EINVAL, "pairs_dev is NULL");
        join_fill_all(*idx, pairs_dev, s);
    });
}

int sj_join_fill_csr(sj_index *idx, uint64_t *row_off_dev, uint32_t *cols_dev, uint64_t capacity,
                     void *stream) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        if (!idx) throw Error(SJ_EINVAL, "index is NULL");
        if (!idx->counted) throw Error(SJ_ESTATE, "sj_join_fill_csr needs a preceding sj_join_count");
        if (capacity < idx->pairs)
            throw Error(SJ_ECAPACITY, "column buffer holds " + std::to_string(capacity) +
                                          " entries, the result has " + std::to_string(idx->pairs));
        if (!row_off_dev) throw Error(SJ_EINVAL, "row_off_dev is NULL");
        if (idx->pairs && !cols_dev) throw Error(SJ_EINVAL, "cols_dev is NULL");
        if (idx->n == 0) {
            sj::launch_fill_u64(row_off_dev, 1, 0, s);
            return;
        }
        SJ_HIP(hipMemcpyAsync(row_off_dev, idx->off_orig.ptr, (idx->n + 1) * sizeof(uint64_t),
                              hipMemcpyDeviceToDevice, s));
        join_fill_all(*idx, nullptr, s, cols_dev);
    });
}

int sj_join_rs_count(sj_index *idx, const double *R, uint64_t nr, int r_on_device, void *stream,
                     uint64_t *total_pairs) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        if (!idx) throw Error(SJ_EINVAL, "index is NULL");
        rs_count(*idx, R, nr, r_on_device, s);
        if (total_pairs) *total_pairs = idx->rs.P;
    });
}

int sj_join_rs_fill(sj_index *idx, uint32_t *pairs_dev, uint64_t capacity_pairs, void *stream) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        if (!idx) throw Error(SJ_EINVAL, "index is NULL");
        if (!idx->rs.counted) throw Error(SJ_ESTATE, "sj_join_rs_fill needs a preceding sj_join_rs_count");
        rs_fill(*idx, pairs_dev, capacity_pairs, s);
    });
}

int sj_join_rs(sj_index *idx, const double *R, uint64_t nr, int r_on_device, uint32_t *pairs_dev,
               uint64_t capacity_pairs, void *stream, uint64_t *total_pairs) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        if (!idx) throw Error(SJ_EINVAL, "index is NULL");
        if (total_pairs) *total_pairs = 0;
        rs_count(*idx, R, nr, r_on_device, s);
        if (total_pairs) *total_pairs = idx->rs.P;
        if (pairs_dev) rs_fill(*idx, pairs_dev, capacity_pairs, s);
        idx->rs.counted = false;  // the one-call form keeps no state
    });
}

int sj_bruteforce(const double *pts, uint64_t n, uint32_t d, double eps, int pts_on_device,
                  uint32_t *pairs_dev, uint64_t capacity_pairs, void *stream, uint64_t *total_pairs) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        validate_brute_args(pts, n, d, eps);
        if (total_pairs) *total_pairs = 0;
        if (n == 0) return;
        DevBuf<double> staged;
        const double *dp = pts;
        if (!pts_on_device) {
            staged.reset(n * d);
            SJ_HIP(hipMemcpyAsync(staged.ptr, pts, n * d * sizeof(double), hipMemcpyHostToDevice, s));
            dp = staged.ptr;
        }
        const BrutePlan pl = brute_plan(n, d);
        const size_t cells = static_cast<size_t>(n) * pl.splits;
        DevBuf<uint32_t> count(cells), flag(1);
        DevBuf<uint64_t> off(cells + 1), part(sj::scan_partials(cells));
        sj::HostStage hs;
        brute_join(dp, n, d, eps, pl, count.ptr, off.ptr, part.ptr, flag.ptr, hs.as<uint64_t>(), pairs_dev,
                   capacity_pairs, s, total_pairs);
    });
}

int sj_dbscan_csr(const uint64_t *row_off_dev, const uint32_t *cols_dev, uint64_t n, uint32_t min_pts,
                  int32_t *labels_dev, void *stream, uint64_t *nclusters) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        if (nclusters) *nclusters = 0;
        if (n == 0) return;
        if (!row_off_dev || !cols_dev || !labels_dev) throw Error(SJ_EINVAL, "NULL argument");
        if (min_pts == 0) throw Error(SJ_EINVAL, "min_pts must be at least 1");
        if (n > 0x7fffffffULL) throw Error(SJ_EINVAL, "n must be below 2^31");
        DevBuf<unsigned long long> cnt(1);
        sj::launch_fill_u64(reinterpret_cast<uint64_t *>(cnt.ptr), 1, 0, s);
        sj::launch_dbscan(row_off_dev, cols_dev, n, min_pts, labels_dev, cnt.ptr, s);
        sj::HostStage hs;
        SJ_HIP(hipMemcpyAsync(hs.p, cnt.ptr, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        SJ_HIP(hipStreamSynchronize(s));
        if (nclusters) *nclusters = *hs.as<uint64_t>();
    });
}

int sj_dbscan(const double *pts, uint64_t n, uint32_t d, double eps, uint32_t min_pts, int pts_on_device,
              int32_t *labels_dev, void *stream, uint64_t *nclusters) {
    hipStream_t s = as_stream(stream);
    if (nclusters) *nclusters = 0;
    if (n >= 0x7fffffffULL) {
        set_error("n must be below 2^31 - 1");
        return SJ_EINVAL;
    }
    if (min_pts == 0) {
        set_error("min_pts must be at least 1");
        return SJ_EINVAL;
    }
    if (n > 0 && !labels_dev) {
        set_error("labels_dev is NULL");
        return SJ_EINVAL;
    }
    sj_index *ix = nullptr;
    int rc = sj_build_index(pts, n, d, eps, pts_on_device, stream, &ix);
    if (rc != SJ_OK) return rc;
    rc = guarded(s, [&] {
        if (n == 0) return;
        sj_join_opts o;
        sj_default_opts(&o);
        o.sort_output = 0;  // the clustering needs each row's members, not their order
        join_count(*ix, o, s);
        DevBuf<uint64_t> off(n + 1);
        DevBuf<uint32_t> cols(std::max<uint64_t>(1, ix->pairs));
        SJ_HIP(hipMemcpyAsync(off.ptr, ix->off_orig.ptr, (n + 1) * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        join_fill_all(*ix, nullptr, s, cols.ptr);
        DevBuf<unsigned long long> cnt(1);
        sj::launch_fill_u64(reinterpret_cast<uint64_t *>(cnt.ptr), 1, 0, s);
        sj::launch_dbscan(off.ptr, cols.ptr, n, min_pts, labels_dev, cnt.ptr, s);
        sj::HostStage hs;
        SJ_HIP(hipMemcpyAsync(hs.p, cnt.ptr, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        SJ_HIP(hipStreamSynchronize(s));
        if (nclusters) *nclusters = *hs.as<uint64_t>();
    });
    sj_destroy_index(ix);
    return rc;
}

int sj_bruteforce_noalloc(const double *pts_dev, uint64_t n, uint32_t d, double eps, uint32_t *pairs_dev,
                          uint64_t capacity_pairs, void *stream, uint64_t *total_pairs) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        validate_brute_args(pts_dev, n, d, eps);
        if (total_pairs) *total_pairs = 0;
        if (n == 0) return;
        const BrutePlan pl = brute_plan(n, d);
        const size_t cells = static_cast<size_t>(n) * pl.splits;
        if (cells > sj::kNoAllocCells || sj::scan_partials(cells) > sj::kNaPartWords)
            throw Error(SJ_EINVAL, "sj_bruteforce_noalloc takes at most " + std::to_string(sj::kNoAllocCells) +
                                       " points (" + std::to_string(n) + " given)");
        unsigned char *base = scratch_on_current_device();
        uint64_t readback = 0;  // pageable host word: no pinned staging block
        brute_join(pts_dev, n, d, eps, pl, reinterpret_cast<uint32_t *>(base + sj::kNaCountOff),
                   reinterpret_cast<uint64_t *>(base + sj::kNaOffOff),
                   reinterpret_cast<uint64_t *>(base + sj::kNaPartOff),
                   reinterpret_cast<uint32_t *>(base + sj::kNaFlagOff), &readback, pairs_dev, capacity_pairs, s,
                   total_pairs);
    });
}

int sj_selfjoin_index(sj_index *idx, const sj_join_opts *opts, sj_run_cb cb, void *user,
                      void *stream, uint64_t *total_pairs) {
    hipStream_t s = as_stream(stream);
    int cb_rc = 0;
    const int rc = guarded(s, [&] {
        if (!idx) throw Error(SJ_EINVAL, "index is NULL");
        validate_opts(opts);
        join_count(*idx, resolve_opts(opts), s);
        if (total_pairs) *total_pairs = idx->pairs;
        cb_rc = join_batched_cells(*idx, cb, user, s);
    });
    if (rc != SJ_OK) return rc;
    if (cb_rc != 0) set_error("the batch callback stopped the join");
    return cb_rc;
}

int sj_selfjoin(const double *pts, uint64_t n, uint32_t d, double eps, const sj_join_opts *opts,
                int pts_on_device, int out_on_device, void *stream, uint32_t **pairs_out,
                uint64_t *npairs) {
    hipStream_t s = as_stream(stream);
    if (!pairs_out || !npairs) {
        set_error("pairs_out and npairs must not be NULL");
        return SJ_EINVAL;
    }
    *pairs_out = nullptr;
    *npairs = 0;
    sj_index *ix = nullptr;
    int rc = sj_build_index(pts, n, d, eps, pts_on_device, stream, &ix);
    if (rc != SJ_OK) return rc;
    uint32_t *buf = nullptr;
    rc = guarded(s, [&] {
        validate_opts(opts);
        const sj_join_opts o = resolve_opts(opts);
        join_count(*ix, o, s);
        const uint64_t P = ix->pairs;
        if (P == 0) return;
        if (out_on_device) {
            SJ_HIP(hipMalloc(reinterpret_cast<void **>(&buf), P * 2 * sizeof(uint32_t)));
            {
                std::lock_guard<std::mutex> lk(g_out_mu);
                g_out_bufs[buf] = true;
            }
            // the whole result is in device memory anyway: one fill into it
            join_fill_all(*ix, buf, s);
        } else {
            SJ_HIP(hipHostMalloc(reinterpret_cast<void **>(&buf), P * 2 * sizeof(uint32_t),
                                 hipHostMallocDefault));
            {
                std::lock_guard<std::mutex> lk(g_out_mu);
                g_out_bufs[buf] = false;
            }
            hipStream_t cs = nullptr;
            SJ_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            struct Ctx { uint32_t *dst; hipStream_t cs; uint64_t at; } ctx{buf, cs, 0};
            auto cb = [](void *u, const uint32_t *p, uint64_t np, uint32_t, uint64_t, uint64_t) -> int {
                auto *c = static_cast<Ctx *>(u);
                if (hipMemcpyAsync(c->dst + 2 * c->at, p, np * 8, hipMemcpyDeviceToHost, c->cs) != hipSuccess)
                    return SJ_EDEVICE;
                if (hipStreamSynchronize(c->cs) != hipSuccess) return SJ_EDEVICE;
                c->at += np;
                return 0;
            };
            int r = 0;
            try {
                r = join_batched_rows(*ix, cb, &ctx, s);
            } catch (...) {
                (void)hipStreamSynchronize(cs);
                (void)hipStreamDestroy(cs);
                throw;
            }
            (void)hipStreamSynchronize(cs);
            (void)hipStreamDestroy(cs);
            if (r) throw Error(r, "batched host copy failed");
        }
        *npairs = P;
        *pairs_out = buf;
    });
    if (rc != SJ_OK && buf) sj_free(buf);
    sj_destroy_index(ix);
    if (rc != SJ_OK) {
        *pairs_out = nullptr;
        *npairs = 0;
    }
    return rc;
}

void sj_free(void *ptr) {
    if (!ptr) return;
    bool on_dev = true;
    {
        std::lock_guard<std::mutex> lk(g_out_mu);
        auto it = g_out_bufs.find(ptr);
        if (it == g_out_bufs.end()) return;
        on_dev = it->second;
        g_out_bufs.erase(it);
    }
    if (on_dev)
        (void)hipFree(ptr);
    else
        (void)hipHostFree(ptr);
}

int sj_index_stats(const sj_index *idx, sj_stats *out) {
    if (!idx || !out) {
        set_error("NULL argument");
        return SJ_EINVAL;
    }
    *out = stats_of(*idx);
    return SJ_OK;
}

int sj_last_run_stats(sj_stats *out) {
    if (!out) {
        set_error("NULL argument");
        return SJ_EINVAL;
    }
    if (!t_have_last_run) {
        set_error("no join has run on this thread");
        return SJ_ESTATE;
    }
    *out = t_last_run;
    return SJ_OK;
}

int sj_index_export_size(const sj_index *idx, int what, uint64_t *bytes) {
    if (!idx || !bytes) {
        set_error("NULL argument");
        return SJ_EINVAL;
    }
    switch (what) {
        case SJ_EXPORT_CELL_IDS: *bytes = idx->ncells * sizeof(uint64_t); break;
        case SJ_EXPORT_CELL_START: *bytes = idx->n ? (idx->ncells + 1) * sizeof(uint32_t) : 0; break;
        case SJ_EXPORT_PERM: *bytes = idx->n * sizeof(uint32_t); break;
        case SJ_EXPORT_MASKS: *bytes = static_cast<uint64_t>(idx->mask_words) * sizeof(uint32_t); break;
        case SJ_EXPORT_RANGE_OFF:
            *bytes = (idx->last_ranges >= 0 && idx->ncells) ? (idx->ncells + 1) * sizeof(uint64_t) : 0;
            break;
        case SJ_EXPORT_RANGES:
            *bytes = idx->last_ranges >= 0 ? idx->ranges[idx->last_ranges].count * 2 * sizeof(uint32_t) : 0;
            break;
        case SJ_EXPORT_GRID: *bytes = (2 * sj::kMaxDim + 2) * sizeof(double); break;
        case SJ_EXPORT_ROW_OFFSETS: *bytes = (idx->counted && idx->n) ? (idx->n + 1) * sizeof(uint64_t) : 0; break;
        default: set_error("unknown export"); return SJ_EINVAL;
    }
    return SJ_OK;
}

int sj_index_export(const sj_index *idx, int what, void *host_dst, uint64_t bytes) {
    uint64_t need = 0;
    int rc = sj_index_export_size(idx, what, &need);
    if (rc != SJ_OK) return rc;
    if (bytes != need) {
        set_error("export size mismatch: expected " + std::to_string(need));
        return SJ_EINVAL;
    }
    if (need == 0) return SJ_OK;
    if (!host_dst) {
        set_error("host_dst is NULL");
        return SJ_EINVAL;
    }
    return guarded(nullptr, [&] {
        const void *src = nullptr;
        switch (what) {
            case SJ_EXPORT_CELL_IDS: src = idx->B.ptr; break;
            case SJ_EXPORT_CELL_START: src = idx->starts.ptr; break;
            case SJ_EXPORT_PERM: src = idx->perm.ptr; break;
            case SJ_EXPORT_MASKS: src = idx->masks.ptr; break;
            case SJ_EXPORT_RANGE_OFF: src = idx->ranges[idx->last_ranges].roff.ptr; break;
            case SJ_EXPORT_RANGES: src = idx->ranges[idx->last_ranges].rng; break;
            case SJ_EXPORT_ROW_OFFSETS: src = idx->off_orig.ptr; break;
            case SJ_EXPORT_GRID: {
                double g[2 * sj::kMaxDim + 2] = {};
                for (uint32_t j = 0; j < idx->d; ++j) {
                    g[j] = idx->grid.gmin[j];
                    g[sj::kMaxDim + j] = static_cast<double>(idx->grid.dims[j]);
                }
                g[2 * sj::kMaxDim] = idx->grid.w;
                g[2 * sj::kMaxDim + 1] = static_cast<double>(1u << idx->grid.sub_shift);
                std::memcpy(host_dst, g, sizeof(g));
                return;
            }
        }
        SJ_HIP(hipMemcpy(host_dst, src, need, hipMemcpyDeviceToHost));
    });
}

int sj_index_search(sj_index *idx, int unicomp, void *stream) {
    hipStream_t s = as_stream(stream);
    return guarded(s, [&] {
        if (!idx) throw Error(SJ_EINVAL, "index is NULL");
        if (idx->n) ensure_ranges(*idx, unicomp ? 1 : 0, s);
    });
}

int sj_memory_info(uint64_t *cached_bytes, uint64_t *live_bytes) {
    sj::pool_info(cached_bytes, live_bytes);
    return SJ_OK;
}

int sj_release_cached_memory(void) {
    return guarded(nullptr, [&] {
        SJ_HIP(hipDeviceSynchronize());
        sj::pool_trim();
    });
}

int sj_profile_enable(int on) {
    if (on) sj::profile_reset();
    sj::profile_set(on != 0);
    return SJ_OK;
}

int sj_profile_read(sj_kernel_time *out, uint32_t cap, uint32_t *count) {
    return sj::profile_read(out, cap, count);
}

int sj_profile_select(const char *prefix) {
    sj::profile_select(prefix);
    return SJ_OK;
}

int sj_band_thresholds(uint32_t d, double eps, double extent, float *lo, float *hi) {
    if (!lo || !hi || d < 1 || d > static_cast<uint32_t>(sj::kMaxDim) || !(eps > 0) ||
        !std::isfinite(eps) || !(extent >= 0) || !std::isfinite(extent)) {
        set_error("bad argument");
        return SJ_EINVAL;
    }
    if (!band_thresholds(d, eps, extent, lo, hi)) {
        set_error("FP32 pre-test not usable: eps too small for the coordinate extent");
        return SJ_EINVAL;
    }
    return SJ_OK;
}

}  // extern "C"
