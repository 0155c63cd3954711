// Continuous-batching request server for self-join jobs.
//
// Requests (points, n, d, eps, options) arrive at any time through
// sj_server_submit. Each of the server's slots is a worker thread with its
// own HIP stream; a free slot takes the oldest queued request whose
// estimated device memory fits in what the budget has left (the first
// request is always admitted when nothing else holds memory, so a request
// larger than the budget still runs, alone). The estimate is the index
// bytes plus the caller's expected result size and a quarter (nothing for
// the result without an expectation); after the count pass the
// exact result size is known, and a request whose result needs more than
// its estimate waits (holding its index) until the extra memory is free or
// nothing else holds memory. Requests on different slots run concurrently
// on the device, so a request that arrives while others are running starts
// as soon as a slot and memory are free rather than after the queue drains.
// Results stay in device memory (counted against the budget) until the
// client releases them; completion records carry the queueing and service
// times.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "sj.h"
#include "sj_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
    uint64_t id = 0;
    const double *pts = nullptr;
    int on_device = 0;
    uint64_t n = 0;
    uint32_t d = 0;
    double eps = 0;
    sj_join_opts opts{};
    uint64_t est_bytes = 0;
    uint64_t hint_pairs = 0;  // the caller's expected result size (0: none)
    uint64_t est_pairs = 0;   // pairs reserved at admission
    uint64_t held_bytes = 0;
    Clock::time_point t_submit, t_start, t_done;
    int status = SJ_OK;
    std::string error;
    uint32_t *pairs = nullptr;
    uint64_t npairs = 0;
    uint32_t slot = 0;
    sj_stats stats{};
};

}  // namespace

struct sj_server {
    sj_server_opts opts{};
    std::mutex mu;
    std::condition_variable cv_work;  // workers wait for admissible requests
    std::condition_variable cv_done;  // pollers wait for completions
    std::condition_variable cv_mem;   // fills wait for memory
    std::deque<Request *> queue;
    std::map<uint64_t, Request *> all;
    std::deque<uint64_t> done;
    std::vector<std::thread> workers;
    uint64_t next_id = 1;
    uint64_t mem_used = 0;
    uint64_t peak_mem = 0;
    uint32_t running = 0;
    uint32_t holders = 0;  // requests holding memory (running or results not released)
    uint32_t waiting_mem = 0;  // running requests waiting for result memory
    uint64_t over_estimate = 0;
    uint64_t completed = 0;
    bool stop = false;
};

namespace {

uint64_t index_bytes(uint64_t n, uint32_t d) {
    // coordinates (FP64 + FP32 copy), A, cell of point, dimension-0 cell
    // coordinate, row lengths and offsets, cell tables (bounded by n), sort
    // scratch during the build
    return n * (8ull * d + 4ull * d + 4 + 4 + 4 + 3 * 4 + 2 * 8 + 8 + 4 + 4 * d + 24) + (1u << 20);
}

uint64_t result_bytes(uint64_t pairs) { return pairs * 12ull; }  // pairs + neighbour-id scratch

// Dry-run backend (SJ_SERVER_DRY_RUN): no device work. A request "runs" for
// n / 1e6 milliseconds and its count pass "finds" expected_pairs pairs (n
// without an expectation), or twice that for even request ids, so that the
// scheduler, the admission steps and the accounting can be exercised
// without a GPU.
void run_request_dry(sj_server *S, Request *r, uint32_t slot) {
    std::this_thread::sleep_for(std::chrono::microseconds(r->n / 1000 + 50));
    const uint64_t expected = r->hint_pairs ? r->hint_pairs : r->n;
    const uint64_t P = (r->id % 2 == 0) ? 2 * expected : expected;
    {
        const uint64_t need = index_bytes(r->n, r->d) + result_bytes(P);
        std::unique_lock<std::mutex> lk(S->mu);
        if (need > r->held_bytes) {
            const uint64_t extra = need - r->held_bytes;
            if (r->hint_pairs) ++S->over_estimate;
            // Waits until the extra memory fits, or until no other request
            // can free memory (it is the only holder, or every running
            // request is itself waiting here): the budget is soft, progress
            // is guaranteed.
            ++S->waiting_mem;
            S->cv_mem.notify_all();
            S->cv_mem.wait(lk, [&] {
                return S->stop || S->mem_used + extra <= S->opts.mem_budget_bytes || S->holders <= 1 ||
                       S->waiting_mem >= S->running;
            });
            --S->waiting_mem;
            S->mem_used += extra;
            r->held_bytes += extra;
            S->peak_mem = std::max(S->peak_mem, S->mem_used);
        }
    }
    std::this_thread::sleep_for(std::chrono::microseconds(r->n / 1000 + 50));
    std::lock_guard<std::mutex> lk(S->mu);
    r->status = SJ_OK;
    r->npairs = P;
    const uint64_t keep = result_bytes(P) * 8 / 12;
    if (r->held_bytes > keep) {
        S->mem_used -= r->held_bytes - keep;
        r->held_bytes = keep;
    }
    r->t_done = Clock::now();
    r->slot = slot;
    S->done.push_back(r->id);
    ++S->completed;
    --S->running;
    S->cv_done.notify_all();
    S->cv_work.notify_all();
    S->cv_mem.notify_all();
}

void run_request(sj_server *S, Request *r, uint32_t slot, hipStream_t stream) {
    sj_index *ix = nullptr;
    int rc = sj_build_index(r->pts, r->n, r->d, r->eps, r->on_device, stream, &ix);
    uint64_t P = 0;
    if (rc == SJ_OK) rc = sj_join_count(ix, &r->opts, stream, &P);
    if (rc == SJ_OK) {
        // second admission step: the exact result size
        const uint64_t need = index_bytes(r->n, r->d) + result_bytes(P);
        std::unique_lock<std::mutex> lk(S->mu);
        if (need > r->held_bytes) {
            const uint64_t extra = need - r->held_bytes;
            if (r->hint_pairs) ++S->over_estimate;
            // Waits until the extra memory fits, or until no other request
            // can free memory (it is the only holder, or every running
            // request is itself waiting here): the budget is soft, progress
            // is guaranteed.
            ++S->waiting_mem;
            S->cv_mem.notify_all();
            S->cv_mem.wait(lk, [&] {
                return S->stop || S->mem_used + extra <= S->opts.mem_budget_bytes || S->holders <= 1 ||
                       S->waiting_mem >= S->running;
            });
            --S->waiting_mem;
            S->mem_used += extra;
            r->held_bytes += extra;
            S->peak_mem = std::max(S->peak_mem, S->mem_used);
        }
    }
    if (rc == SJ_OK && P > 0) {
        try {
            r->pairs = static_cast<uint32_t *>(sj::dev_alloc(P * 8));
        } catch (const sj::Error &e) {
            rc = e.code;
        }
        if (rc == SJ_OK) rc = sj_join_fill(ix, r->pairs, P, stream);
    }
    if (rc != SJ_OK) r->error = sj_last_error();
    if (ix) {
        (void)sj_index_stats(ix, &r->stats);
        sj_destroy_index(ix);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    r->status = rc;
    r->npairs = rc == SJ_OK ? P : 0;
    if (rc != SJ_OK && r->pairs) {
        sj::dev_free(r->pairs);
        r->pairs = nullptr;
    }
    // the index is gone: keep only the result's bytes held until release
    const uint64_t keep = result_bytes(r->npairs) * 8 / 12;
    if (r->held_bytes > keep) {
        S->mem_used -= r->held_bytes - keep;
        r->held_bytes = keep;
    }
    r->t_done = Clock::now();
    r->slot = slot;
    S->done.push_back(r->id);
    ++S->completed;
    --S->running;
    S->cv_done.notify_all();
    S->cv_work.notify_all();
    S->cv_mem.notify_all();
}

void worker(sj_server *S, uint32_t slot) {
    const bool dry = (S->opts.flags & SJ_SERVER_DRY_RUN) != 0;
    hipStream_t stream = nullptr;
    if (!dry && hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return;
    while (true) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] {
                if (S->stop) return true;
                if (S->queue.empty()) return false;
                const Request *f = S->queue.front();
                return S->holders == 0 || S->mem_used + f->est_bytes <= S->opts.mem_budget_bytes;
            });
            if (S->stop && S->queue.empty()) break;
            if (S->stop) break;
            r = S->queue.front();
            S->queue.pop_front();
            r->held_bytes = r->est_bytes;
            S->mem_used += r->held_bytes;
            S->peak_mem = std::max(S->peak_mem, S->mem_used);
            ++S->holders;
            ++S->running;
            r->t_start = Clock::now();
        }
        if (dry)
            run_request_dry(S, r, slot);
        else
            run_request(S, r, slot, stream);
    }
    if (!dry) {
        (void)hipStreamSynchronize(stream);
        (void)hipStreamDestroy(stream);
    }
}

}  // namespace

extern "C" {

int sj_server_create(const sj_server_opts *opts, sj_server **out) {
    if (!out || !opts || opts->slots == 0 || opts->slots > 64 || opts->mem_budget_bytes == 0 ||
        (opts->flags & ~static_cast<uint32_t>(SJ_SERVER_DRY_RUN)) != 0)
        return SJ_EINVAL;
    auto *S = new sj_server;
    S->opts = *opts;
    for (uint32_t k = 0; k < opts->slots; ++k) S->workers.emplace_back(worker, S, k);
    *out = S;
    return SJ_OK;
}

int sj_server_submit(sj_server *S, const double *pts, uint64_t n, uint32_t d, double eps,
                     int pts_on_device, const sj_join_opts *opts, uint64_t expected_pairs,
                     uint64_t *req_id) {
    if (!S || !req_id) return SJ_EINVAL;
    auto *r = new Request;
    r->pts = pts;
    r->on_device = pts_on_device;
    r->n = n;
    r->d = d;
    r->eps = eps;
    sj_default_opts(&r->opts);
    if (opts) r->opts = *opts;
    if (r->opts.min_batches == 0) r->opts.min_batches = 1;
    r->hint_pairs = expected_pairs;
    r->est_pairs = expected_pairs + expected_pairs / 4;
    r->est_bytes = index_bytes(n, d) + result_bytes(r->est_pairs);
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        delete r;
        return SJ_ESTATE;
    }
    r->id = S->next_id++;
    S->all[r->id] = r;
    S->queue.push_back(r);
    *req_id = r->id;
    S->cv_work.notify_all();
    return SJ_OK;
}

int sj_server_poll(sj_server *S, sj_completion *out, uint32_t cap, uint32_t *count,
                   int32_t timeout_ms) {
    if (!S || !count || (cap && !out)) return SJ_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done.empty() && timeout_ms != 0) {
        if (timeout_ms < 0)
            S->cv_done.wait(lk, [&] { return !S->done.empty() || S->stop; });
        else
            S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !S->done.empty(); });
    }
    uint32_t k = 0;
    while (k < cap && !S->done.empty()) {
        const uint64_t id = S->done.front();
        S->done.pop_front();
        const auto it = S->all.find(id);
        if (it == S->all.end()) continue;  // released before it was polled
        Request *r = it->second;
        sj_completion &c = out[k++];
        std::memset(&c, 0, sizeof(c));
        c.req_id = id;
        c.status = r->status;
        c.pairs_dev = r->pairs;
        c.npairs = r->npairs;
        c.slot = r->slot;
        c.queue_ms = ms_between(r->t_submit, r->t_start);
        c.service_ms = ms_between(r->t_start, r->t_done);
        c.latency_ms = ms_between(r->t_submit, r->t_done);
        c.evals = r->stats.evals;
        c.band_rechecks = r->stats.band_rechecks;
    }
    *count = k;
    return SJ_OK;
}

int sj_server_release(sj_server *S, uint64_t req_id) {
    if (!S) return SJ_EINVAL;
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(req_id);
        if (it == S->all.end() || it->second->t_done == Clock::time_point{}) return SJ_ESTATE;
        r = it->second;
        S->all.erase(it);
        for (auto d = S->done.begin(); d != S->done.end(); ++d)
            if (*d == req_id) {
                S->done.erase(d);
                break;
            }
        S->mem_used -= r->held_bytes;
        --S->holders;
        S->cv_work.notify_all();
        S->cv_mem.notify_all();
    }
    if (r->pairs) sj::dev_free(r->pairs);
    delete r;
    return SJ_OK;
}

int sj_server_info(sj_server *S, sj_server_info_t *info) {
    if (!S || !info) return SJ_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    info->queued = S->queue.size();
    info->running = S->running;
    info->mem_used_bytes = S->mem_used;
    info->peak_mem_bytes = S->peak_mem;
    info->over_estimate = S->over_estimate;
    info->completed = S->completed;
    return SJ_OK;
}

void sj_server_destroy(sj_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (Request *r : S->queue) {
            S->all.erase(r->id);
            delete r;
        }
        S->queue.clear();
        S->cv_work.notify_all();
        S->cv_mem.notify_all();
        S->cv_done.notify_all();
    }
    for (auto &t : S->workers) t.join();
    for (auto &kv : S->all) {
        if (kv.second->pairs) sj::dev_free(kv.second->pairs);
        delete kv.second;
    }
    delete S;
}

}  // extern "C"
