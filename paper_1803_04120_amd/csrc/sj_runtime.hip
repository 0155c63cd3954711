// Host runtime: error plumbing and the caching device-memory pool.
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "sj_internal.h"

namespace sj {

void hip_check(hipError_t e, const char *what, const char *file, int line) {
    if (e == hipSuccess) return;
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    throw Error(e == hipErrorOutOfMemory ? SJ_ENOMEM : SJ_EDEVICE, buf);
}

// ---------------------------------------------------------------------
// Caching pool. Sizes are rounded up to 2 MiB above 1 MiB (or to a power of
// two below), blocks are kept per (device, size) in free lists. A freed
// block is not reusable at once: frees made while an API call is running go
// to the calling thread's pending list and are released by the call's guard
// after it has synchronised its stream, so no kernel of that call can still
// be touching the block when another stream gets it.
// ---------------------------------------------------------------------
namespace {

struct Pool {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void *>> free_blocks;
    std::map<void *, std::pair<int, size_t>> live;
    size_t cached_bytes = 0;
};

Pool &pool() {
    static Pool *p = new Pool;  // never destroyed: may be used during process exit
    return *p;
}

thread_local std::vector<void *> t_pending;
thread_local int t_depth = 0;

size_t round_size(size_t b) {
    if (b <= 256) return 256;
    if (b < (1u << 20)) {
        size_t p = 256;
        while (p < b) p <<= 1;
        return p;
    }
    const size_t g = 2u << 20;
    return (b + g - 1) / g * g;
}

void release_now(void *p) {
    Pool &P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    auto it = P.live.find(p);
    if (it == P.live.end()) return;
    P.free_blocks[it->second].push_back(p);
    P.cached_bytes += it->second.second;
    P.live.erase(it);
}

}  // namespace

namespace {
struct StagePool {
    std::mutex mu;
    std::vector<void *> free_blocks;
};
StagePool &stage_pool() {
    static StagePool *p = new StagePool;  // never destroyed: may be used during process exit
    return *p;
}
}  // namespace

void *stage_acquire() {
    StagePool &P = stage_pool();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        if (!P.free_blocks.empty()) {
            void *p = P.free_blocks.back();
            P.free_blocks.pop_back();
            return p;
        }
    }
    void *p = nullptr;
    SJ_HIP(hipHostMalloc(&p, kStageBytes, hipHostMallocDefault));
    return p;
}

void stage_release(void *p) {
    if (!p) return;
    StagePool &P = stage_pool();
    std::lock_guard<std::mutex> lk(P.mu);
    P.free_blocks.push_back(p);
}

void *dev_alloc(size_t bytes) {
    int dev = 0;
    SJ_HIP(hipGetDevice(&dev));
    const size_t sz = round_size(bytes);
    Pool &P = pool();
    {
        // best fit: the smallest cached block of at least sz and at most a
        // quarter larger, so that requests of nearly equal size (the results
        // of one workload at slightly different sizes) share blocks instead
        // of each keeping its own
        std::lock_guard<std::mutex> lk(P.mu);
        const size_t limit = sz + sz / 4;
        for (auto it = P.free_blocks.lower_bound({dev, sz});
             it != P.free_blocks.end() && it->first.first == dev && it->first.second <= limit; ++it) {
            if (it->second.empty()) continue;
            void *p = it->second.back();
            it->second.pop_back();
            P.cached_bytes -= it->first.second;
            P.live[p] = it->first;
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        pool_trim();
        e = hipMalloc(&p, sz);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        char buf[128];
        std::snprintf(buf, sizeof(buf), "device allocation of %zu bytes failed", sz);
        throw Error(SJ_ENOMEM, buf);
    }
    std::lock_guard<std::mutex> lk(P.mu);
    P.live[p] = {dev, sz};
    return p;
}

void dev_free(void *p) {
    if (!p) return;
    if (t_depth > 0)
        t_pending.push_back(p);
    else
        release_now(p);
}

void pool_info(uint64_t *cached, uint64_t *live) {
    Pool &P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    uint64_t l = 0;
    for (const auto &kv : P.live) l += kv.second.second;
    if (cached) *cached = P.cached_bytes;
    if (live) *live = l;
}

void pool_trim() {
    Pool &P = pool();
    std::lock_guard<std::mutex> lk(P.mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : P.free_blocks) {
        for (void *p : kv.second) {
            (void)hipSetDevice(kv.first.first);
            (void)hipFree(p);
        }
        P.cached_bytes -= kv.first.second * kv.second.size();
        kv.second.clear();
    }
    (void)hipSetDevice(cur);
}

// ---------------------------------------------------------------------
// Kernel timing
// ---------------------------------------------------------------------
namespace {
struct ProfEntry {
    uint64_t launches = 0;
    double total_ms = 0.0;
};
std::mutex g_prof_mu;
std::map<std::string, ProfEntry> g_prof;
bool g_prof_on = false;
std::string g_prof_prefix;  // written only while no call is running
struct PendingEvent {
    const char *name;
    hipEvent_t e0, e1;
};
thread_local std::vector<PendingEvent> t_prof_pending;
thread_local std::vector<hipEvent_t> t_event_pool;

hipEvent_t take_event() {
    if (!t_event_pool.empty()) {
        hipEvent_t e = t_event_pool.back();
        t_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool profiling_enabled() { return g_prof_on; }

KTimer::KTimer(const char *name, hipStream_t s) : name_(name), s_(s) {
    if (!g_prof_on) return;
    if (!g_prof_prefix.empty() && std::strncmp(name, g_prof_prefix.c_str(), g_prof_prefix.size()) != 0) return;
    e0_ = take_event();
    e1_ = take_event();
    if (!e0_ || !e1_) {
        if (e0_) t_event_pool.push_back(e0_);
        if (e1_) t_event_pool.push_back(e1_);
        e0_ = e1_ = nullptr;
        return;
    }
    (void)hipEventRecord(e0_, s_);
}

KTimer::~KTimer() {
    if (!e0_) return;
    (void)hipEventRecord(e1_, s_);
    t_prof_pending.push_back({name_, e0_, e1_});
}

void profile_resolve_pending() {
    std::vector<PendingEvent> v;
    v.swap(t_prof_pending);
    for (auto &p : v) {
        float ms = 0.f;
        if (hipEventSynchronize(p.e1) == hipSuccess && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            auto &e = g_prof[p.name];
            e.launches += 1;
            e.total_ms += ms;
        }
        t_event_pool.push_back(p.e0);
        t_event_pool.push_back(p.e1);
    }
}

void profile_reset() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.clear();
}

void profile_set(bool on) { g_prof_on = on; }
void profile_select(const char *prefix) { g_prof_prefix = prefix ? prefix : ""; }

// out: array of {char name[48]; uint64 launches; double total_ms} records
int profile_read(void *out, uint32_t cap, uint32_t *count) {
    struct Rec {
        char name[48];
        uint64_t launches;
        double total_ms;
    };
    std::lock_guard<std::mutex> lk(g_prof_mu);
    uint32_t k = 0;
    for (auto &kv : g_prof) {
        if (out && k < cap) {
            Rec &r = static_cast<Rec *>(out)[k];
            std::memset(r.name, 0, sizeof(r.name));
            std::strncpy(r.name, kv.first.c_str(), sizeof(r.name) - 1);
            r.launches = kv.second.launches;
            r.total_ms = kv.second.total_ms;
        }
        ++k;
    }
    if (count) *count = k;
    return 0;
}

// Called by the API guard (sj_api.hip).
void pool_enter() { ++t_depth; }
void pool_leave_after_sync() {
    profile_resolve_pending();
    if (--t_depth == 0) {
        std::vector<void *> v;
        v.swap(t_pending);
        for (void *p : v) release_now(p);
    }
}

}  // namespace sj
