// Host runtime: error plumbing and the caching device-memory pool.
#include <cstdio>
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

void *dev_alloc(size_t bytes) {
    int dev = 0;
    SJ_HIP(hipGetDevice(&dev));
    const size_t sz = round_size(bytes);
    Pool &P = pool();
    {
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.free_blocks.find({dev, sz});
        if (it != P.free_blocks.end() && !it->second.empty()) {
            void *p = it->second.back();
            it->second.pop_back();
            P.cached_bytes -= sz;
            P.live[p] = {dev, sz};
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

// Called by the API guard (sj_api.hip).
void pool_enter() { ++t_depth; }
void pool_leave_after_sync() {
    if (--t_depth == 0) {
        std::vector<void *> v;
        v.swap(t_pending);
        for (void *p : v) release_now(p);
    }
}

}  // namespace sj
