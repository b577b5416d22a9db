// Device memory of the library's buffers (see common.h).
//
// Stream-ordered allocations from the device's default pool, plus a cache of large
// blocks: a handle's workspace (GMRES bases, factors, sparse-solve buffers) is freed on
// destroy and asked for again, in the same sizes, by the next setup of the same
// problem shape.  Returning such blocks to the pool costs milliseconds per call, so
// blocks of at least kCacheMin bytes are kept here instead, keyed by device and exact
// size, with an event recorded on the freeing stream; a later allocation of that size
// takes the block back and orders its stream after the event.  At most kCacheMax bytes
// are kept (oldest blocks are returned first), and everything cached is returned to
// the pool when an allocation fails, before it is tried again.
#include <list>
#include <mutex>
#include <set>
#include <unordered_map>

#include "common.h"

namespace pomm {

hipStream_t& alloc_stream() {
    static thread_local hipStream_t s = nullptr;
    return s;
}

namespace {

constexpr size_t kCacheMin = size_t(1) << 20;
constexpr size_t kCacheMax = size_t(64) << 30;

struct Cached {
    void* p;
    size_t bytes;
    int dev;
    hipEvent_t ready;   // recorded on the freeing stream
};

struct Cache {
    std::mutex mu;
    std::unordered_map<void*, std::pair<size_t, int>> live;   // cacheable blocks in use: size, device
    std::list<Cached> idle;                                    // oldest first
    size_t idle_bytes = 0;
    std::set<int> pool_done;
};

Cache& cache() {
    static Cache* c = new Cache();   // never destroyed: blocks may be freed during process exit
    return *c;
}

// Raise the release threshold of the current device's default pool once, so that
// memory returned to it stays mapped for the next setup.
void keep_pool_reserved(Cache& c, int dev) {
    if (c.pool_done.count(dev)) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t threshold = ~0ull;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
    }
    c.pool_done.insert(dev);
}

// Return a cached block to its device's pool once the work that used it has finished.
void release(Cached& b) {
    (void)hipEventSynchronize(b.ready);
    (void)hipEventDestroy(b.ready);
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != b.dev) (void)hipSetDevice(b.dev);
    (void)hipFreeAsync(b.p, nullptr);
    if (cur != b.dev) (void)hipSetDevice(cur);
}

// caller holds c.mu
void trim(Cache& c, size_t keep) {
    while (c.idle_bytes > keep && !c.idle.empty()) {
        Cached b = c.idle.front();
        c.idle.pop_front();
        c.idle_bytes -= b.bytes;
        release(b);
    }
}

}  // namespace

hipError_t dev_alloc_raw(void** p, size_t bytes) {
    Cache& c = cache();
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(c.mu);
    keep_pool_reserved(c, dev);
    const hipStream_t s = alloc_stream();
    if (bytes >= kCacheMin) {
        for (auto it = c.idle.begin(); it != c.idle.end(); ++it) {
            if (it->bytes != bytes || it->dev != dev) continue;
            e = hipStreamWaitEvent(s, it->ready, 0);   // after the work that used it before
            if (e != hipSuccess) return e;
            (void)hipEventDestroy(it->ready);
            *p = it->p;
            c.idle_bytes -= bytes;
            c.live[*p] = {bytes, dev};
            c.idle.erase(it);
            return hipSuccess;
        }
    }
    e = hipMallocAsync(p, bytes, s);
    if (e != hipSuccess && !c.idle.empty()) {   // give the cached blocks back and try once more
        (void)hipGetLastError();
        trim(c, 0);
        e = hipMallocAsync(p, bytes, s);
    }
    if (e == hipSuccess && bytes >= kCacheMin) c.live[*p] = {bytes, dev};
    return e;
}

hipError_t dev_free(void* p) {
    if (!p) return hipSuccess;
    Cache& c = cache();
    std::lock_guard<std::mutex> lock(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return hipFreeAsync(p, alloc_stream());
    const size_t bytes = it->second.first;
    const int dev = it->second.second;
    c.live.erase(it);
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, alloc_stream());
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return hipFreeAsync(p, alloc_stream());
    }
    c.idle.push_back(Cached{p, bytes, dev, ev});
    c.idle_bytes += bytes;
    trim(c, kCacheMax);
    return hipSuccess;
}

}  // namespace pomm
