// Device memory of the library's buffers (see common.h).
#include <mutex>
#include <set>

#include "common.h"

namespace pomm {

hipStream_t& alloc_stream() {
    static thread_local hipStream_t s = nullptr;
    return s;
}

namespace {

// Raise the release threshold of the current device's default pool once, so that
// memory returned by one handle stays mapped for the next setup.
void keep_pool_reserved() {
    static std::mutex mu;
    static std::set<int> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(mu);
    if (done.count(dev)) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t threshold = ~0ull;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
    }
    done.insert(dev);
}

}  // namespace

hipError_t dev_alloc_raw(void** p, size_t bytes) {
    keep_pool_reserved();
    return hipMallocAsync(p, bytes, alloc_stream());
}

hipError_t dev_free(void* p) { return p ? hipFreeAsync(p, alloc_stream()) : hipSuccess; }

}  // namespace pomm
