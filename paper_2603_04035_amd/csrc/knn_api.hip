// Status strings, thread-local error text, scratch management and argument
// checks shared by every entry point.
#include <stdio.h>

#include <mutex>

#include "knn_common.hpp"

namespace knn {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

knn_status fail(knn_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

// Scratch that does not fit the arena (below), and the arena itself when it
// is first made, come from a memory pool owned by the library, one per
// device, whose release threshold keeps freed blocks mapped.  Pools are held
// until the process ends.
static knn_status scratch_pool(int dev, hipMemPool_t* out)
{
    static std::mutex mu;
    static hipMemPool_t pools[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (!pools[dev]) {
        hipMemPoolProps props = {};
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        hipError_t e = hipMemPoolCreate(&pool, &props);
        if (e != hipSuccess) return fail(KNN_EDEVICE, std::string("hipMemPoolCreate: ") + hipGetErrorString(e));
        uint64_t keep = ~0ull;
        e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        if (e != hipSuccess) return fail(KNN_EDEVICE, std::string("hipMemPoolSetAttribute: ") + hipGetErrorString(e));
        pools[dev] = pool;
    }
    *out = pools[dev];
    return KNN_OK;
}

// The per-device arena: a block of `cap` bytes, the lock that one call holds
// while it uses the block, and an event after the last holder's work.
struct Arena {
    std::mutex mu;
    void* base = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};
static Arena g_arena[64];

unsigned long long* pinned_counters()
{
    // one small pinned block per host thread, held until the process ends
    static thread_local unsigned long long* p = nullptr;
    if (!p && hipHostMalloc((void**)&p, 64, hipHostMallocDefault) != hipSuccess) p = nullptr;
    return p;
}

Workspace::Workspace(hipStream_t s, int64_t limit) : stream_(s), limit_(limit)
{
    if (hipGetDevice(&dev_) != hipSuccess || dev_ < 0 || dev_ >= 64) {
        (void)hipGetLastError();
        dev_ = -1;
        return;
    }
    Arena& a = g_arena[dev_];
    a.mu.lock();
    if (a.done) (void)hipStreamWaitEvent(stream_, a.done, 0);
}

Workspace::~Workspace()
{
    if (dev_ < 0) return;
    Arena& a = g_arena[dev_];
    for (int i = 0; i < nptr_; ++i) (void)hipFreeAsync(ptrs_[i], stream_);
    if (used_ > a.cap) {
        // regrow for the next call; the old block is released once this
        // call's work, the last that may touch it, has finished
        (void)hipStreamSynchronize(stream_);
        if (a.base) (void)hipFree(a.base);
        a.base = nullptr;
        a.cap = 0;
        const size_t cap = (size_t)round_up((int64_t)(used_ + used_ / 8), (int64_t)1 << 20);
        if (hipMalloc(&a.base, cap) == hipSuccess) a.cap = cap;
        else (void)hipGetLastError();
    }
    if (!a.done && hipEventCreateWithFlags(&a.done, hipEventDisableTiming) != hipSuccess) a.done = nullptr;
    if (a.done) (void)hipEventRecord(a.done, stream_);
    a.mu.unlock();
}

knn_status Workspace::alloc(void** p, size_t bytes)
{
    *p = nullptr;
    if (dev_ < 0) return fail(KNN_EDEVICE, "no current device");
    if (bytes == 0) bytes = 256;
    bytes = (size_t)round_up((int64_t)bytes, 256);
    if (limit_ > 0 && (int64_t)(used_ + bytes) > limit_)
        return fail(KNN_ENOMEM, "workspace limit exceeded: need " + std::to_string(used_ + bytes) +
                                    " bytes, limit " + std::to_string(limit_));
    Arena& a = g_arena[dev_];
    if (nptr_ == 0 && off_ + bytes <= a.cap) {
        *p = (char*)a.base + off_;
        off_ += bytes;
        used_ += bytes;
        return KNN_OK;
    }
    if (nptr_ == 64) return fail(KNN_ENOMEM, "too many scratch buffers");
    hipMemPool_t pool = nullptr;
    knn_status r = scratch_pool(dev_, &pool);
    if (r != KNN_OK) return r;
    hipError_t e = hipMallocFromPoolAsync(p, bytes, pool, stream_);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(KNN_ENOMEM, std::string("hipMallocFromPoolAsync(") + std::to_string(bytes) +
                                    "): " + hipGetErrorString(e));
    }
    ptrs_[nptr_++] = *p;
    used_ += bytes;
    return KNN_OK;
}

knn_status FixedScratch::alloc(void** p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    bytes = (size_t)round_up((int64_t)bytes, 256);
    if (off_ + bytes > cap_)
        return fail(KNN_ENOMEM, "static scratch exhausted: need " + std::to_string(off_ + bytes) +
                                    " bytes, the array holds " + std::to_string(cap_));
    *p = base_ + off_;
    off_ += bytes;
    return KNN_OK;
}

knn_status check_matrix(const knn_matrix& X, const char* name)
{
    std::string n(name);
    if (!X.data) return fail(KNN_EINVAL, n + ".data is null");
    if (X.n < 1) return fail(KNN_EINVAL, n + ".n must be >= 1");
    if (X.n >= (int64_t)0x7FFFFFFF) return fail(KNN_EINVAL, n + ".n must be below 2^31 - 1");
    if (X.d < 1) return fail(KNN_EINVAL, n + ".d must be >= 1");
    if (X.ld < X.d) return fail(KNN_EINVAL, n + ".ld must be >= d");
    if (X.dtype != KNN_F32 && X.dtype != KNN_BF16 && X.dtype != KNN_F16)
        return fail(KNN_EINVAL, n + ".dtype unknown");
    return KNN_OK;
}

}  // namespace knn

extern "C" const char* knn_status_str(knn_status s)
{
    switch (s) {
    case KNN_OK: return "KNN_OK";
    case KNN_EINVAL: return "KNN_EINVAL";
    case KNN_ENOMEM: return "KNN_ENOMEM";
    case KNN_EDEVICE: return "KNN_EDEVICE";
    case KNN_ENOTSUP: return "KNN_ENOTSUP";
    default: return "KNN_UNKNOWN";
    }
}

extern "C" const char* knn_last_error(void) { return knn::g_last_error.c_str(); }
