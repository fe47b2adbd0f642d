// Status strings, thread-local error text, scratch management and argument
// checks shared by every entry point.
#include <stdio.h>

#include "knn_common.hpp"

namespace knn {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

knn_status fail(knn_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

Workspace::~Workspace()
{
    for (int i = 0; i < nptr_; ++i) (void)hipFreeAsync(ptrs_[i], stream_);
}

knn_status Workspace::alloc(void** p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    bytes = (size_t)round_up((int64_t)bytes, 256);
    if (limit_ > 0 && (int64_t)(used_ + bytes) > limit_)
        return fail(KNN_ENOMEM, "workspace limit exceeded: need " + std::to_string(used_ + bytes) +
                                    " bytes, limit " + std::to_string(limit_));
    if (nptr_ == 64) return fail(KNN_ENOMEM, "too many scratch buffers");
    hipError_t e = hipMallocAsync(p, bytes, stream_);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(KNN_ENOMEM, std::string("hipMallocAsync(") + std::to_string(bytes) +
                                    "): " + hipGetErrorString(e));
    }
    ptrs_[nptr_++] = *p;
    used_ += bytes;
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
