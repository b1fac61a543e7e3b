// Host helpers shared by the C ABI sources: error codes with detail text,
// HIP status checks and owning device buffers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace ldopf {

// Stores the detail text of the calling thread's most recent failure.
void record_error_detail(const std::string& detail);

inline void hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? LDOPF_OUT_OF_MEMORY : LDOPF_DEVICE_ERROR;
    fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

// Owning device allocation. With `ordered` set, allocation and release are
// stream-ordered on that stream (hipMallocAsync / hipFreeAsync), so that
// freeing one problem's memory does not wait for every kernel on the device
// (hipFree does); the stream must outlive the buffer.
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t count = 0;
    hipStream_t ordered = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            if (ordered)
                (void)hipFreeAsync(p, ordered);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        count = 0;
    }
    void alloc(size_t n, const char* what) {
        release();
        const size_t bytes = std::max<size_t>(1, n) * sizeof(T);
        if (ordered)
            hip_check(hipMallocAsync(reinterpret_cast<void**>(&p), bytes, ordered), what);
        else
            hip_check(hipMalloc(reinterpret_cast<void**>(&p), bytes), what);
        count = n;
    }
    void upload(const std::vector<T>& v, hipStream_t s, const char* what) {
        alloc(v.size(), what);
        if (!v.empty()) hip_check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), what);
    }
};

// Runs f, turning library errors into return codes.
template <typename F>
int guard(F&& f) {
    try {
        f();
        return LDOPF_OK;
    } catch (const Error& e) {
        record_error_detail(e.detail);
        return e.code;
    } catch (const std::bad_alloc&) {
        record_error_detail("host allocation failed");
        return LDOPF_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        record_error_detail(e.what());
        return LDOPF_DEVICE_ERROR;
    }
}

inline void need(const void* p, const char* what) {
    if (!p) fail(LDOPF_INVALID_ARGUMENT, std::string(what) + " must not be NULL");
}

// Option checks shared by the plain and the batched solver.
void check_options(const ldopf_options& o);
// What the batched form adds: the literal residual form and a fixed rho.
void check_batch_options(const ldopf_options& o);

}  // namespace ldopf
