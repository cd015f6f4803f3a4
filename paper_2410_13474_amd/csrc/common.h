// Shared types of libnufds (host and device): complex arithmetic, errors, plan layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "nufds.h"

namespace nufds {

template <typename R>
struct alignas(2 * sizeof(R)) cpx {
    R x, y;
};

template <typename R>
__host__ __device__ __forceinline__ cpx<R> mk(R x, R y) {
    cpx<R> c;
    c.x = x;
    c.y = y;
    return c;
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator*(cpx<R> a, cpx<R> b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__host__ __device__ __forceinline__ cpx<R> operator*(cpx<R> a, R s) { return mk(a.x * s, a.y * s); }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> conjg(cpx<R> a) { return mk(a.x, -a.y); }
// a * (-i) and a * (+i)
template <typename R>
__host__ __device__ __forceinline__ cpx<R> mul_mi(cpx<R> a) { return mk(a.y, -a.x); }
template <typename R>
__host__ __device__ __forceinline__ cpx<R> mul_pi(cpx<R> a) { return mk(-a.y, a.x); }

// Status with a message, set by the host code and reported through nufds_last_error.
void set_error(const std::string& msg);
nufds_status_t fail(nufds_status_t st, const std::string& msg);
nufds_status_t hip_fail(hipError_t e, const char* what);

#define NUFDS_HIP_TRY(call)                                     \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return ::nufds::hip_fail(e_, #call); \
    } while (0)

}  // namespace nufds
