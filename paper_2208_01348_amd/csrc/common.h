// Shared device/host definitions of the gfx950 DDA library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace dda {

// Interleaved complex number (re, im), layout-compatible with complex64 /
// complex128 tensors.
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

using z64 = cx<float>;
using z128 = cx<double>;

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.x, -a.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename T>
__host__ __device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
    return INV ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}
template <typename T>
__host__ __device__ __forceinline__ T norm2(cx<T> a) { return a.x * a.x + a.y * a.y; }

template <typename TO, typename TI>
__host__ __device__ __forceinline__ cx<TO> cvt(cx<TI> a) { return {TO(a.x), TO(a.y)}; }

// Load through a global-address-space pointer.  Pointers read from a table
// in memory (the per-system D spectra) are generic to the compiler, whose
// flat loads also count against the LDS wait counter; these do not.
template <typename T>
__device__ __forceinline__ cx<T> gload(const cx<T>* p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = *(const __attribute__((address_space(1))) v2*)(p);
    return cx<T>{v.x, v.y};
}

// Error carried from the host orchestration to the C ABI boundary.
struct Error : std::runtime_error {
    int status;
    Error(int st, const std::string& msg) : std::runtime_error(msg), status(st) {}
};

}  // namespace dda

#define DDA_HIP_CHECK(expr)                                                            \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess) {                                                        \
            throw ::dda::Error(_e == hipErrorOutOfMemory ? -2 : -3,                    \
                               std::string(#expr) + ": " + hipGetErrorString(_e));     \
        }                                                                              \
    } while (0)

#define DDA_LAUNCH_CHECK() DDA_HIP_CHECK(hipGetLastError())
