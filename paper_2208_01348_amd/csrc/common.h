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
