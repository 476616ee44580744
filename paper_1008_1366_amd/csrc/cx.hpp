// cx.hpp -- complex arithmetic on interleaved (re, im) pairs for the gfx950
// kernels.  C<T> has the memory layout of numpy complex64/complex128 and of
// torch.complex64/complex128 (8- and 16-byte aligned pairs), so global loads
// compile to one dwordx2/dwordx4 per element.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace impconv {

template <typename T>
struct alignas(2 * sizeof(T)) C {
    T re, im;
};

template <typename T> __host__ __device__ __forceinline__ C<T> mk(T a, T b) { return C<T>{a, b}; }
template <typename T> __host__ __device__ __forceinline__ C<T> zero() { return C<T>{T(0), T(0)}; }
template <typename T> __host__ __device__ __forceinline__ C<T> operator+(C<T> a, C<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ __forceinline__ C<T> operator-(C<T> a, C<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ __forceinline__ C<T> operator*(C<T> a, C<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ __forceinline__ C<T> scale(C<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T> __host__ __device__ __forceinline__ C<T> conj(C<T> a) { return {a.re, -a.im}; }
// a * conj(b)
template <typename T> __host__ __device__ __forceinline__ C<T> mulc(C<T> a, C<T> b)
{
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// multiply by i (s = +1) or by -i (s = -1)
template <int S, typename T> __host__ __device__ __forceinline__ C<T> muli(C<T> a)
{
    if constexpr (S > 0) return {-a.im, a.re};
    else return {a.im, -a.re};
}
// root of unity with sign: DIR = +1 uses w, DIR = -1 uses conj(w)
template <int DIR, typename T> __host__ __device__ __forceinline__ C<T> mulw(C<T> a, C<T> w)
{
    if constexpr (DIR > 0) return a * w;
    else return mulc(a, w);
}

}  // namespace impconv
