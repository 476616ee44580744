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

// Compensated root of unity: w = h + l with h the rounding of the FP64 value
// to T and l the rounding of the remainder.  a * w is formed as a h + a l
// with the small product added first, so the representation error of the
// twiddle (about 2^-24 |w| in FP32) drops to second order.
template <typename T>
struct TwHL {
    C<T> h, l;
};
template <typename T> __host__ __device__ __forceinline__ T fmat(T a, T b, T c)
{
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}
template <int DIR, typename T> __host__ __device__ __forceinline__ C<T> mulw(C<T> a, TwHL<T> w)
{
    const C<T> s = mulw<DIR>(a, w.l);
    if constexpr (DIR > 0)
        return {fmat(a.re, w.h.re, fmat(-a.im, w.h.im, s.re)), fmat(a.re, w.h.im, fmat(a.im, w.h.re, s.im))};
    else
        return {fmat(a.re, w.h.re, fmat(a.im, w.h.im, s.re)), fmat(a.im, w.h.re, fmat(-a.re, w.h.im, s.im))};
}
// Twiddle source over a pair of tables (high and low parts, same indexing):
// usable wherever the FFT takes a twiddle pointer.
template <typename T>
struct CompTw {
    const C<T>* h;
    const C<T>* l;
    __host__ __device__ __forceinline__ CompTw operator+(int64_t z) const { return CompTw{h + z, l + z}; }
    __host__ __device__ __forceinline__ TwHL<T> operator[](int64_t j) const { return TwHL<T>{h[j], l[j]}; }
};

}  // namespace impconv
