// fft_wg.hpp -- workgroup-cooperative power-of-two FFT for gfx950.
//
// One FFT of size N is computed by G = N / E threads ("a group").  Thread t of
// the group keeps E elements in registers, element i being sequence position
// t + i*G.  Each radix-R Stockham stage takes its butterfly inputs straight
// from registers (a butterfly's R inputs sit E/R registers apart in one
// thread), applies the stage twiddles and the radix-R DFT, and scatters its R
// outputs through LDS so that every thread again holds positions t + i*G.
// The last stage needs no exchange: its outputs already land on positions
// t + i*G.  A forward transform can therefore start directly on the output
// registers of a backward one, which is how the convolution kernels apply
// their pointwise products without touching LDS or HBM.
//
// Sign convention (Sec. 2.1 of Bowman & Roberts): the backward transform
// (DIR = +1) is u_j = sum_k zeta_N^{jk} U_k with zeta_N = exp(2 pi i / N); the
// forward transform (DIR = -1) uses zeta_N^{-jk}.  Neither is normalized.
//
// Twiddles come from a table tw_N[j] = zeta_N^j (j < N) generated in FP64 on
// the host (twiddle.cpp); the FP32 table holds the correctly rounded values.
#pragma once
#include <type_traits>
#include <utility>

#include "cx.hpp"

namespace impconv {

// LDS position of sequence element p: one padding slot every 16 elements
// breaks the power-of-two strides of the early Stockham stages across banks.
__device__ __forceinline__ int lpad(int p) { return p + (p >> 4); }

// Synchronization around a stage exchange of a transform spread over G
// threads with LDS stride LS.  The row kernels (LS = 1) give each transform
// G consecutive threads and LDS of its own; with G <= 64 (a power of two)
// those threads lie in one wave, whose LDS operations the hardware performs
// in issue order, so the exchange needs no workgroup barrier: only that the
// compiler keep the reads after the writes and that the writes have
// completed.  The column passes (LS > 1 there whenever G <= 64) interleave
// their transforms across waves and take the barrier.
#ifndef IMPCONV_NO_WAVE_SYNC
template <int G>
__device__ __forceinline__ void xsync(int LS)
{
    if (G <= 64 && LS == 1) {
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    } else {
        __syncthreads();
    }
}
#else
template <int G>
__device__ __forceinline__ void xsync(int) { __syncthreads(); }
#endif
__host__ __device__ constexpr int lpad_size(int n) { return n + (n >> 4); }

// ------------------------------------------------------------------ radix-R DFTs
template <int DIR, typename T>
__device__ __forceinline__ void dft2(C<T>& a, C<T>& b)
{
    C<T> s = a + b;
    b = a - b;
    a = s;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(C<T>& a0, C<T>& a1, C<T>& a2, C<T>& a3)
{
    C<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = muli<DIR>(a1 - a3);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
}

template <int DIR, typename T>
__device__ __forceinline__ C<T> rot8(C<T> a, int j)  // a * zeta_8^{DIR j}, j in 0..3
{
    const T h = T(0.70710678118654752440);
    switch (j) {
        case 1: return mulw<DIR>(a, C<T>{h, h});
        case 2: return muli<DIR>(a);
        case 3: return mulw<DIR>(a, C<T>{-h, h});
        default: return a;
    }
}

template <int R, int DIR, typename T> struct DFT;

template <int DIR, typename T> struct DFT<1, DIR, T> {
    static __device__ __forceinline__ void run(C<T>*) {}
};
template <int DIR, typename T> struct DFT<2, DIR, T> {
    static __device__ __forceinline__ void run(C<T>* u) { dft2<DIR>(u[0], u[1]); }
};
template <int DIR, typename T> struct DFT<4, DIR, T> {
    static __device__ __forceinline__ void run(C<T>* u) { dft4<DIR>(u[0], u[1], u[2], u[3]); }
};
template <int DIR, typename T> struct DFT<8, DIR, T> {
    static __device__ __forceinline__ void run(C<T>* u)
    {
        C<T> e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6];
        C<T> o0 = u[1], o1 = u[3], o2 = u[5], o3 = u[7];
        dft4<DIR>(e0, e1, e2, e3);
        dft4<DIR>(o0, o1, o2, o3);
        o1 = rot8<DIR>(o1, 1);
        o2 = rot8<DIR>(o2, 2);
        o3 = rot8<DIR>(o3, 3);
        u[0] = e0 + o0; u[4] = e0 - o0;
        u[1] = e1 + o1; u[5] = e1 - o1;
        u[2] = e2 + o2; u[6] = e2 - o2;
        u[3] = e3 + o3; u[7] = e3 - o3;
    }
};
template <int DIR, typename T> struct DFT<16, DIR, T> {
    // 4 x 4 decomposition: n = 4 n1 + n2, k = k1 + 4 k2.
    static __device__ __forceinline__ void run(C<T>* u)
    {
        const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
        const T h = T(0.70710678118654752440);
        C<T> b[16];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            C<T> a0 = u[n2], a1 = u[4 + n2], a2 = u[8 + n2], a3 = u[12 + n2];
            dft4<DIR>(a0, a1, a2, a3);
            b[4 * n2 + 0] = a0; b[4 * n2 + 1] = a1; b[4 * n2 + 2] = a2; b[4 * n2 + 3] = a3;
        }
        // twiddles zeta_16^{DIR n2 k1}
        b[4 * 1 + 1] = mulw<DIR>(b[4 * 1 + 1], C<T>{c1, s1});
        b[4 * 1 + 2] = mulw<DIR>(b[4 * 1 + 2], C<T>{h, h});
        b[4 * 1 + 3] = mulw<DIR>(b[4 * 1 + 3], C<T>{s1, c1});
        b[4 * 2 + 1] = mulw<DIR>(b[4 * 2 + 1], C<T>{h, h});
        b[4 * 2 + 2] = muli<DIR>(b[4 * 2 + 2]);
        b[4 * 2 + 3] = mulw<DIR>(b[4 * 2 + 3], C<T>{-h, h});
        b[4 * 3 + 1] = mulw<DIR>(b[4 * 3 + 1], C<T>{s1, c1});
        b[4 * 3 + 2] = mulw<DIR>(b[4 * 3 + 2], C<T>{-h, h});
        b[4 * 3 + 3] = mulw<DIR>(b[4 * 3 + 3], C<T>{-c1, -s1});
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            C<T> a0 = b[k1], a1 = b[4 + k1], a2 = b[8 + k1], a3 = b[12 + k1];
            dft4<DIR>(a0, a1, a2, a3);
            u[k1] = a0; u[k1 + 4] = a1; u[k1 + 8] = a2; u[k1 + 12] = a3;
        }
    }
};

// ------------------------------------------------------------------ Stockham stages
// Group-local LDS view: element p of this group's sequence lives at
// lds[lpad(p) * LS], LS = element stride (1 for rows, tile width for columns).
// Addressing: lpad(x + c) = lpad(x) + c + (c >> 4) whenever
// (x mod 16) + (c mod 16) < 16.  Both access patterns below satisfy it for
// every power-of-two stage shape -- reads at t + i G (t < G, G a power of
// two) and writes at base + r NS (base mod 16 < 16 - (R-1) NS mod 16) -- so
// each butterfly computes one padded base and every element adds a
// compile-time offset (an immediate in the LDS instruction).
template <typename T, int N, int E, int DIR, int NS, typename TW>
__device__ __forceinline__ void fft_stage(C<T> (&v)[E], int t, C<T>* lds, int LS, TW tw)
{
    constexpr int R = (N / NS < E) ? (N / NS) : E;
    constexpr bool LAST = (NS * R == N);
    constexpr int G = N / E;
    constexpr int Q = E / R;
    static_assert(E % R == 0, "radix must divide the per-thread element count");
    static_assert(R >= 2, "every stage must have radix >= 2");
    // The thread index and a zero table offset are laundered through empty
    // asm statements so the compiler recomputes this stage's LDS addresses
    // and reloads its twiddles here instead of hoisting them out of the
    // caller's loops, which would keep the addresses and twiddles of every
    // stage of every transform live at once and exhaust the register file.
    int zoff = 0;
    asm volatile("" : "+s"(zoff));
    asm volatile("" : "+v"(t));
    const TW tws = tw + zoff;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = t + q * G;
        const int k = b & (NS - 1);
        C<T> u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[q + r * Q];
        if constexpr (NS > 1) {
            const int ks = k * (N / (NS * R));  // twiddle r of this butterfly: zeta_N^{r ks}
#pragma unroll
            for (int r = 1; r < R; ++r) u[r] = mulw<DIR>(u[r], tws[r * ks]);
        }
        DFT<R, DIR, T>::run(u);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q + r * Q] = u[r];
        } else {
            C<T>* wp = lds + lpad((b - k) * R + k) * LS;
#pragma unroll
            for (int r = 0; r < R; ++r) wp[(r * NS + ((r * NS) >> 4)) * LS] = u[r];
        }
    }
    if constexpr (!LAST) {
        xsync<G>(LS);
        const C<T>* rp = lds + lpad(t) * LS;
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = rp[(i * G + ((i * G) >> 4)) * LS];
        xsync<G>(LS);
        fft_stage<T, N, E, DIR, NS * R, TW>(v, t, lds, LS, tw);
    }
}

// Two independent FFTs of the same size and direction advanced stage by
// stage together: one set of twiddle loads and one pair of barriers per
// stage serves both, and the two butterfly streams interleave to hide LDS
// latency.  lds0 / lds1 are two disjoint exchange buffers.
template <typename T, int N, int E, int DIR, int NS, typename TW>
__device__ __forceinline__ void fft2_stage(C<T> (&v0)[E], C<T> (&v1)[E], int t, C<T>* lds0, C<T>* lds1,
                                           int LS, TW tw)
{
    constexpr int R = (N / NS < E) ? (N / NS) : E;
    constexpr bool LAST = (NS * R == N);
    constexpr int G = N / E;
    constexpr int Q = E / R;
    int zoff = 0;
    asm volatile("" : "+s"(zoff));
    asm volatile("" : "+v"(t));
    const TW tws = tw + zoff;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = t + q * G;
        const int k = b & (NS - 1);
        C<T> u0[R], u1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            u0[r] = v0[q + r * Q];
            u1[r] = v1[q + r * Q];
        }
        if constexpr (NS > 1) {
            const int ks = k * (N / (NS * R));
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const auto w = tws[r * ks];
                u0[r] = mulw<DIR>(u0[r], w);
                u1[r] = mulw<DIR>(u1[r], w);
            }
        }
        DFT<R, DIR, T>::run(u0);
        DFT<R, DIR, T>::run(u1);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                v0[q + r * Q] = u0[r];
                v1[q + r * Q] = u1[r];
            }
        } else {
            const int wb = lpad((b - k) * R + k) * LS;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                lds0[wb + (r * NS + ((r * NS) >> 4)) * LS] = u0[r];
                lds1[wb + (r * NS + ((r * NS) >> 4)) * LS] = u1[r];
            }
        }
    }
    if constexpr (!LAST) {
        xsync<G>(LS);
        const int rb = lpad(t) * LS;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            v0[i] = lds0[rb + (i * G + ((i * G) >> 4)) * LS];
            v1[i] = lds1[rb + (i * G + ((i * G) >> 4)) * LS];
        }
        xsync<G>(LS);
        fft2_stage<T, N, E, DIR, NS * R, TW>(v0, v1, t, lds0, lds1, LS, tw);
    }
}

template <typename T, int N, int E, int DIR, typename TW>
__device__ __forceinline__ void fft2(C<T> (&v0)[E], C<T> (&v1)[E], int t, C<T>* lds0, C<T>* lds1, int LS,
                                     TW tw)
{
    if constexpr (N > 1) fft2_stage<T, N, E, DIR, 1, TW>(v0, v1, t, lds0, lds1, LS, tw);
}

// Three independent FFTs advanced together (as fft2_stage, three exchange
// buffers): the three residues of the 2/3 rule share every barrier and
// twiddle load.
template <typename T, int N, int E, int DIR, int NS, typename TW>
__device__ __forceinline__ void fft3_stage(C<T> (&v0)[E], C<T> (&v1)[E], C<T> (&v2)[E], int t, C<T>* lds0,
                                           C<T>* lds1, C<T>* lds2, int LS, TW tw)
{
    constexpr int R = (N / NS < E) ? (N / NS) : E;
    constexpr bool LAST = (NS * R == N);
    constexpr int G = N / E;
    constexpr int Q = E / R;
    int zoff = 0;
    asm volatile("" : "+s"(zoff));
    asm volatile("" : "+v"(t));
    const TW tws = tw + zoff;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = t + q * G;
        const int k = b & (NS - 1);
        C<T> u0[R], u1[R], u2[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            u0[r] = v0[q + r * Q];
            u1[r] = v1[q + r * Q];
            u2[r] = v2[q + r * Q];
        }
        if constexpr (NS > 1) {
            const int ks = k * (N / (NS * R));
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const auto w = tws[r * ks];
                u0[r] = mulw<DIR>(u0[r], w);
                u1[r] = mulw<DIR>(u1[r], w);
                u2[r] = mulw<DIR>(u2[r], w);
            }
        }
        DFT<R, DIR, T>::run(u0);
        DFT<R, DIR, T>::run(u1);
        DFT<R, DIR, T>::run(u2);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                v0[q + r * Q] = u0[r];
                v1[q + r * Q] = u1[r];
                v2[q + r * Q] = u2[r];
            }
        } else {
            const int wb = lpad((b - k) * R + k) * LS;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                lds0[wb + (r * NS + ((r * NS) >> 4)) * LS] = u0[r];
                lds1[wb + (r * NS + ((r * NS) >> 4)) * LS] = u1[r];
                lds2[wb + (r * NS + ((r * NS) >> 4)) * LS] = u2[r];
            }
        }
    }
    if constexpr (!LAST) {
        xsync<G>(LS);
        const int rb = lpad(t) * LS;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            v0[i] = lds0[rb + (i * G + ((i * G) >> 4)) * LS];
            v1[i] = lds1[rb + (i * G + ((i * G) >> 4)) * LS];
            v2[i] = lds2[rb + (i * G + ((i * G) >> 4)) * LS];
        }
        xsync<G>(LS);
        fft3_stage<T, N, E, DIR, NS * R, TW>(v0, v1, v2, t, lds0, lds1, lds2, LS, tw);
    }
}

template <typename T, int N, int E, int DIR, typename TW>
__device__ __forceinline__ void fft3(C<T> (&v0)[E], C<T> (&v1)[E], C<T> (&v2)[E], int t, C<T>* lds0,
                                     C<T>* lds1, C<T>* lds2, int LS, TW tw)
{
    if constexpr (N > 1) fft3_stage<T, N, E, DIR, 1, TW>(v0, v1, v2, t, lds0, lds1, lds2, LS, tw);
}

// Full FFT.  All threads of the workgroup must call this together (it
// contains workgroup barriers whenever N > E).  tw is the twiddle source
// zeta_N^j: a pointer to tw_N in global memory, or any type with the same
// `tw + offset` and `tw[j]` operations (LdsTw below).
template <typename T, int N, int E, int DIR, typename TW>
__device__ __forceinline__ void fft(C<T> (&v)[E], int t, C<T>* lds, int LS, TW tw)
{
    static_assert(N % E == 0, "E must divide N");
    if constexpr (N > 1) fft_stage<T, N, E, DIR, 1, TW>(v, t, lds, LS, tw);
}

// The same transform over two exchange buffers used in turn (rows, LS = 1,
// G > 64): stage s writes the buffer that stage s - 1 did not read from, so
// one barrier per stage suffices -- every wave has finished reading that
// buffer (at stage s - 2) before it arrived at the barrier of stage s - 1.
// One barrier at the end lets the caller reuse both buffers.
template <typename T, int N, int E, int DIR, int NS, typename TW>
__device__ __forceinline__ void fft_pp_stage(C<T> (&v)[E], int t, C<T>* lds, C<T>* ldsn, TW tw)
{
    constexpr int R = (N / NS < E) ? (N / NS) : E;
    constexpr bool LAST = (NS * R == N);
    constexpr int G = N / E;
    constexpr int Q = E / R;
    static_assert(E % R == 0 && R >= 2, "radix must divide the per-thread element count");
    int zoff = 0;
    asm volatile("" : "+s"(zoff));
    asm volatile("" : "+v"(t));
    const TW tws = tw + zoff;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = t + q * G;
        const int k = b & (NS - 1);
        C<T> u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[q + r * Q];
        if constexpr (NS > 1) {
            const int ks = k * (N / (NS * R));
#pragma unroll
            for (int r = 1; r < R; ++r) u[r] = mulw<DIR>(u[r], tws[r * ks]);
        }
        DFT<R, DIR, T>::run(u);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q + r * Q] = u[r];
        } else {
            C<T>* wp = lds + lpad((b - k) * R + k);
#pragma unroll
            for (int r = 0; r < R; ++r) wp[r * NS + ((r * NS) >> 4)] = u[r];
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
        const C<T>* rp = lds + lpad(t);
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = rp[i * G + ((i * G) >> 4)];
        fft_pp_stage<T, N, E, DIR, NS * R, TW>(v, t, ldsn, lds, tw);
    }
}

template <typename T, int N, int E, int DIR, typename TW>
__device__ __forceinline__ void fft_pp(C<T> (&v)[E], int t, C<T>* lds0, C<T>* lds1, TW tw)
{
    static_assert(N % E == 0 && N / E > 64, "ping-pong exchanges serve workgroup-wide transforms");
    fft_pp_stage<T, N, E, DIR, 1, TW>(v, t, lds0, lds1, tw);
    __syncthreads();
}

// Two independent transforms advanced together (as fft2_stage) over two
// pairs of exchange buffers used in turn (as fft_pp_stage): one barrier per
// stage for both.
template <typename T, int N, int E, int DIR, int NS, typename TW>
__device__ __forceinline__ void fft2_pp_stage(C<T> (&v0)[E], C<T> (&v1)[E], int t, C<T>* l0, C<T>* l1, C<T>* n0,
                                              C<T>* n1, TW tw)
{
    constexpr int R = (N / NS < E) ? (N / NS) : E;
    constexpr bool LAST = (NS * R == N);
    constexpr int G = N / E;
    constexpr int Q = E / R;
    int zoff = 0;
    asm volatile("" : "+s"(zoff));
    asm volatile("" : "+v"(t));
    const TW tws = tw + zoff;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = t + q * G;
        const int k = b & (NS - 1);
        C<T> u0[R], u1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            u0[r] = v0[q + r * Q];
            u1[r] = v1[q + r * Q];
        }
        if constexpr (NS > 1) {
            const int ks = k * (N / (NS * R));
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const auto w = tws[r * ks];
                u0[r] = mulw<DIR>(u0[r], w);
                u1[r] = mulw<DIR>(u1[r], w);
            }
        }
        DFT<R, DIR, T>::run(u0);
        DFT<R, DIR, T>::run(u1);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                v0[q + r * Q] = u0[r];
                v1[q + r * Q] = u1[r];
            }
        } else {
            const int wb = lpad((b - k) * R + k);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                l0[wb + r * NS + ((r * NS) >> 4)] = u0[r];
                l1[wb + r * NS + ((r * NS) >> 4)] = u1[r];
            }
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
        const int rb = lpad(t);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            v0[i] = l0[rb + i * G + ((i * G) >> 4)];
            v1[i] = l1[rb + i * G + ((i * G) >> 4)];
        }
        fft2_pp_stage<T, N, E, DIR, NS * R, TW>(v0, v1, t, n0, n1, l0, l1, tw);
    }
}

template <typename T, int N, int E, int DIR, typename TW>
__device__ __forceinline__ void fft2_pp(C<T> (&v0)[E], C<T> (&v1)[E], int t, C<T>* l0, C<T>* l1, C<T>* n0,
                                        C<T>* n1, TW tw)
{
    static_assert(N % E == 0 && N / E > 64, "ping-pong exchanges serve workgroup-wide transforms");
    fft2_pp_stage<T, N, E, DIR, 1, TW>(v0, v1, t, l0, l1, n0, n1, tw);
    __syncthreads();
}

// Compile-time loop: f(std::integral_constant<int, i>{}) for i = 0..n-1.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int n, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    static_for_impl(f, std::make_integer_sequence<int, n>{});
}

// A zero the compiler cannot see through.  Adding it to a pointer keeps
// loads through that pointer at the point of use (no hoisting, no merging
// with identical loads elsewhere), trading a cached reload for registers.
__device__ __forceinline__ int opaque_zero()
{
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

// Elements per thread for an FFT of size N: 16 complex64 or 8 complex128
// values (32 VGPRs), so that three such arrays plus butterfly temporaries fit
// the 256-VGPR budget of two waves per SIMD.
#ifndef IMPCONV_EMAX_F32
#define IMPCONV_EMAX_F32 16
#endif
#ifndef IMPCONV_EMAX_F64
#define IMPCONV_EMAX_F64 8
#endif
template <typename T>
__host__ __device__ constexpr int fft_E(int N)
{
    constexpr int emax = sizeof(T) == 4 ? IMPCONV_EMAX_F32 : IMPCONV_EMAX_F64;
    return N < emax ? N : emax;
}

// Offset of tw_N inside the concatenated table of all power-of-two sizes.
__host__ __device__ constexpr int64_t tw_off(int64_t N) { return N - 1; }

}  // namespace impconv
