// rowconv.hpp -- fused 1D implicitly dealiased convolutions, one FFT group per
// row, everything between the HBM load of the inputs and the HBM store of the
// result kept in registers and LDS.
//
// A "row" is one independent 1D convolution: the contiguous inputs f_i, g_i
// (i < M, the dot-product width of Sec. 3.3) and the contiguous output h.
// Rows are batch entries in 1D and the innermost-axis lines of the
// multidimensional convolutions.  The logical length m of a row may be any
// value up to the kernel's padded size; entries at and beyond m read as zero,
// which leaves the dealiased sum for k < m unchanged (zero padding of the
// inputs beyond m contributes no terms).
#pragma once
#include "fft_wg.hpp"

namespace impconv {

enum : uint32_t {
    kRevF = 1u << 1,    // read f reversed within its logical length
    kConjG = 1u << 2,   // read g conjugated
    kRevOut = 1u << 3,  // write h reversed within its logical length
    kHermAdj = 1u << 5, // Hermitian adjoint: f_0 read as 2 Re f_0, h_0 stored halved (real)
    kComp = 1u << 7,    // complex64: compensated twiddle products (tables tw + twlo)
};

struct RowArgs {
    const void* f;
    const void* g;
    const void* e;  // third input of the ternary convolution
    void* h;
    int64_t nrows;
    int64_t m;      // logical input length (all rows, unless row_m is given)
    int64_t m_out;  // logical output length (cyclic kernel only)
    int64_t M;      // dot-product width
    int64_t f_row, f_i, g_row, g_i, e_row, h_row;  // element strides
    const int64_t* row_off;  // optional per-row element offset (f, g, h share it)
    const int64_t* row_m;    // optional per-row logical length
    uint32_t flags;
    double scale;            // cyclic kernel output scale
    const void* tw;          // concatenated zeta_N^j tables, N = 1, 2, 4, ...
    const void* tw3;         // concatenated zeta_{3N}^j tables (j < N)
    int64_t h_pad;           // Hermitian rows: stored output length; entries m..h_pad-1 are zeroed
    const void* twq;         // general p/q rule: zeta_{q NP}^j, j < q NP
    const void* twlo;        // complex64 low parts of the tw tables (compensated products)
    int q;                   // general p/q rule: residues
};

// Elements per thread of the row kernels: family 0 (complex, cyclic) keeps
// fft_E values per thread; family 1 (Hermitian, ternary), whose prologues
// read four inputs per element and keep five arrays live, keeps half as many.
template <typename T, int FAM>
__host__ __device__ constexpr int row_E(int N)
{
    // at least 2 (a radix-1 stage would make no progress) unless N == 1, and
    // large enough that one group fits a 1024-thread workgroup
    const int e = FAM == 0 ? fft_E<T>(N) : (fft_E<T>(N) / 2 >= 2 ? fft_E<T>(N) / 2 : fft_E<T>(N));
    return N / e > 1024 ? N / 1024 : e;
}
// Threads per group and groups per block for a row kernel of FFT size N.
template <typename T, int FAM = 0> __host__ __device__ constexpr int row_G(int N) { return N / row_E<T, FAM>(N); }
template <typename T, int FAM = 0> __host__ __device__ constexpr int row_GPB(int N)
{
    return row_G<T, FAM>(N) >= 128 ? 1 : 128 / row_G<T, FAM>(N);
}
template <typename T, int FAM = 0> __host__ __device__ constexpr int row_block(int N)
{
    return row_G<T, FAM>(N) * row_GPB<T, FAM>(N);
}
template <typename T, int FAM = 0> __host__ __device__ constexpr int row_lds(int N)
{
    return N > row_E<T, FAM>(N) ? lpad_size(N) : 1;
}

// Waves per SIMD the row kernels are compiled for: the register budget of
// each wave is 512 / waves.  Small blocks would otherwise let the compiler
// take all 512 registers and leave one wave per SIMD to hide HBM latency.
template <typename T>
__host__ __device__ constexpr int row_waves(int)
{
    return 2;
}

// Whether narr live arrays of E complex values fit the VGPR budget a block
// of `threads` leaves each wave (512 per SIMD lane, shared by the waves a
// SIMD holds).  If not, the kernel accumulates its result in HBM instead of
// registers.
template <typename T>
__host__ __device__ constexpr bool regs_fit(int narr, int E, int threads)
{
    int waves = (threads + 63) / 64;
    int per_simd = (waves + 3) / 4;
    if (per_simd < row_waves<T>(0)) per_simd = row_waves<T>(0);
    int budget = 512 / per_simd;
    int need = narr * E * 2 * int(sizeof(T) / 4);
    return need * 5 <= budget * 4;  // leave ~20% for addresses and temporaries
}

struct RowCtx {
    int64_t row, of, og, oe, oh;
    int m;  // logical length of this row (0 for the padding groups past nrows)
    bool act;
};

// Twiddle source of the tw tables at offset off: a plain pointer, or with
// COMP the (high, low) pair of tables for compensated products.
template <typename T, bool COMP>
using TwSrc = std::conditional_t<COMP, CompTw<T>, const C<T>*>;
template <typename T, bool COMP>
__device__ __forceinline__ TwSrc<T, COMP> tw_src(const RowArgs& a, int64_t off)
{
    if constexpr (COMP) return CompTw<T>{(const C<T>*)a.tw + off, (const C<T>*)a.twlo + off};
    else return (const C<T>*)a.tw + off;
}

// Rows past nrows (the idle groups of the last block) read row 0 with
// length 0, so every load below stays in bounds and yields zero.
__device__ __forceinline__ RowCtx row_ctx(const RowArgs& a, int64_t row)
{
    RowCtx c;
    c.row = row;
    c.act = row < a.nrows;
    const int64_t r = c.act ? row : 0;
    c.m = c.act ? (int)a.m : 0;
    c.of = r * a.f_row;
    c.og = r * a.g_row;
    c.oe = r * a.e_row;
    c.oh = r * a.h_row;
    if (a.row_off) c.of = c.og = c.oe = c.oh = a.row_off[r];
    if (c.act && a.row_m) c.m = (int)a.row_m[r];
    return c;
}

// U[j] for j < m, else 0, without a branch: the load always executes at a
// clamped in-bounds index and the value is selected afterwards.  (A guarded
// load per element would put every element in its own basic block, which
// defeats instruction scheduling and forces register spills.)
template <typename T>
__device__ __forceinline__ C<T> ldz(const C<T>* U, int j, int m)
{
    const bool ok = unsigned(j) < unsigned(m);  // 0 <= j < m
    const C<T> v = U[ok ? j : 0];
    return ok ? v : zero<T>();
}

// The same value, loaded unconditionally and masked.  With the condition in
// view the compiler may turn ldz's selection back into a load under the
// condition (a branch per element); here the clamped index and the
// all-ones / zero mask pass through an empty asm statement, so the load
// always executes, and the mask clears the bits (+0 whatever U[0] holds).
template <typename T>
__device__ __forceinline__ T mask_bits(T x, int mask)
{
    if constexpr (sizeof(T) == 4) {
        return __uint_as_float(__float_as_uint(x) & unsigned(mask));
    } else {
        return __longlong_as_double(__double_as_longlong(x) & (long long)mask);
    }
}
template <typename T>
__device__ __forceinline__ C<T> ldz_masked(const C<T>* U, int j, int m)
{
    const bool ok = unsigned(j) < unsigned(m);  // 0 <= j < m
    int jj = ok ? j : 0;
    int mask = ok ? -1 : 0;
    asm volatile("" : "+v"(jj), "+v"(mask));
    const C<T> v = U[jj];
    return C<T>{mask_bits(v.re, mask), mask_bits(v.im, mask)};
}

// ======================================================================
// Complex 1D convolution, 1/2 padding rule (Sec. 2.1, fftpadBackward /
// fftpadForward / cconv): the 2N-padded backward transform splits into two
// size-N transforms of zeta_{2N}^{rk} f_k (r = 0, 1); their products are
// transformed forward and recombined as (F_0 + zeta_{2N}^{-k} F_1) / 2N.
// ======================================================================
// One M = 1 row by one group: f and g are read once; both residues r = 0, 1
// are formed from the same registers (x0 = f, x1 = zeta_{2N}^k f, likewise
// g) and transformed together, through two exchange buffers (fft2, DUAL) or
// one after the other through one.  E values per thread (G = N / E threads
// per row, t < G).
template <typename T, int N, int E, bool DUAL, bool COMP>
__device__ __forceinline__ void conv_complex_row(const RowArgs& a, const RowCtx& c, int t, C<T>* lds,
                                                 C<T>* lds1, TwSrc<T, COMP> twN, TwSrc<T, COMP> tw2N)
{
    constexpr int G = N / E;
    const C<T>* F = (const C<T>*)a.f + c.of;
    const C<T>* Gp = (const C<T>*)a.g + c.og;
    C<T>* H = (C<T>*)a.h + c.oh;
    const bool revf = a.flags & kRevF, cjg = a.flags & kConjG, revo = a.flags & kRevOut;
    const T s = T(1) / T(2 * N);
    auto pair = [&](auto& a0, auto& a1, auto dir) {
        constexpr int D = decltype(dir)::value;
        if constexpr (DUAL) {
            fft2<T, N, E, D>(a0, a1, t, lds, lds1, 1, twN);
        } else {
            fft<T, N, E, D>(a0, t, lds, 1, twN);
            fft<T, N, E, D>(a1, t, lds, 1, twN);
        }
    };
    C<T> x0[E], x1[E];
    {
        const int z = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * G;
            x0[e] = ldz(F + z, revf ? c.m - 1 - k : k, c.m);
            x1[e] = mulw<+1>(x0[e], tw2N[k + z]);
        }
    }
    pair(x0, x1, std::integral_constant<int, +1>{});
    {
        C<T> y[E];
        const int z = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            C<T> gv = ldz(Gp + z, t + e * G, c.m);
            y[e] = cjg ? conj(gv) : gv;
        }
        C<T> y1[E];
#pragma unroll
        for (int e = 0; e < E; ++e) y1[e] = mulw<+1>(y[e], tw2N[t + e * G + z]);
        pair(y, y1, std::integral_constant<int, +1>{});
#pragma unroll
        for (int e = 0; e < E; ++e) {
            x0[e] = x0[e] * y[e];
            x1[e] = x1[e] * y1[e];
        }
    }
    pair(x0, x1, std::integral_constant<int, -1>{});
    const int z = opaque_zero();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * G;
        if (k < c.m) H[revo ? c.m - 1 - k : k] = scale(x0[e] + mulw<-1>(x1[e], tw2N[k + z]), s);
    }
}

#ifndef IMPCONV_ROW_TW_LDS
#define IMPCONV_ROW_TW_LDS 1
#endif
#ifndef IMPCONV_ROW_TW_LDS_MAX
#define IMPCONV_ROW_TW_LDS_MAX (40 * 1024)
#endif
template <typename T, int N, bool ACCG, bool MD, bool COMP = false>
__global__ void __launch_bounds__(row_block<T>(N), row_waves<T>(N))
k_conv1d_complex(RowArgs a)
{
    constexpr int E = fft_E<T>(N), G = N / E, GPB = row_GPB<T>(N), LDSN = row_lds<T>(N);
    // second exchange buffer for the paired transforms when both fit in LDS
    constexpr bool DUAL = !MD && 2 * GPB * LDSN * int(sizeof(C<T>)) <= 160 * 1024;
    __shared__ C<T> sh[(DUAL ? 2 : 1) * GPB * LDSN];
    static_assert(sizeof(sh) <= 160 * 1024, "LDS footprint exceeds 160 KB");
    // short rows, several per workgroup: the twiddle tables a row uses
    // (zeta_N^j and zeta_2N^k, j, k < N) are copied into LDS once per
    // workgroup, where every transform stage and residue shift reads them,
    // where the workgroup's LDS stays within IMPCONV_ROW_TW_LDS_MAX bytes
    constexpr bool TWL = IMPCONV_ROW_TW_LDS && !COMP && N >= 2 && GPB > 1 &&
                         int(sizeof(sh)) + 2 * N * int(sizeof(C<T>)) <= IMPCONV_ROW_TW_LDS_MAX;
    __shared__ C<T> twl[TWL ? 2 * N : 1];
    const int grp = threadIdx.x / G, t = threadIdx.x % G;
    const RowCtx c = row_ctx(a, (int64_t)blockIdx.x * GPB + grp);
    C<T>* lds = sh + grp * LDSN;
    TwSrc<T, COMP> twN = tw_src<T, COMP>(a, tw_off(N));
    TwSrc<T, COMP> tw2N = tw_src<T, COMP>(a, tw_off(2 * N));
    if constexpr (TWL) {
        for (int j = threadIdx.x; j < 2 * N; j += blockDim.x) twl[j] = j < N ? twN[j] : tw2N[j - N];
        __syncthreads();
        twN = twl;
        tw2N = twl + N;
    }

    if constexpr (!MD) {
        conv_complex_row<T, N, E, DUAL, COMP>(a, c, t, lds, DUAL ? sh + (GPB + grp) * LDSN : lds, twN, tw2N);
        return;
    }

    const C<T>* F = (const C<T>*)a.f + c.of;
    const C<T>* Gp = (const C<T>*)a.g + c.og;
    C<T>* H = (C<T>*)a.h + c.oh;
    const bool revf = a.flags & kRevF, cjg = a.flags & kConjG, revo = a.flags & kRevOut;
    const T s = T(1) / T(2 * N);

    C<T> acc[ACCG ? 1 : E];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        C<T> P[E];
        for (int64_t i = 0; i < a.M; ++i) {
            C<T> x[E], y[E];
            const int z = opaque_zero();
            const C<T>* Fz = F + z;
            const C<T>* Gz = Gp + z;
            const TwSrc<T, COMP> Wz = tw2N + z;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * G;
                C<T> fv = ldz(Fz + i * a.f_i, revf ? c.m - 1 - k : k, c.m);
                C<T> gv = ldz(Gz + i * a.g_i, k, c.m);
                if (cjg) gv = conj(gv);
                if (r) {
                    const auto w = Wz[k];
                    fv = mulw<+1>(fv, w);
                    gv = mulw<+1>(gv, w);
                }
                x[e] = fv;
                y[e] = gv;
            }
            fft<T, N, E, +1>(x, t, lds, 1, twN);
            fft<T, N, E, +1>(y, t, lds, 1, twN);
#pragma unroll
            for (int e = 0; e < E; ++e) P[e] = i > 0 ? P[e] + x[e] * y[e] : x[e] * y[e];
        }
        fft<T, N, E, -1>(P, t, lds, 1, twN);
        const TwSrc<T, COMP> Wo = tw2N + opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * G;
            const C<T> v = r ? mulw<-1>(P[e], Wo[k]) : P[e];
            if constexpr (ACCG) {
                if (k < c.m) {
                    C<T>* hp = H + (revo ? c.m - 1 - k : k);
                    *hp = r ? *hp + scale(v, s) : scale(v, s);
                }
            } else {
                acc[e] = r ? acc[e] + v : v;
            }
        }
    }
    if constexpr (!ACCG) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * G;
            if (k < c.m) H[revo ? c.m - 1 - k : k] = scale(acc[e], s);
        }
    }
}

// One M = 1 row per 1024-thread workgroup for the lengths whose transform
// takes G = 1024 threads (complex128 N = 8192), where the paired form above
// (both residues of f and g live at once) exceeds the 128 registers per
// thread such a workgroup leaves and spills.  The residues run one
// after the other through one exchange buffer: residue 0 is transformed,
// multiplied and transformed back; then residue 1's entries of f and g are
// read (from the caches) before residue 0's share of h_k is stored, so that
// h may be f or g; residue 1 follows and its share is added to the stored
// one (each thread reads back only what it stored itself).
template <typename T, int N>
__host__ __device__ constexpr bool complex_serial()
{
    return N / fft_E<T>(N) == 1024;
}

template <typename T, int N>
__global__ void __launch_bounds__(1024, 1)
k_conv1d_complex_serial(RowArgs a)
{
    constexpr int E = fft_E<T>(N), G = N / E, LDSN = lpad_size(N);
    static_assert(G == 1024, "serial complex rows take one 1024-thread workgroup per row");
    __shared__ C<T> lds[LDSN];
    static_assert(sizeof(lds) <= 160 * 1024, "LDS footprint exceeds 160 KB");
    const int t = threadIdx.x;
    const RowCtx c = row_ctx(a, (int64_t)blockIdx.x);
    const C<T>* twN = (const C<T>*)a.tw + tw_off(N);
    const C<T>* tw2N = (const C<T>*)a.tw + tw_off(2 * N);
    const C<T>* F = (const C<T>*)a.f + c.of;
    const C<T>* Gp = (const C<T>*)a.g + c.og;
    C<T>* H = (C<T>*)a.h + c.oh;
    const bool revf = a.flags & kRevF, cjg = a.flags & kConjG, revo = a.flags & kRevOut;
    const T s = T(1) / T(2 * N);
    // a fresh copy of t per phase keeps the addresses from being computed
    // once and held across the whole kernel
    auto fresh = [](int v) {
        asm volatile("" : "+v"(v));
        return v;
    };
    auto load_f = [&](C<T>* v) {
        const int tt = fresh(t), z = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = tt + e * G;
            v[e] = ldz(F + z, revf ? c.m - 1 - k : k, c.m);
        }
    };
    auto load_g = [&](C<T>* v) {
        const int tt = fresh(t), z = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const C<T> u = ldz(Gp + z, tt + e * G, c.m);
            v[e] = cjg ? conj(u) : u;
        }
    };
    // multiply by zeta_{2N}^{+-k}: the shift of residue 1
    auto shift = [&](C<T>* v, bool inv) {
        const int tt = fresh(t), z = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const C<T> w = tw2N[tt + e * G + z];
            v[e] = inv ? mulw<-1>(v[e], w) : mulw<+1>(v[e], w);
        }
    };
    auto store = [&](const C<T>* v, bool add) {
        const int tt = fresh(t);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = tt + e * G;
            if (k < c.m) {
                C<T>* hp = H + (revo ? c.m - 1 - k : k);
                const C<T> u = scale(v[e], s);
                *hp = add ? *hp + u : u;
            }
        }
    };
    C<T> x[E];
    {
        // residue 0
        C<T> y[E];
        load_f(x);
        fft<T, N, E, +1>(x, t, lds, 1, twN);
        load_g(y);
        fft<T, N, E, +1>(y, t, lds, 1, twN);
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = x[e] * y[e];
        fft<T, N, E, -1>(x, t, lds, 1, twN);
    }
    C<T> x1[E], y1[E];
    load_f(x1);
    load_g(y1);
    // every thread's reads of the row have completed before any thread
    // stores into it
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    store(x, false);
    // residue 1
    shift(x1, false);
    fft<T, N, E, +1>(x1, t, lds, 1, twN);
    shift(y1, false);
    fft<T, N, E, +1>(y1, t, lds, 1, twN);
#pragma unroll
    for (int e = 0; e < E; ++e) x1[e] = x1[e] * y1[e];
    fft<T, N, E, -1>(x1, t, lds, 1, twN);
    shift(x1, true);
    store(x1, true);
}

// ======================================================================
// Complex 1D convolution with general p/q padding (Sec. 2.4).  The inputs
// (zero beyond m) are taken as P blocks of NP values, P NP >= m, and padded
// implicitly to Nq = q NP with Nq >= 2m - 1, so that the cyclic convolution
// of length Nq is the linear one on k < m.  For each residue r < q
//   x_r[s] = zeta_Nq^{rs} sum_{t<P} zeta_q^{rt} f_{t NP + s},  s < NP,
// is transformed backward at size NP (likewise g), the products, summed over
// the M terms, are transformed forward, and
//   Nq h_{t NP + s} = sum_{r<q} zeta_q^{-rt} zeta_Nq^{-rs} V_r[s].
// q NP transforms of size NP replace the 2N of size N = 2^ceil(log2 m) of
// the 1/2 rule.  The inputs are re-read for each residue (from cache); the
// P output blocks accumulate in registers.
// ======================================================================
template <typename T, int NP, int P>
__global__ void __launch_bounds__((row_block<T, 1>(NP)), row_waves<T>(NP))
k_conv1d_pq(RowArgs a)
{
    constexpr int E = row_E<T, 1>(NP), G = NP / E, GPB = row_GPB<T, 1>(NP), LDSN = row_lds<T, 1>(NP);
    constexpr bool DUAL = 2 * GPB * LDSN * int(sizeof(C<T>)) <= 160 * 1024;
    __shared__ C<T> sh[(DUAL ? 2 : 1) * GPB * LDSN];
    static_assert(sizeof(sh) <= 160 * 1024, "LDS footprint exceeds 160 KB");
    const int grp = threadIdx.x / G, t = threadIdx.x % G;
    const RowCtx c = row_ctx(a, (int64_t)blockIdx.x * GPB + grp);
    C<T>* lds = sh + grp * LDSN;
    C<T>* lds1 = DUAL ? sh + (GPB + grp) * LDSN : lds;
    const C<T>* twN = (const C<T>*)a.tw + tw_off(NP);
    const C<T>* twq = (const C<T>*)a.twq;
    const int q = a.q, m = c.m;
    const C<T>* F = (const C<T>*)a.f + c.of;
    const C<T>* Gp = (const C<T>*)a.g + c.og;
    C<T>* H = (C<T>*)a.h + c.oh;
    const bool revf = a.flags & kRevF, cjg = a.flags & kConjG, revo = a.flags & kRevOut;

    C<T> acc[P][E];
    for (int r = 0; r < q; ++r) {
        // zeta_q^{rt} = zeta_Nq^{(rt mod q) NP} for the P blocks (wave uniform)
        C<T> zq[P];
        {
            int j = 0;
#pragma unroll
            for (int b = 0; b < P; ++b) {
                zq[b] = twq[j * NP];
                j += r;
                if (j >= q) j -= q;
            }
        }
        C<T> w[E];  // zeta_Nq^{rs}, s = t + eG
        {
            const int z = opaque_zero();
#pragma unroll
            for (int e = 0; e < E; ++e) w[e] = twq[r * (t + e * G) + z];
        }
        C<T> Pr[E];
        for (int64_t i = 0; i < a.M; ++i) {
            C<T> x[E], y[E];
            const int z = opaque_zero();
            const C<T>* Fi = F + i * a.f_i + z;
            const C<T>* Gi = Gp + i * a.g_i + z;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int s = t + e * G;
                C<T> sf = ldz(Fi, revf ? m - 1 - s : s, m);
#pragma unroll
                for (int b = 1; b < P; ++b) {
                    const int k = b * NP + s;
                    sf = sf + zq[b] * ldz(Fi, revf ? m - 1 - k : k, m);
                }
                x[e] = sf * w[e];
            }
            // keep the two inputs' loads apart: the P E values of one input
            // in flight at a time
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int s = t + e * G;
                auto gld = [&](int k) {  // g_k, conjugated before the block weights
                    const C<T> v = ldz(Gi, k, m);
                    return cjg ? conj(v) : v;
                };
                C<T> sg = gld(s);
#pragma unroll
                for (int b = 1; b < P; ++b) sg = sg + zq[b] * gld(b * NP + s);
                y[e] = sg * w[e];
            }
            if constexpr (DUAL) {
                fft2<T, NP, E, +1>(x, y, t, lds, lds1, 1, twN);
            } else {
                fft<T, NP, E, +1>(x, t, lds, 1, twN);
                fft<T, NP, E, +1>(y, t, lds, 1, twN);
            }
#pragma unroll
            for (int e = 0; e < E; ++e) Pr[e] = i > 0 ? Pr[e] + x[e] * y[e] : x[e] * y[e];
        }
        fft<T, NP, E, -1>(Pr, t, lds, 1, twN);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const C<T> v = mulc(Pr[e], w[e]);  // zeta_Nq^{-rs} V_r[s]
#pragma unroll
            for (int b = 0; b < P; ++b) {
                const C<T> u = mulc(v, zq[b]);  // zeta_q^{-rb}
                acc[b][e] = r > 0 ? acc[b][e] + u : u;
            }
        }
    }
    const T sc = T(1) / T(q * NP);
#pragma unroll
    for (int b = 0; b < P; ++b) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = b * NP + t + e * G;
            if (k < m) H[revo ? m - 1 - k : k] = scale(acc[b][e], sc);
        }
    }
}

// ======================================================================
// Plain cyclic convolution of size N (no dealiasing): the building block of
// the explicitly padded comparator (inputs already zero padded in HBM) and
// the middle pass of the multi-pass large-N convolutions.
// h_k = scale * sum_i IFFT(FFT(f_i) FFT(g_i))_k, k < m_out.
// ======================================================================
template <typename T, int N>
__global__ void __launch_bounds__(row_block<T>(N), row_waves<T>(N))
k_conv1d_cyclic(RowArgs a)
{
    constexpr int E = fft_E<T>(N), G = N / E, GPB = row_GPB<T>(N), LDSN = row_lds<T>(N);
    __shared__ C<T> sh[GPB * LDSN];
    static_assert(sizeof(sh) <= 160 * 1024, "LDS footprint exceeds 160 KB");
    const int grp = threadIdx.x / G, t = threadIdx.x % G;
    const RowCtx c = row_ctx(a, (int64_t)blockIdx.x * GPB + grp);
    C<T>* lds = sh + grp * LDSN;
    const C<T>* twN = (const C<T>*)a.tw + tw_off(N);
    // several rows per workgroup: the stage table (N entries) is copied
    // into LDS once per workgroup, as in k_conv1d_complex
    constexpr bool TWL = IMPCONV_ROW_TW_LDS && GPB > 1 && N > E &&
                         int(sizeof(sh)) + N * int(sizeof(C<T>)) <= IMPCONV_ROW_TW_LDS_MAX;
    __shared__ C<T> twl[TWL ? N : 1];
    if constexpr (TWL) {
        for (int j = threadIdx.x; j < N; j += blockDim.x) twl[j] = twN[j];
        __syncthreads();
        twN = twl;
    }
    const C<T>* F = (const C<T>*)a.f + c.of;
    const C<T>* Gp = (const C<T>*)a.g + c.og;
    C<T>* H = (C<T>*)a.h + c.oh;
    C<T> P[E];
#pragma unroll
    for (int e = 0; e < E; ++e) P[e] = zero<T>();
    for (int64_t i = 0; i < a.M; ++i) {
        C<T> x[E], y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * G;
            x[e] = ldz(F + i * a.f_i, k, c.m);
            y[e] = ldz(Gp + i * a.g_i, k, c.m);
        }
        fft<T, N, E, +1>(x, t, lds, 1, twN);
        fft<T, N, E, +1>(y, t, lds, 1, twN);
#pragma unroll
        for (int e = 0; e < E; ++e) P[e] = P[e] + x[e] * y[e];
    }
    fft<T, N, E, -1>(P, t, lds, 1, twN);
    const T s = T(a.scale);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * G;
        if (c.act && k < a.m_out) H[k] = scale(P[e], s);  // stores may branch
    }
}

// Value P_{(n - k) mod n} of the sequence whose position t + e*G this thread
// holds in P[e]; used by the real-to-complex post-processing, which pairs
// frequency k with n - k.  Goes through LDS unless one thread holds it all.
template <typename T, int NC, int E>
__device__ __forceinline__ void mirror(const C<T> (&P)[E], C<T> (&Pm)[E], int t, C<T>* lds)
{
    constexpr int G = NC / E;
    if constexpr (G == 1) {
#pragma unroll
        for (int e = 0; e < E; ++e) Pm[e] = P[(NC - e) & (NC - 1)];
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) lds[lpad(t + e * G)] = P[e];
        xsync<G>(1);
#pragma unroll
        for (int e = 0; e < E; ++e) Pm[e] = lds[lpad((NC - (t + e * G)) & (NC - 1))];
        xsync<G>(1);
    }
}

// mirror of two or three sequences through as many disjoint LDS buffers,
// with one pair of barriers
template <typename T, int NC, int E>
__device__ __forceinline__ void mirror2(const C<T> (&A)[E], C<T> (&Am)[E], const C<T> (&B)[E], C<T> (&Bm)[E],
                                        int t, C<T>* lds0, C<T>* lds1)
{
    constexpr int G = NC / E;
    if constexpr (G == 1) {
        mirror<T, NC, E>(A, Am, t, lds0);
        mirror<T, NC, E>(B, Bm, t, lds1);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            lds0[lpad(t + e * G)] = A[e];
            lds1[lpad(t + e * G)] = B[e];
        }
        xsync<G>(1);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = lpad((NC - (t + e * G)) & (NC - 1));
            Am[e] = lds0[j];
            Bm[e] = lds1[j];
        }
        xsync<G>(1);
    }
}
template <typename T, int NC, int E>
__device__ __forceinline__ void mirror3(const C<T> (&A)[E], C<T> (&Am)[E], const C<T> (&B)[E], C<T> (&Bm)[E],
                                        const C<T> (&D)[E], C<T> (&Dm)[E], int t, C<T>* lds0, C<T>* lds1,
                                        C<T>* lds2)
{
    constexpr int G = NC / E;
    if constexpr (G == 1) {
        mirror<T, NC, E>(A, Am, t, lds0);
        mirror<T, NC, E>(B, Bm, t, lds1);
        mirror<T, NC, E>(D, Dm, t, lds2);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            lds0[lpad(t + e * G)] = A[e];
            lds1[lpad(t + e * G)] = B[e];
            lds2[lpad(t + e * G)] = D[e];
        }
        xsync<G>(1);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = lpad((NC - (t + e * G)) & (NC - 1));
            Am[e] = lds0[j];
            Bm[e] = lds1[j];
            Dm[e] = lds2[j];
        }
        xsync<G>(1);
    }
}

// Spectrum V_k (k = 0..NC) of a real sequence v of length 2 NC from the
// size-NC forward FFT P of its packing z_l = v_{2l} + i v_{2l+1}:
// V_k = (P_k + conj P_{NC-k}) / 2 - i zeta_{2NC}^{-k} (P_k - conj P_{NC-k}) / 2.
template <typename T>
__device__ __forceinline__ C<T> r2c_post(C<T> p, C<T> pm, C<T> w2k)
{
    const C<T> ev = scale(p + conj(pm), T(0.5));
    const C<T> od = scale(p - conj(pm), T(0.5));
    return ev + muli<-1>(mulc(od, w2k));
}

// Packed input Z_k = (X_k + conj X_{NC-k}) + i zeta_{2NC}^k (X_k - conj X_{NC-k})
// whose size-NC backward FFT is x_{2l} + i x_{2l+1}, x the length-2NC real
// backward transform of the Hermitian half X_0..X_NC.
template <typename T>
__device__ __forceinline__ C<T> c2r_pre(C<T> xk, C<T> xmk, C<T> w2k)
{
    const C<T> cx = conj(xmk);
    return (xk + cx) + muli<+1>((xk - cx) * w2k);
}

// ======================================================================
// Centered Hermitian 1D convolution, 2/3 padding rule (Sec. 2.3).  The input
// half U_0..U_{N-1} (N = 2 NC >= m, zero beyond m) is implicitly padded to
// 3N.  For each residue r in {-1, 0, 1} the Hermitian sequence
//   w_{0,r} = U_0,  w_{k,r} = zeta_{3N}^{rk} (U_k + zeta_3^{-r} conj U_{N-k}),
// is transformed complex-to-real (packed into one size-NC complex FFT), the
// real products of the two inputs are transformed real-to-complex, and
//   3N H_k = sum_r zeta_{3N}^{-rk} V_r(k),  V_r(N-k) = conj V_r(k).
// ======================================================================
// zeta_3^{-R} and zeta_6^{-R} for R in {-1, 0, 1}
template <typename T, int R>
__device__ __forceinline__ C<T> z3m()
{
    const T h = T(0.86602540378443864676);
    return R == 0 ? C<T>{T(1), T(0)} : (R > 0 ? C<T>{T(-0.5), -h} : C<T>{T(-0.5), h});
}
template <typename T, int R>
__device__ __forceinline__ C<T> z6m()
{
    const T h = T(0.86602540378443864676);
    return R == 0 ? C<T>{T(1), T(0)} : (R > 0 ? C<T>{T(0.5), -h} : C<T>{T(0.5), h});
}

// zeta_{3N}^{R k}, 0 <= k < N, from the zeta_{3N}^j table
template <typename T, int R>
__device__ __forceinline__ C<T> zeta3N(const C<T>* tw3N, int k)
{
    if constexpr (R == 0) return C<T>{T(1), T(0)};
    const C<T> w = tw3N[k];
    return R > 0 ? w : conj(w);
}

// Packed c2r inputs of the three residues r = 0, +1, -1 at this thread's
// frequencies k = t + e G (0 <= k < NC), from one read of the Hermitian half
// U (length m, zero beyond).  Each thread loads U_k and U_{NC+k}; the mirrored
// values U_{NC-k} and U_{N-k} come from the thread holding NC - k through the
// exchange buffer.  With w_{k,r} = zeta_{3N}^{rk} (U_k + zeta_3^{-r} conj U_{N-k}),
// w_{0,r} = Re U_0 and the real w_{NC,r}, Z_{k,r} = c2r_pre(w_{k,r}, w_{NC-k,r}).
template <typename T, int NC, int E, bool PAIRED = false>
__device__ __forceinline__ void herm_build3(const C<T>* U, int m, int t, C<T>* lds, const C<T>* tw3N,
                                            const C<T>* twN, C<T> (&z0)[E], C<T> (&z1)[E], C<T> (&z2)[E],
                                            T dc = T(1), C<T>* lds1 = nullptr)
{
    constexpr int N = 2 * NC, G = NC / E;
    const T h3 = T(0.86602540378443864676), sq3 = T(1.73205080756887729353);
    C<T> lo[E], hi[E], lom[E], him[E];
    {
        const int z = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            lo[e] = ldz(U + z, t + e * G, m);
            hi[e] = ldz(U + z, NC + t + e * G, m);
        }
        // U_0 scaled by dc (the adjoint's doubled mean; only its real part is read)
        if (t == 0) lo[0] = scale(lo[0], dc);
    }
    // lom[e] = U_{(NC - k) mod NC}, him[e] = U_{NC + (NC - k) mod NC}
    if constexpr (PAIRED) {
        mirror2<T, NC, E>(lo, lom, hi, him, t, lds, lds1);
    } else {
        mirror<T, NC, E>(lo, lom, t, lds);
        mirror<T, NC, E>(hi, him, t, lds);
    }
    const int z = opaque_zero();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * G;
        const bool k0 = e == 0 && k == 0;
        const C<T> a = lo[e];                         // U_k
        const C<T> b = k0 ? zero<T>() : him[e];       // U_{N-k}
        const C<T> c = k0 ? hi[e] : lom[e];           // U_{NC-k}
        const C<T> d = hi[e];                         // U_{NC+k}
        const C<T> wk = tw3N[k + z], wc = tw3N[NC - k + z], w2 = twN[k + z];
        // r = 0
        C<T> p = a + conj(b), q = c + conj(d);
        if (k0) { p = C<T>{a.re, T(0)}; q = C<T>{T(2) * c.re, T(0)}; }
        z0[e] = c2r_pre(p, q, w2);
        // r = +1: zeta_3^{-1} = (-1/2, -sqrt3/2)
        const C<T> z3p{T(-0.5), -h3}, z3m{T(-0.5), h3};
        p = wk * (a + z3p * conj(b));
        q = wc * (c + z3p * conj(d));
        if (k0) { p = C<T>{a.re, T(0)}; q = C<T>{c.re - sq3 * c.im, T(0)}; }
        z1[e] = c2r_pre(p, q, w2);
        // r = -1: zeta_3^{+1}, conjugate shifts
        p = mulc(a + z3m * conj(b), wk);
        q = mulc(c + z3m * conj(d), wc);
        if (k0) { p = C<T>{a.re, T(0)}; q = C<T>{c.re + sq3 * c.im, T(0)}; }
        z2[e] = c2r_pre(p, q, w2);
    }
}

// This thread's entries of the Hermitian half U (length m, zero beyond):
// lo[e] = U_k, hi[e] = U_{NC+k}, k = t + e G.
template <typename T, int NC, int E>
__device__ __forceinline__ void herm_load(const C<T>* U, int m, int t, C<T> (&lo)[E], C<T> (&hi)[E])
{
    constexpr int G = NC / E;
    const int z = opaque_zero();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        lo[e] = ldz(U + z, t + e * G, m);
        hi[e] = ldz(U + z, NC + t + e * G, m);
    }
}

// a if c, else b, selected bit by bit: a select between two array elements
// may otherwise become a load from a selected address, which keeps the
// arrays in scratch memory
template <typename T>
__device__ __forceinline__ C<T> pick(bool c, C<T> a, C<T> b)
{
    int ma = c ? -1 : 0;
    asm volatile("" : "+v"(ma));
    const int mb = ~ma;
    return C<T>{mask_bits(a.re, ma) + mask_bits(b.re, mb), mask_bits(a.im, ma) + mask_bits(b.im, mb)};
}

// herm_build3 from entries already loaded by herm_load (lo, hi are consumed;
// the prefetching form of the row kernel).  BITSEL: the k = 0 selections
// through pick.
template <typename T, int NC, int E, bool PAIRED = false, bool BITSEL = false>
__device__ __forceinline__ void herm_build3_from(C<T> (&lo)[E], C<T> (&hi)[E], int t, C<T>* lds,
                                                 const C<T>* tw3N, const C<T>* twN, C<T> (&z0)[E],
                                                 C<T> (&z1)[E], C<T> (&z2)[E], T dc = T(1),
                                                 C<T>* lds1 = nullptr)
{
    constexpr int N = 2 * NC, G = NC / E;
    const T h3 = T(0.86602540378443864676), sq3 = T(1.73205080756887729353);
    C<T> lom[E], him[E];
    // U_0 scaled by dc (the adjoint's doubled mean; only its real part is read)
    if (t == 0) lo[0] = scale(lo[0], dc);
    // lom[e] = U_{(NC - k) mod NC}, him[e] = U_{NC + (NC - k) mod NC}
    if constexpr (PAIRED) {
        mirror2<T, NC, E>(lo, lom, hi, him, t, lds, lds1);
    } else {
        mirror<T, NC, E>(lo, lom, t, lds);
        mirror<T, NC, E>(hi, him, t, lds);
    }
    const int z = opaque_zero();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * G;
        const bool k0 = e == 0 && k == 0;
        const C<T> a = lo[e];                         // U_k
        const C<T> b = BITSEL ? pick(k0, zero<T>(), him[e]) : (k0 ? zero<T>() : him[e]);  // U_{N-k}
        const C<T> c = BITSEL ? pick(k0, hi[e], lom[e]) : (k0 ? hi[e] : lom[e]);          // U_{NC-k}
        const C<T> d = hi[e];                         // U_{NC+k}
        const C<T> wk = tw3N[k + z], wc = tw3N[NC - k + z], w2 = twN[k + z];
        // r = 0
        C<T> p = a + conj(b), q = c + conj(d);
        if (k0) { p = C<T>{a.re, T(0)}; q = C<T>{T(2) * c.re, T(0)}; }
        z0[e] = c2r_pre(p, q, w2);
        // r = +1: zeta_3^{-1} = (-1/2, -sqrt3/2)
        const C<T> z3p{T(-0.5), -h3}, z3m{T(-0.5), h3};
        p = wk * (a + z3p * conj(b));
        q = wc * (c + z3p * conj(d));
        if (k0) { p = C<T>{a.re, T(0)}; q = C<T>{c.re - sq3 * c.im, T(0)}; }
        z1[e] = c2r_pre(p, q, w2);
        // r = -1: zeta_3^{+1}, conjugate shifts
        p = mulc(a + z3m * conj(b), wk);
        q = mulc(c + z3m * conj(d), wc);
        if (k0) { p = C<T>{a.re, T(0)}; q = C<T>{c.re + sq3 * c.im, T(0)}; }
        z2[e] = c2r_pre(p, q, w2);
    }
}

// ======================================================================
// Centered Hermitian 1D convolution, 2/3 padding rule (Sec. 2.3).  The input
// half U_0..U_{N-1} (N = 2 NC >= m, zero beyond m) is implicitly padded to
// 3N.  For each residue r in {-1, 0, 1} the Hermitian sequence
//   w_{0,r} = U_0,  w_{k,r} = zeta_{3N}^{rk} (U_k + zeta_3^{-r} conj U_{N-k}),
// is transformed complex-to-real (packed into one size-NC complex FFT), the
// real products of the two inputs are transformed real-to-complex, and
//   3N H_k = sum_r zeta_{3N}^{-rk} V_r(k),  V_r(N-k) = conj V_r(k).
// Each input row is read once; the three residues are built from registers.
// ======================================================================
#ifndef IMPCONV_HERM_TW_LDS
#define IMPCONV_HERM_TW_LDS 1
#endif
#ifndef IMPCONV_HERM_TW_LDS_MAXNC
#define IMPCONV_HERM_TW_LDS_MAXNC 256
#endif
#ifndef IMPCONV_HERM_TW_LDS_BYTES
#define IMPCONV_HERM_TW_LDS_BYTES (40 * 1024)
#endif
#ifndef IMPCONV_TER_TW_LDS
#define IMPCONV_TER_TW_LDS 1
#endif
#ifndef IMPCONV_TER_TW_LDS_BYTES
#define IMPCONV_TER_TW_LDS_BYTES (40 * 1024)
#endif
template <typename T, int NC, bool MD>
__global__ void __launch_bounds__((row_block<T, 1>(NC)), row_waves<T>(NC))
k_conv1d_hermitian(RowArgs a)
{
    constexpr int N = 2 * NC;
    constexpr int E = row_E<T, 1>(NC), G = NC / E, GPB = row_GPB<T, 1>(NC), LDSN = row_lds<T, 1>(NC);
    // three exchange buffers per row (the three residues transformed
    // together) where they fit in LDS; else, for workgroup-wide transforms,
    // two used in turn (one barrier per stage) where those fit
    constexpr bool TRI = 3 * GPB * LDSN * int(sizeof(C<T>)) <= 160 * 1024;
    constexpr bool PP = !TRI && G > 64 && 2 * GPB * LDSN * int(sizeof(C<T>)) <= 160 * 1024;
    __shared__ C<T> sh[(TRI ? 3 : (PP ? 2 : 1)) * GPB * LDSN];
    static_assert(sizeof(sh) <= 160 * 1024, "LDS footprint exceeds 160 KB");
    // short rows: the twiddle tables a row uses (zeta_NC, zeta_N, zeta_3N:
    // NC + 2N values) are copied into LDS once per workgroup, so that every
    // transform stage and residue shift reads them there instead of waiting
    // on global loads; only where the workgroup's LDS stays within 40 KB
    // (four workgroups per compute unit)
    constexpr bool TWL = IMPCONV_HERM_TW_LDS && NC >= 2 && NC <= IMPCONV_HERM_TW_LDS_MAXNC &&
                         int(sizeof(sh)) + (NC + 2 * N) * int(sizeof(C<T>)) <= IMPCONV_HERM_TW_LDS_BYTES;
    __shared__ C<T> twl[TWL ? NC + 2 * N : 1];
    const int grp = threadIdx.x / G, t = threadIdx.x % G;
    const RowCtx c = row_ctx(a, (int64_t)blockIdx.x * GPB + grp);
    C<T>* lds = sh + grp * LDSN;
    C<T>* lds1 = (TRI || PP) ? sh + (GPB + grp) * LDSN : lds;
    C<T>* lds2 = TRI ? sh + (2 * GPB + grp) * LDSN : lds;
    const C<T>* twb = (const C<T>*)a.tw;
    const C<T>* twNC = twb + tw_off(NC);
    const C<T>* twN = twb + tw_off(N);
    const C<T>* tw3N = (const C<T>*)a.tw3 + tw_off(N);
    if constexpr (TWL) {
        for (int j = threadIdx.x; j < NC + 2 * N; j += blockDim.x)
            twl[j] = j < NC ? twNC[j] : (j < NC + N ? twN[j - NC] : tw3N[j - NC - N]);
        __syncthreads();
        twNC = twl;
        twN = twl + NC;
        tw3N = twl + NC + N;
    }
    const int m = c.m;
    auto fft3x = [&](C<T> (&v0)[E], C<T> (&v1)[E], C<T> (&v2)[E], auto dir) {
        constexpr int D = decltype(dir)::value;
        if constexpr (TRI) {
            fft3<T, NC, E, D>(v0, v1, v2, t, lds, lds1, lds2, 1, twNC);
        } else if constexpr (PP) {
            fft_pp<T, NC, E, D>(v0, t, lds, lds1, twNC);
            fft_pp<T, NC, E, D>(v1, t, lds, lds1, twNC);
            fft_pp<T, NC, E, D>(v2, t, lds, lds1, twNC);
        } else {
            fft<T, NC, E, D>(v0, t, lds, 1, twNC);
            fft<T, NC, E, D>(v1, t, lds, 1, twNC);
            fft<T, NC, E, D>(v2, t, lds, 1, twNC);
        }
    };
    C<T> P0[E], P1[E], P2[E];
    const int64_t nM = MD ? a.M : 1;
    // rows of up to 256 points: g's entries are loaded before f's
    // transforms, so that the loads are in flight while the wave computes
    // (measured faster on the 512 x 512 x 257 z rows: complex64 10.69 ->
    // 10.25 ms per step, complex128 16.73 -> 16.68 ms; in complex128 the
    // k = 0 selections go through pick, without which the compiler kept two
    // of the arrays in scratch memory and the kernel ran slower; in longer
    // rows the extra live registers cost more than the latency they hide)
    constexpr bool PREFETCH = NC <= 128;
    for (int64_t i = 0; i < nM; ++i) {
        C<T> x0[E], x1[E], x2[E], y0[E], y1[E], y2[E];
        const C<T>* Fi = (const C<T>*)a.f + c.of + i * a.f_i;
        const C<T>* Gi = (const C<T>*)a.g + c.og + i * a.g_i;
        const T dc = (a.flags & kHermAdj) ? T(2) : T(1);
        if constexpr (PREFETCH) {
            constexpr bool BS = sizeof(T) == 8;  // in complex64 pick costs registers (spills)
            C<T> lo[E], hi[E];
            herm_load<T, NC, E>(Fi, m, t, lo, hi);
            herm_build3_from<T, NC, E, TRI, BS>(lo, hi, t, lds, tw3N, twN, x0, x1, x2, dc, lds1);
            herm_load<T, NC, E>(Gi, m, t, lo, hi);
            fft3x(x0, x1, x2, std::integral_constant<int, +1>{});
            herm_build3_from<T, NC, E, TRI, BS>(lo, hi, t, lds, tw3N, twN, y0, y1, y2, T(1), lds1);
        } else {
            herm_build3<T, NC, E, TRI>(Fi, m, t, lds, tw3N, twN, x0, x1, x2, dc, lds1);
            fft3x(x0, x1, x2, std::integral_constant<int, +1>{});
            herm_build3<T, NC, E, TRI>(Gi, m, t, lds, tw3N, twN, y0, y1, y2, T(1), lds1);
        }
        fft3x(y0, y1, y2, std::integral_constant<int, +1>{});
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const C<T> p0{x0[e].re * y0[e].re, x0[e].im * y0[e].im};
            const C<T> p1{x1[e].re * y1[e].re, x1[e].im * y1[e].im};
            const C<T> p2{x2[e].re * y2[e].re, x2[e].im * y2[e].im};
            P0[e] = (MD && i > 0) ? P0[e] + p0 : p0;
            P1[e] = (MD && i > 0) ? P1[e] + p1 : p1;
            P2[e] = (MD && i > 0) ? P2[e] + p2 : p2;
        }
    }
    fft3x(P0, P1, P2, std::integral_constant<int, -1>{});
    // recombination: V_r(k) from P_r(k), P_r(NC-k); H_k, H_{N-k}, H_NC
    C<T> olo[E], ohi[E], ocen = zero<T>();
    const T h3 = T(0.86602540378443864676);
    C<T> Pm0[E], Pm1[E], Pm2[E];
    if constexpr (TRI) mirror3<T, NC, E>(P0, Pm0, P1, Pm1, P2, Pm2, t, lds, lds1, lds2);
    static_for<3>([&](auto ri) {
        constexpr int R = decltype(ri)::value == 0 ? 0 : (decltype(ri)::value == 1 ? 1 : -1);
        C<T>(&P)[E] = R == 0 ? P0 : (R > 0 ? P1 : P2);
        C<T>(&Pm)[E] = R == 0 ? Pm0 : (R > 0 ? Pm1 : Pm2);
        if constexpr (!TRI) mirror<T, NC, E>(P, Pm, t, lds);
        const C<T> z3 = R == 0 ? C<T>{T(1), T(0)} : (R > 0 ? C<T>{T(-0.5), -h3} : C<T>{T(-0.5), h3});
        const int zo = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * G;
            const C<T> V = r2c_post(P[e], Pm[e], twN[k + zo]);
            C<T> lo = V, hi = conj(V);
            if constexpr (R != 0) {
                const C<T> w = tw3N[k + zo];
                lo = R > 0 ? mulc(V, w) : V * w;                     // zeta_{3N}^{-Rk} V
                hi = z3 * (R > 0 ? w * conj(V) : mulc(conj(V), w));  // zeta_3^{-R} zeta_{3N}^{Rk} conj V
            }
            olo[e] = R == 0 ? lo : olo[e] + lo;
            ohi[e] = R == 0 ? hi : ohi[e] + hi;
            if (e == 0 && k == 0) {
                // V_R(NC) = Re P_0 - Im P_0 enters H_NC with zeta_6^{-R}
                const C<T> z6 = R == 0 ? C<T>{T(1), T(0)} : (R > 0 ? C<T>{T(0.5), -h3} : C<T>{T(0.5), h3});
                const C<T> cen = z6 * C<T>{P[e].re - P[e].im, T(0)};
                ocen = R == 0 ? cen : ocen + cen;
            }
        }
    });
    C<T>* H = (C<T>*)a.h + c.oh;
    const T s = T(1) / T(3 * N);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * G;
        if (k < m) H[k] = (e == 0 && k == 0 && (a.flags & kHermAdj)) ? C<T>{T(0.5) * s * olo[e].re, T(0)}
                                                                     : scale(olo[e], s);
        if (k > 0 && N - k < m) H[N - k] = scale(ohi[e], s);
    }
    if (t == 0 && NC < m) H[NC] = scale(ocen, s);
    if (c.act) {
        for (int64_t j = m + t; j < a.h_pad; j += G) H[j] = zero<T>();
    }
}

// The same convolution for rows whose transform would take a whole
// 1024-thread workgroup in the register-resident kernel (G = 1024: its build
// of three residues of two inputs exceeds the 128 registers such a
// workgroup leaves each thread).  Here the residues are formed and convolved
// one at a time: for residue R every thread builds its entries of w_{k,R}
// from U_k, U_{NC+k} and the mirrored U_{NC-k}, U_{N-k}, read from the input
// row itself, transforms them, and the forward transform of the products is
// folded into the output before the next residue starts.  Each input row is
// read twice per residue (its own and its mirrored entries); all but the
// first read are served by the caches.  Where two exchange-sized LDS buffers
// fit, the transformed f waits in the second one while g is built and
// transformed; otherwise (complex128, NC = 8192) it stays in registers.  The
// output accumulates in h itself (stored for R = 0, read, added to and
// stored again for R = +1, -1 by the same thread): accumulators in
// registers made the build spill.
template <typename T, int NC>
__host__ __device__ constexpr bool herm_staged()
{
    // complex128 only: in complex64 the register-resident kernel, spills and
    // all, measured faster (m = 16384: 0.166 against 0.181 ms for 256 rows,
    // one row per compute unit, where the time is one row's latency)
    return sizeof(T) == 8 && NC > 1 && row_G<T, 1>(NC) == 1024;
}
// The staged kernel's threads per row: 512, each holding NC / 512 values
// (twice the register-resident kernel's), which leaves every thread 256
// registers.
constexpr int kHermStagedThreads = 1024;

// The thread index through an empty asm statement: addresses computed from
// the result are recomputed where they are used instead of being computed
// once and kept live (or spilled) across the whole kernel.
__device__ __forceinline__ int fresh_tid(int t)
{
    asm volatile("" : "+v"(t));
    return t;
}

// Packed c2r input of residue R at frequency k (the per-residue part of
// herm_build3) from the half U (length m, zero beyond; U_0 scaled by dc).
template <typename T, int NC, int R>
__device__ __forceinline__ C<T> herm_build_one(const C<T>* U, int m, int k, T dc, const C<T>* tw3N,
                                               const C<T>* twN)
{
    const T h3 = T(0.86602540378443864676), sq3 = T(1.73205080756887729353);
    const bool k0 = k == 0;
    // unconditional loads (a load under a condition would become a branch):
    // at k = 0, U_{N-k} = U_N lies beyond m <= N and reads as 0, and
    // U_{NC-k} is U_NC, as the k = 0 terms need
    C<T> a = ldz_masked(U, k, m);                                      // U_k
    const C<T> d = ldz_masked(U, NC + k, m);                           // U_{NC+k}
    const C<T> b = ldz_masked(U, 2 * NC - k, m);                       // U_{N-k}
    const C<T> c = ldz_masked(U, NC - k, m);                           // U_{NC-k}
    a = k0 ? scale(a, dc) : a;
    const C<T> w2 = twN[k];
    C<T> p, q;
    if constexpr (R == 0) {
        p = a + conj(b);
        q = c + conj(d);
        if (k0) { p = C<T>{a.re, T(0)}; q = C<T>{T(2) * c.re, T(0)}; }
    } else if constexpr (R > 0) {
        const C<T> z3p{T(-0.5), -h3};
        p = tw3N[k] * (a + z3p * conj(b));
        q = tw3N[NC - k] * (c + z3p * conj(d));
        if (k0) { p = C<T>{a.re, T(0)}; q = C<T>{c.re - sq3 * c.im, T(0)}; }
    } else {
        const C<T> z3m{T(-0.5), h3};
        p = mulc(a + z3m * conj(b), tw3N[k]);
        q = mulc(c + z3m * conj(d), tw3N[NC - k]);
        if (k0) { p = C<T>{a.re, T(0)}; q = C<T>{c.re + sq3 * c.im, T(0)}; }
    }
    return c2r_pre(p, q, w2);
}

// Whether the staged kernel keeps f's transform in LDS (else in registers).
template <typename T, int NC>
__host__ __device__ constexpr bool herm_staged_xlds()
{
    return 2 * lpad_size(NC) * int(sizeof(C<T>)) <= 160 * 1024;
}

template <typename T, int NC, bool MD>
__global__ void __launch_bounds__(kHermStagedThreads, kHermStagedThreads / 256)
k_conv1d_hermitian_staged(RowArgs a)
{
    constexpr int N = 2 * NC, G = kHermStagedThreads, E = NC / G, LDSN = lpad_size(NC);
    static_assert(E >= 2 && NC % G == 0, "staged Hermitian rows: NC / 512 values per thread");
    constexpr bool XLDS = herm_staged_xlds<T, NC>();  // f's transform waits in LDS
    __shared__ C<T> sh[(XLDS ? 2 : 1) * LDSN];
    static_assert(sizeof(sh) <= 160 * 1024, "LDS footprint exceeds 160 KB");
    C<T>* A = sh;           // exchange buffer
    C<T>* X = sh + LDSN;    // transformed f (XLDS)
    const int t = threadIdx.x;
    const RowCtx c = row_ctx(a, (int64_t)blockIdx.x);
    const C<T>* twb = (const C<T>*)a.tw;
    const C<T>* twNC = twb + tw_off(NC);
    const C<T>* twN = twb + tw_off(N);
    const C<T>* tw3N = (const C<T>*)a.tw3 + tw_off(N);
    const int m = c.m;
    const int64_t nM = MD ? a.M : 1;
    const bool adj = a.flags & kHermAdj;
    const T dc = adj ? T(2) : T(1);
    const T s = T(1) / T(3 * N);
    C<T>* H = (C<T>*)a.h + c.oh;
    C<T> ocen = zero<T>();
    const T h3 = T(0.86602540378443864676);
    static_for<3>([&](auto ri) {
        constexpr int R = decltype(ri)::value == 0 ? 0 : (decltype(ri)::value == 1 ? 1 : -1);
        C<T> P[E];
        for (int64_t i = 0; i < nM; ++i) {
            C<T> x[E];
            {
                const int z = opaque_zero();
                const int tt = fresh_tid(t);
                const C<T>* U = (const C<T>*)a.f + c.of + i * a.f_i + z;
#pragma unroll
                for (int e = 0; e < E; ++e) x[e] = herm_build_one<T, NC, R>(U, m, tt + e * G, dc, tw3N + z, twN + z);
            }
            fft<T, NC, E, +1>(x, t, A, 1, twNC);
            if constexpr (XLDS) {
                // each thread keeps its own entries: no barrier
                const int tt = fresh_tid(t);
#pragma unroll
                for (int e = 0; e < E; ++e) X[lpad(tt + e * G)] = x[e];
            }
            C<T> y[E];
            {
                const int z = opaque_zero();
                const int tt = fresh_tid(t);
                const C<T>* U = (const C<T>*)a.g + c.og + i * a.g_i + z;
#pragma unroll
                for (int e = 0; e < E; ++e) y[e] = herm_build_one<T, NC, R>(U, m, tt + e * G, T(1), tw3N + z, twN + z);
            }
            fft<T, NC, E, +1>(y, t, A, 1, twNC);
            const int tt = fresh_tid(t);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const C<T> xv = XLDS ? X[lpad(tt + e * G)] : x[e];
                const C<T> p{xv.re * y[e].re, xv.im * y[e].im};
                P[e] = (MD && i > 0) ? P[e] + p : p;
            }
        }
        fft<T, NC, E, -1>(P, t, A, 1, twNC);
        // P_R(NC - k) through A, then this residue's share of H_k, H_{N-k}, H_NC
        const int tt = fresh_tid(t);
#pragma unroll
        for (int e = 0; e < E; ++e) A[lpad(tt + e * G)] = P[e];
        __syncthreads();
        const C<T> z3 = R == 0 ? C<T>{T(1), T(0)} : (R > 0 ? C<T>{T(-0.5), -h3} : C<T>{T(-0.5), h3});
        const int zo = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = tt + e * G;
            const C<T> Pm = A[lpad((NC - k) & (NC - 1))];
            const C<T> V = r2c_post(P[e], Pm, twN[k + zo]);
            C<T> lo = V, hi = conj(V);
            if constexpr (R != 0) {
                const C<T> w = tw3N[k + zo];
                lo = R > 0 ? mulc(V, w) : V * w;
                hi = z3 * (R > 0 ? w * conj(V) : mulc(conj(V), w));
            }
            {
                // H_0 of the adjoint form is real and halved
                const C<T> vlo = (e == 0 && k == 0 && adj) ? C<T>{T(0.5) * s * lo.re, T(0)} : scale(lo, s);
                if (k < m) H[k] = R == 0 ? vlo : H[k] + vlo;
                if (k > 0 && N - k < m) H[N - k] = R == 0 ? scale(hi, s) : H[N - k] + scale(hi, s);
            }
            if (e == 0 && k == 0) {
                const C<T> z6 = R == 0 ? C<T>{T(1), T(0)} : (R > 0 ? C<T>{T(0.5), -h3} : C<T>{T(0.5), h3});
                const C<T> cen = z6 * C<T>{P[e].re - P[e].im, T(0)};
                ocen = R == 0 ? cen : ocen + cen;
            }
        }
        __syncthreads();  // A is the exchange buffer of the next residue's transforms
    });
    if (t == 0 && NC < m) H[NC] = scale(ocen, s);
    if (c.act) {
        for (int64_t j = m + t; j < a.h_pad; j += G) H[j] = zero<T>();
    }
}

// Centered Hermitian ternary convolution (Sec. 4.2, tconv).  With the input
// half U_0..U_{N-1} (N >= m) padded to Fourier size 4N: for r in {0, 1} the
// sequence {zeta_{4N}^{rk} U_k : k = 0..N}, U_N = 0, is transformed
// complex-to-real at length 2N, the three real transforms are multiplied,
// transformed back, and 4N H_k = sum_r zeta_{4N}^{-rk} V_r(k).
// ======================================================================
template <typename T, int NN, int R>
__device__ __forceinline__ C<T> tern_Z(const C<T>* U, int m, int k, const C<T>* tw4N,
                                       const C<T>* tw2N)
{
    auto X = [&](int j) -> C<T> {  // zeta_{4N}^{Rj} U_j for 0 <= j <= N (U_N = 0)
        C<T> u = ldz(U, j, m < NN ? m : NN);
        if (j == 0) u.im = T(0);
        if constexpr (R != 0) u = u * tw4N[j & (NN - 1)];
        return u;
    };
    return c2r_pre(X(k), X(NN - k), tw2N[k]);
}

template <typename T, int NN, int R>
__device__ __forceinline__ void tern_load(const void* base, int64_t off, int m, int t,
                                          const RowArgs& a, C<T> (&x)[row_E<T, 1>(NN)])
{
    constexpr int E = row_E<T, 1>(NN), G = NN / E;
    const int q = opaque_zero();
    const C<T>* twb = (const C<T>*)a.tw;
    const C<T>* U = (const C<T>*)base + off + q;
#pragma unroll
    for (int e = 0; e < E; ++e)
        x[e] = tern_Z<T, NN, R>(U, m, t + e * G, twb + tw_off(4 * NN) + q, twb + tw_off(2 * NN) + q);
}

template <typename T, int NN, int R, bool ACCG>
__device__ __forceinline__ void tern_residue(const RowArgs& a, const RowCtx& c, int m, int t,
                                             C<T>* lds, C<T> (&acc)[ACCG ? 1 : row_E<T, 1>(NN)])
{
    constexpr int E = row_E<T, 1>(NN), G = NN / E;
    const C<T>* twb = (const C<T>*)a.tw;
    const C<T>* twNN = twb + tw_off(NN);
    C<T>* H = (C<T>*)a.h + c.oh;
    const T s = T(1) / T(4 * NN);
    C<T> x[E], y[E];
    tern_load<T, NN, R>(a.f, c.of, m, t, a, x);
    fft<T, NN, E, +1>(x, t, lds, 1, twNN);
    tern_load<T, NN, R>(a.g, c.og, m, t, a, y);
    fft<T, NN, E, +1>(y, t, lds, 1, twNN);
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = C<T>{x[e].re * y[e].re, x[e].im * y[e].im};
    tern_load<T, NN, R>(a.e, c.oe, m, t, a, y);
    fft<T, NN, E, +1>(y, t, lds, 1, twNN);
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = C<T>{x[e].re * y[e].re, x[e].im * y[e].im};
    fft<T, NN, E, -1>(x, t, lds, 1, twNN);
    mirror<T, NN, E>(x, y, t, lds);
    const int qo = opaque_zero();
    const C<T>* tw2N = twb + tw_off(2 * NN) + qo;
    const C<T>* tw4N = twb + tw_off(4 * NN) + qo;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * G;
        C<T> V = r2c_post(x[e], y[e], tw2N[k]);
        if constexpr (R != 0) V = mulc(V, tw4N[k]);
        if constexpr (ACCG) {
            if (k < m) H[k] = R == 0 ? scale(V, s) : H[k] + scale(V, s);
        } else {
            acc[e] = R == 0 ? V : acc[e] + V;
        }
    }
}

// ======================================================================
// Centered Hermitian ternary convolution (Sec. 4.2, tconv).  With the input
// half U_0..U_{N-1} (N >= m) padded to Fourier size 4N: for r in {0, 1} the
// sequence {zeta_{4N}^{rk} U_k : k = 0..N}, U_N = 0, is transformed
// complex-to-real at length 2N, the three real transforms are multiplied,
// transformed back, and 4N H_k = sum_r zeta_{4N}^{-rk} V_r(k).
// ======================================================================
template <typename T>
__device__ __forceinline__ C<T>* sh_dual(C<T>* sh, int GPB, int LDSN, int grp)
{
    return sh + (GPB + grp) * LDSN;
}

template <typename T, int NN, bool ACCG>
__global__ void __launch_bounds__((row_block<T, 1>(NN)), row_waves<T>(NN))
k_conv1d_ternary(RowArgs a)
{
    constexpr int E = row_E<T, 1>(NN), G = NN / E, GPB = row_GPB<T, 1>(NN), LDSN = row_lds<T, 1>(NN);
    constexpr bool DUALS = !ACCG && 2 * GPB * LDSN * int(sizeof(C<T>)) <= 160 * 1024;
    // transforms of 256 threads or more: two pairs of exchange buffers used
    // in turn (one barrier per stage) where they fit
    constexpr bool PP2 = DUALS && G >= 256 && 4 * GPB * LDSN * int(sizeof(C<T>)) <= 160 * 1024;
    __shared__ C<T> sh[(PP2 ? 4 : (DUALS ? 2 : 1)) * GPB * LDSN];
    static_assert(sizeof(sh) <= 160 * 1024, "LDS footprint exceeds 160 KB");
    const int grp = threadIdx.x / G, t = threadIdx.x % G;
    const RowCtx c = row_ctx(a, (int64_t)blockIdx.x * GPB + grp);
    C<T>* lds = sh + grp * LDSN;
    const int m = c.m;
    C<T>* H = (C<T>*)a.h + c.oh;
    if constexpr (ACCG) {
        // large rows: one residue at a time, accumulating in h
        C<T> acc[1];
        tern_residue<T, NN, 0, ACCG>(a, c, m, t, lds, acc);
        tern_residue<T, NN, 1, ACCG>(a, c, m, t, lds, acc);
    } else {
        // Each input row is read once; both residues are built from the
        // same registers and transformed together (paired transforms share
        // twiddles and barriers, through two exchange buffers when they fit).
        constexpr bool DUAL = 2 * GPB * LDSN * int(sizeof(C<T>)) <= 160 * 1024;
        C<T>* lds1 = DUAL ? sh_dual<T>(sh, GPB, LDSN, grp) : lds;
        const C<T>* twb = (const C<T>*)a.tw;
        const C<T>* twNN = twb + tw_off(NN);
        const C<T>* tw2b = twb + tw_off(2 * NN);  // zeta_2NN^k, k < NN
        const C<T>* tw4b = twb + tw_off(4 * NN);  // zeta_4NN^k, k < NN
        // the three tables (3 NN entries) copied into LDS once per
        // workgroup where the workgroup's LDS stays small
        constexpr bool TWL = IMPCONV_TER_TW_LDS && NN > E &&
                             int(sizeof(sh)) + 3 * NN * int(sizeof(C<T>)) <= IMPCONV_TER_TW_LDS_BYTES;
        __shared__ C<T> twl[TWL ? 3 * NN : 1];
        if constexpr (TWL) {
            for (int j = threadIdx.x; j < 3 * NN; j += blockDim.x)
                twl[j] = j < NN ? twNN[j] : (j < 2 * NN ? tw2b[j - NN] : tw4b[j - 2 * NN]);
            __syncthreads();
            twNN = twl;
            tw2b = twl + NN;
            tw4b = twl + 2 * NN;
        }
        const int mm = m < NN ? m : NN;
        auto pair = [&](auto& a0, auto& a1, auto dir) {
            constexpr int D = decltype(dir)::value;
            if constexpr (PP2) {
                fft2_pp<T, NN, E, D>(a0, a1, t, lds, lds1, sh + (2 * GPB + grp) * LDSN, sh + (3 * GPB + grp) * LDSN,
                                     twNN);
            } else if constexpr (DUAL) {
                fft2<T, NN, E, D>(a0, a1, t, lds, lds1, 1, twNN);
            } else {
                fft<T, NN, E, D>(a0, t, lds, 1, twNN);
                fft<T, NN, E, D>(a1, t, lds, 1, twNN);
            }
        };
        // packed c2r inputs of residues 0 and 1: X_r(j) = zeta_{4NN}^{rj} U_j
        // (U_0 real, U_NN = 0), Z_r(k) = c2r_pre(X_r(k), X_r(NN - k))
        auto build = [&](const void* base, int64_t off, C<T> (&z0)[E], C<T> (&z1)[E]) {
            const int q = opaque_zero();
            const C<T>* U = (const C<T>*)base + off + q;
            const C<T>* tw2N = tw2b + q;
            const C<T>* tw4N = tw4b + q;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * G;
                C<T> u = ldz(U, k, mm), v = ldz(U, NN - k, mm);
                if (e == 0 && k == 0) u.im = T(0);
                const C<T> w = tw2N[k];
                z0[e] = c2r_pre(u, v, w);
                z1[e] = c2r_pre(u * tw4N[k], v * tw4N[(NN - k) & (NN - 1)], w);
            }
        };
        C<T> x0[E], x1[E];
        build(a.f, c.of, x0, x1);
        pair(x0, x1, std::integral_constant<int, +1>{});
        static_for<2>([&](auto qi) {
            C<T> y0[E], y1[E];
            build(decltype(qi)::value == 0 ? a.g : a.e, decltype(qi)::value == 0 ? c.og : c.oe, y0, y1);
            pair(y0, y1, std::integral_constant<int, +1>{});
#pragma unroll
            for (int e = 0; e < E; ++e) {
                x0[e] = C<T>{x0[e].re * y0[e].re, x0[e].im * y0[e].im};
                x1[e] = C<T>{x1[e].re * y1[e].re, x1[e].im * y1[e].im};
            }
        });
        pair(x0, x1, std::integral_constant<int, -1>{});
        C<T> y0[E], y1[E];
        mirror<T, NN, E>(x0, y0, t, lds);
        mirror<T, NN, E>(x1, y1, t, lds);
        const int q = opaque_zero();
        const C<T>* tw2N = tw2b + q;
        const C<T>* tw4N = tw4b + q;
        const T s = T(1) / T(4 * NN);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * G;
            const C<T> w = tw2N[k];
            const C<T> V = r2c_post(x0[e], y0[e], w) + mulc(r2c_post(x1[e], y1[e], w), tw4N[k]);
            if (k < m) H[k] = scale(V, s);
        }
    }
    // stored slots past the logical length (zero slots of multi-D rows)
    if (c.act) {
        for (int64_t j = m + t; j < a.h_pad; j += G) H[j] = zero<T>();
    }
}

}  // namespace impconv

namespace impconv {

// ======================================================================
// Plain cyclic convolution of two (or, with a.e, three) real sequences of
// length 2 NC given by their half spectra X_0..X_NC (rows of length >= NC + 1):
// the explicitly padded centered Hermitian comparators (materialized
// padding).  h_k = scale * r2c(c2r(f) c2r(g) [c2r(e)])_k, k < m_out.
// ======================================================================
template <typename T, int NC>
__global__ void __launch_bounds__((row_block<T, 1>(NC)), row_waves<T>(NC))
k_conv1d_realcyclic(RowArgs a)
{
    constexpr int E = row_E<T, 1>(NC), G = NC / E, GPB = row_GPB<T, 1>(NC), LDSN = row_lds<T, 1>(NC);
    __shared__ C<T> sh[GPB * LDSN];
    static_assert(sizeof(sh) <= 160 * 1024, "LDS footprint exceeds 160 KB");
    const int grp = threadIdx.x / G, t = threadIdx.x % G;
    const RowCtx c = row_ctx(a, (int64_t)blockIdx.x * GPB + grp);
    C<T>* lds = sh + grp * LDSN;
    const C<T>* twb = (const C<T>*)a.tw;
    const C<T>* twNC = twb + tw_off(NC);
    const C<T>* tw2 = twb + tw_off(2 * NC);
    const int m = c.m;
    C<T> P[E];
    for (int64_t i = 0; i < a.M; ++i) {
        C<T> x[E], y[E];
        {
            const int z = opaque_zero();
            const C<T>* F = (const C<T>*)a.f + c.of + i * a.f_i + z;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * G;
                C<T> xk = ldz(F, k, m), xm = ldz(F, NC - k, m);
                if (k == 0) xk.im = T(0);
                x[e] = c2r_pre(xk, xm, tw2[k + z]);
            }
        }
        fft<T, NC, E, +1>(x, t, lds, 1, twNC);
        {
            const int z = opaque_zero();
            const C<T>* Gp = (const C<T>*)a.g + c.og + i * a.g_i + z;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * G;
                C<T> xk = ldz(Gp, k, m), xm = ldz(Gp, NC - k, m);
                if (k == 0) xk.im = T(0);
                y[e] = c2r_pre(xk, xm, tw2[k + z]);
            }
        }
        fft<T, NC, E, +1>(y, t, lds, 1, twNC);
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = C<T>{x[e].re * y[e].re, x[e].im * y[e].im};
        if (a.e) {
            // third real factor (explicitly padded ternary comparator)
            const int z = opaque_zero();
            const C<T>* Ep = (const C<T>*)a.e + c.oe + z;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * G;
                C<T> xk = ldz(Ep, k, m), xm = ldz(Ep, NC - k, m);
                if (k == 0) xk.im = T(0);
                y[e] = c2r_pre(xk, xm, tw2[k + z]);
            }
            fft<T, NC, E, +1>(y, t, lds, 1, twNC);
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = C<T>{x[e].re * y[e].re, x[e].im * y[e].im};
        }
#pragma unroll
        for (int e = 0; e < E; ++e) P[e] = i ? P[e] + x[e] : x[e];
    }
    fft<T, NC, E, -1>(P, t, lds, 1, twNC);
    C<T> Pm[E];
    mirror<T, NC, E>(P, Pm, t, lds);
    C<T>* H = (C<T>*)a.h + c.oh;
    const T s = T(a.scale);
    const int zo = opaque_zero();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + e * G;
        if (c.act && k < a.m_out) H[k] = scale(r2c_post(P[e], Pm[e], tw2[k + zo]), s);
    }
}

// dst[r][j] = j < copy ? src[r][j] : 0 for j < dst_ld (zero padding or crop).
template <typename T>
__global__ void k_pad_rows(const C<T>* __restrict__ src, C<T>* __restrict__ dst, int64_t nrows,
                           int64_t src_ld, int64_t copy, int64_t dst_ld)
{
    const int64_t total = nrows * dst_ld;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / dst_ld, j = i - r * dst_ld;
        dst[i] = j < copy ? src[r * src_ld + j] : zero<T>();
    }
}

// 2D copy with zero fill: for slab b = b1 * nsub + b2 (b < nb),
// dst[b1 dbs + b2 dbs2 + x dld + y] = (x < cx && y < cy) ? src[b1 sbs + b2 sbs2 + x sld + y] : 0
// for x < dx, y < dy.  Materializes the explicitly padded arrays of the
// comparator and crops its result.
template <typename T>
__global__ void k_copy2d(const C<T>* __restrict__ src, C<T>* __restrict__ dst, int64_t nb, int64_t nsub,
                         int64_t sbs, int64_t sbs2, int64_t sld, int64_t dbs, int64_t dbs2, int64_t dld,
                         int64_t cx, int64_t cy, int64_t dx, int64_t dy)
{
    const int64_t per = dx * dy, total = nb * per;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / per, r = i - b * per, x = r / dy, y = r - x * dy;
        const int64_t b1 = b / nsub, b2 = b - b1 * nsub;
        const bool in = x < cx && y < cy;
        dst[b1 * dbs + b2 * dbs2 + x * dld + y] = in ? src[b1 * sbs + b2 * sbs2 + x * sld + y] : zero<T>();
    }
}

}  // namespace impconv
