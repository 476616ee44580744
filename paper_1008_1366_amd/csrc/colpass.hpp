// colpass.hpp -- implicitly padded transforms along a strided (outer) axis.
//
// A column is one line along the transformed axis: `rows` elements at
// element stride `ld`; neighbouring columns are adjacent in memory.  One
// workgroup transforms a tile of TC adjacent columns, so every row segment
// it loads or stores is TC contiguous complex values (64-128 bytes).  This is
// the GPU form of the paper's multivector outer transforms (Sec. 3.1: one
// root of unity per row serves a whole row of columns).
//
// Modes (Sec. 2.1 fftpadBackward/Forward and Sec. 2.2 fft0padBackward/
// Forward, with the padded size N >= m a power of two):
//   kPadBwd : in[0] (m rows) -> out[r] = FFT+(zeta_{2N}^{rk} U_k), r = 0, 1
//   kPadFwd : in[0], in[1] (N rows) -> out_k = s (F0_k + zeta_{2N}^{-k} F1_k), k < m
//   kCenBwd : in[0] (centered, wavenumber k at row k + off_in) ->
//             out[r+1] = FFT+(w_{.,r}), r = -1, 0, 1, with w_{0,r} = U_0 and
//             w_{k,r} = zeta_{3N}^{rk} (U_k + zeta_3^{-r} U_{k-N})
//   kCenFwd : in[r+1] (N rows each) -> out (wavenumber k at row k + off_out):
//             3N U_k = sum_r zeta_{3N}^{-rk} F_r(k mod N), |k| < m; zero slots 0
//   kFft    : plain FFT of direction DIR of in[0] (n_in rows, zero padded to
//             N) into out[0] (n_out rows), scaled by s (explicit comparator)
//   kTerBwd : in[0] (centered, wavenumber k at row k + off_in, |k| < m) ->
//             out[r] = FFT+ of size N (= 2 N', N' >= m) of
//             a_{r,j} = zeta_{2N}^{r(j - N')} U_{j-N'}, j = 0..N-1, r = 0, 1:
//             the residues of the centered transform padded to 2N (Sec. 4.1,
//             fft0tpadBackward; the sign (-1)^l of each residue is dropped,
//             it cancels in a ternary product and the forward pass)
//   kTerFwd : in[0], in[1] (N rows each) -> out (wavenumber k at row
//             k + off_out): 2N U_k = F0(k + N') + zeta_{2N}^{-(k)} F1(k + N')
//             for |k| < m (Sec. 4.1, fft0tpadForward); zero slots 0
//   kFsBwd / kFsFwd : first and last pass of the four-step form of the 1D
//             complex convolution of length NF = N1 * N (N1 = ncols): a 1D
//             input f_k, k = k1 + N1 k2, is read as an N x N1 matrix; the
//             backward pass applies the residue shift zeta_{2NF}^{rk}, an
//             N-point FFT down each column and the twiddle zeta_{NF}^{j2 k1};
//             the forward pass undoes the twiddle, transforms back and
//             recombines (F0 + zeta_{2NF}^{-k} F1) / 2NF.
#pragma once
#include "fft_wg.hpp"

namespace impconv {

enum ColMode { kPadBwd = 0, kPadFwd = 1, kCenBwd = 2, kCenFwd = 3, kFft = 4, kFsBwd = 5, kFsFwd = 6,
               kTerBwd = 7, kTerFwd = 8 };

__host__ __device__ constexpr const char* col_mode_name(int mode)
{
    return mode == kPadBwd ? "colpass_pad_bwd" : mode == kPadFwd ? "colpass_pad_fwd"
         : mode == kCenBwd ? "colpass_cen_bwd" : mode == kCenFwd ? "colpass_cen_fwd"
         : mode == kFft ? "colpass_fft" : mode == kFsBwd ? "colpass_fourstep_bwd"
         : mode == kFsFwd ? "colpass_fourstep_fwd" : mode == kTerBwd ? "colpass_ter_bwd" : "colpass_ter_fwd";
}
#define MODE_NAME(x) col_mode_name(x)

struct ColArgs {
    const void* in[3];
    void* out[3];
    int64_t nslab;                 // independent 2D slabs, slab = s1 * nsub + s2
    int64_t nsub;                  // >= 1
    int64_t in_bs, out_bs;         // element stride of s1
    int64_t in_bs2, out_bs2;       // element stride of s2
    int64_t ncols;                 // columns per slab
    int64_t in_ld, out_ld;         // element stride between rows
    int n_in, n_out;               // stored rows of input / output
    int m;                         // logical modes along the axis
    int off_in, off_out;           // row of wavenumber 0 (centered modes)
    int sym;                       // k_last = 0 symmetrization: 0 off, 1 2D rule, 2 3D rule
    int64_t sym_nz;                // 3D rule: storage length of the last axis
    int sym_offy;                  // 3D rule: row of k_y = 0 in the y storage
    int sym_ny;                    // 3D rule: storage length of the y axis
    // valid columns c = iy * mask_nz + iz: ylo <= iy < yhi and iz < zhi; the
    // others (zero slots of the transverse axes) read as zero
    int64_t mask_nz;
    int mask_ylo, mask_yhi, mask_zhi;
    int64_t nf;                    // four-step: full 1D length N1 * N
    const int64_t* slab_off;       // four-step, optional: element offset of each s1 slab's 1D data
    const int64_t* slab_m;         // four-step, optional: logical length of each s1 slab
    int64_t nslab2;                // k_colpass: 0, or the slabs of a first set, the rest (nslab - nslab2)
                                   // reading in[0] + in2_off and writing out[r] + out2_off (elements),
                                   // with the same strides and flags
    int64_t in2_off, out2_off;
    uint32_t fsflags;              // 1 = reverse within m (input of kFsBwd / kPadBwd, output of kFsFwd /
                                   // kPadFwd), 2 = conjugate the input (kFsBwd / kPadBwd), 4 = Hermitian
                                   // adjoint on the k_last = 0 hyperplane (kCenBwd: load U_k + conj U_{-k};
                                   // kCenFwd: zero the overwritten half, DC halved and real; needs sym),
                                   // 8 = compensated twiddle products (complex64 kPadBwd / kPadFwd,
                                   // selects the COMP instantiation)
    double scale;
    const void* tw;
    const void* tw3;
    int ncu;                       // compute units of the device (persistent grids)
    const void* twlo;              // complex64 low parts of tw (fsflags 8: compensated products)
    const void* twfs;              // four-step: zeta_nf^{j2 c} at [j2][c] (j2 < N, c < ncols)
};

// Elements per thread of a column pass.  The centered passes keep three
// arrays of E values live (U_k and U_{k-N} plus one residue; or two output
// accumulators plus one residue).  The forward (accumulating) pass takes half
// the FFT elements per thread at every length, which lifts it from one or two
// waves per SIMD to three or four; the backward pass does so from N = 2048 on,
// where the full count no longer fits the 128 registers its block allows.
// Measured on 256-point columns, halving the backward pass costs 4%.
#ifndef IMPCONV_CEN_BWD_HALF_E_MINN
#define IMPCONV_CEN_BWD_HALF_E_MINN 2048
#endif
template <typename T, int MODE = -1>
__host__ __device__ constexpr int col_E(int N)
{
    const int e = fft_E<T>(N);
    const bool half = MODE == 3 || (MODE == 2 && N >= IMPCONV_CEN_BWD_HALF_E_MINN);  // kCenFwd, kCenBwd
    return (half && e >= 4) ? e / 2 : e;
}

// Columns per tile: a 64-byte row segment (8 complex64 / 4 complex128), up to
// 128 bytes for short transforms, limited by 1024 threads and ~140 KB of LDS.
#ifndef IMPCONV_COL_SEG_BYTES
#define IMPCONV_COL_SEG_BYTES 64
#endif
template <typename T, int MODE = -1>
__host__ __device__ constexpr int col_TC(int N)
{
    // short columns: 128-byte segments, except the centered forward pass
    // (three input arrays, one output), measured faster with 64 (0.27 vs
    // 0.30 ms per launch at 256 points)
    const int seg = N <= 512 ? (MODE == 3 ? 64 : 128) : IMPCONV_COL_SEG_BYTES;  // 3 = kCenFwd
    int tc = seg / int(sizeof(C<T>));
    const int G = N / col_E<T, MODE>(N);
    while (tc > 1 && (tc * G > 1024 || (N > col_E<T, MODE>(N) && tc * lpad_size(N) * int(sizeof(C<T>)) > 143360)))
        tc /= 2;
    return tc;
}
template <typename T, int MODE = -1> __host__ __device__ constexpr int col_block(int N)
{
    return col_TC<T, MODE>(N) * (N / col_E<T, MODE>(N));
}

// blockIdx -> logical tile so that consecutive tiles (which share cache lines
// and run concurrently) are issued to the same XCD: the hardware deals
// workgroups to the 8 XCDs round-robin.  Returns -1 for the padding blocks.
__device__ __forceinline__ int64_t xcd_tile(int64_t nblocks)
{
    const int64_t bid = blockIdx.x;
    const int64_t per = (nblocks + 7) / 8;
    const int64_t lg = (bid % 8) * per + bid / 8;
    return lg < nblocks ? lg : -1;
}

#ifndef IMPCONV_COL_TW_LDS
#define IMPCONV_COL_TW_LDS 1
#endif
#ifndef IMPCONV_COL_TW_LDS_MAXN
#define IMPCONV_COL_TW_LDS_MAXN 2048
#endif
#ifndef IMPCONV_COL_TW_LDS_FS
#define IMPCONV_COL_TW_LDS_FS 1
#endif
// Whether k_colpass<T, N, MODE> keeps its twiddle tables in LDS: plain
// (not compensated) tables of the padded, centered and ternary modes, for
// columns of up to IMPCONV_COL_TW_LDS_MAXN points transformed across threads,
// where the 2N table entries leave the number of workgroups the LDS admits
// per compute unit unchanged, or the workgroup within 64 KB (two or more
// workgroups per compute unit), or, for the padded, centered and ternary
// passes of 1024 and 2048 points (workgroups of 512 or 1024 threads, of which
// their registers admit one or two), within the 160 KB of one compute unit.
// The plain FFT pass of the explicit comparators at 1024 points lost a
// workgroup per compute unit to the copy and ran slower (3D Hermitian
// comparator 89 -> 100 ms), so the four-step and FFT modes take only the
// first two rules.  Where the copy
// costs a workgroup per compute unit (the complex128 padded backward pass at
// 256 points: 0.257 -> 0.295 ms per launch on its own), the 3D step that
// overlaps it with the rows is still faster (256^3 complex128: 4.63 -> 4.57
// ms); at 2048 points the 2D Euler step goes 0.711 -> 0.685 ms.
// Tables of N entries a mode reads with N-independent indices: the stage
// table, and for the padded, centered and ternary modes the residue shifts.
__host__ __device__ constexpr int col_tw_tables(int mode)
{
    return (mode == kFsBwd || mode == kFsFwd || mode == kFft) ? 1 : 2;
}
template <typename T, int N, int MODE, bool COMP>
constexpr bool COL_TWL = [] {
    constexpr int E = col_E<T, MODE>(N), TC = col_TC<T, MODE>(N);
    constexpr int sh = (N > E ? lpad_size(N) * TC : 1) * int(sizeof(C<T>));
    constexpr int tw = col_tw_tables(MODE) * N * int(sizeof(C<T>));
    return IMPCONV_COL_TW_LDS && !COMP && N > E && N <= IMPCONV_COL_TW_LDS_MAXN &&
           (MODE == kPadBwd || MODE == kPadFwd || MODE == kCenBwd || MODE == kCenFwd || MODE == kTerBwd ||
            MODE == kTerFwd || (IMPCONV_COL_TW_LDS_FS && (MODE == kFsBwd || MODE == kFsFwd || MODE == kFft))) &&
           ((160 * 1024) / sh == (160 * 1024) / (sh + tw) ||
            sh + tw <= (N >= 1024 && col_tw_tables(MODE) == 2 ? 160 : 64) * 1024);
}();

template <typename T, int N, int MODE, int DIR, bool COMP = false>
__global__ void __launch_bounds__((col_block<T, MODE>(N)))
k_colpass(ColArgs a)
{
    constexpr int E = col_E<T, MODE>(N), G = N / E, TC = col_TC<T, MODE>(N);
    constexpr int LDSN = N > E ? lpad_size(N) * TC : 1;
    __shared__ C<T> sh[LDSN];
    static_assert(sizeof(sh) <= 160 * 1024, "LDS footprint exceeds 160 KB");
    const int col = threadIdx.x % TC, t = threadIdx.x / TC;
    const int64_t ntile = (a.ncols + TC - 1) / TC;
    const int64_t lg = xcd_tile(a.nslab * ntile);
    if (lg < 0) return;  // whole padding block: no barrier is reached
    // two sets in one launch (nslab2 > 0): slabs from nslab2 on read and
    // write the second set, at element offsets in2_off / out2_off
    const int64_t slab0 = lg / ntile, tile = lg - slab0 * ntile;
    const bool set2 = a.nslab2 > 0 && slab0 >= a.nslab2;
    const int64_t slab = set2 ? slab0 - a.nslab2 : slab0;
    const int64_t io2 = set2 ? a.in2_off : 0, oo2 = set2 ? a.out2_off : 0;
    const int64_t s1 = slab / a.nsub, s2 = slab - s1 * a.nsub;
    const int64_t c = tile * TC + col;
    const bool cin = c < a.ncols;  // column exists: stores go through
    const int64_t cc = cin ? c : 0;
    bool cact = cin;               // column carries data: loads go through
    if (a.mask_nz > 0) {
        const int64_t iy = cc / a.mask_nz, iz = cc - iy * a.mask_nz;
        cact = cin && iy >= a.mask_ylo && iy < a.mask_yhi && iz < a.mask_zhi;
    }
    C<T>* lds = sh + col;
    const C<T>* twb = (const C<T>*)a.tw;
    // twiddle sources: plain tables, or (COMP) the high/low pairs
    using TWT = std::conditional_t<COMP, CompTw<T>, const C<T>*>;
    auto twsrc = [&](int64_t off) -> TWT {
        if constexpr (COMP) return CompTw<T>{twb + off, (const C<T>*)a.twlo + off};
        else return twb + off;
    };
    TWT twN = twsrc(tw_off(N));
    TWT tw2N = twsrc(tw_off(2 * N));
    const C<T>* tw3N = (const C<T>*)a.tw3 + tw_off(N);
    const C<T>* tw2Np = twb + tw_off(2 * N);  // plain zeta_2N table (ternary modes)
    // short columns: the two tables a pass reads (zeta_N^j for the transform
    // stages; zeta_2N^k or, centered modes, zeta_3N^k, for the residue
    // shifts; j, k < N) are copied into LDS once per workgroup, where no
    // fewer workgroups then fit a compute unit
    if constexpr (COL_TWL<T, N, MODE, COMP>) {
        // the four-step and plain FFT modes copy the stage table only
        constexpr int NT = col_tw_tables(MODE) * N;
        __shared__ C<T> twl[NT];
        const C<T>* t2 = (MODE == kCenBwd || MODE == kCenFwd) ? tw3N : twb + tw_off(2 * N);
        for (int j = threadIdx.x; j < NT; j += blockDim.x) twl[j] = j < N ? twb[tw_off(N) + j] : t2[j - N];
        __syncthreads();
        twN = twl;
        if constexpr (MODE == kCenBwd || MODE == kCenFwd) tw3N = twl + N;
        else if constexpr (NT == 2 * N) { tw2N = twl + N; tw2Np = twl + N; }
    }
    const int64_t ib = s1 * a.in_bs + s2 * a.in_bs2 + cc + io2, ob = s1 * a.out_bs + s2 * a.out_bs2 + cc + oo2;
    auto ldrow = [&](int q, int row, int nrows) -> C<T> {  // in[q] at (row, c), zero outside
        const C<T>* p = (const C<T>*)a.in[q] + ib;
        const bool ok = cact && row >= 0 && row < nrows;
        const C<T> v = p[(ok ? row : 0) * a.in_ld];
        return ok ? v : zero<T>();
    };
    auto strow = [&](int q, int row, C<T> v) {
        if (cin) ((C<T>*)a.out[q])[ob + int64_t(row) * a.out_ld] = v;
    };

    if constexpr (MODE == kPadBwd) {
        // adjoint forms: rows read reversed within m and/or conjugated
        const bool rev = a.fsflags & 1, cj = a.fsflags & 2;
        C<T> x[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int row = t + e * G;
            x[e] = ldrow(0, rev ? a.m - 1 - row : row, a.m);
            if (cj) x[e] = conj(x[e]);
        }
        C<T> y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) y[e] = x[e];
        fft<T, N, E, +1>(y, t, lds, TC, twN);
#pragma unroll
        for (int e = 0; e < E; ++e) strow(0, t + e * G, y[e]);
        const int z = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = mulw<+1>(x[e], tw2N[t + e * G + z]);
        fft<T, N, E, +1>(x, t, lds, TC, twN);
#pragma unroll
        for (int e = 0; e < E; ++e) strow(1, t + e * G, x[e]);
    } else if constexpr (MODE == kPadFwd) {
        C<T> x[E], y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = ldrow(0, t + e * G, N);
        fft<T, N, E, -1>(x, t, lds, TC, twN);
        {
            const int z = opaque_zero();
#pragma unroll
            for (int e = 0; e < E; ++e) y[e] = ldrow(1, t + e * G + z, N);
        }
        fft<T, N, E, -1>(y, t, lds, TC, twN);
        const T s = T(a.scale);
        const bool rev = a.fsflags & 1;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * G;
            if (k < a.m) strow(0, rev ? a.m - 1 - k : k, scale(x[e] + mulw<-1>(y[e], tw2N[k]), s));
        }
    } else if constexpr (MODE == kCenBwd) {
        // U_k and U_{k-N} of this thread's frequencies, with the optional
        // conjugate mirror of the k_last = 0 hyperplane.
        C<T> up[E], un[E];
        int64_t mcol = cc;
        bool plane = false;
        int ky = 0;
        if (a.sym == 1) {
            plane = c == 0;
        } else if (a.sym == 2) {
            const int64_t iy = cc / a.sym_nz, iz = cc - iy * a.sym_nz;
            plane = iz == 0;
            ky = int(iy) - a.sym_offy;
            const int iym = -ky + a.sym_offy;
            mcol = (iym >= 0 && iym < a.sym_ny) ? int64_t(iym) * a.sym_nz : cc;
        }
        const C<T>* base = (const C<T>*)a.in[0] + s1 * a.in_bs + s2 * a.in_bs2 + io2;
        // wavenumber k of this column (|k| < m)
        auto ldk = [&](int k) -> C<T> {
            const bool in = cact && k > -a.m && k < a.m;
            // mirror: k < 0, or k = 0 with ky < 0 (3D); DC real
            const bool mir = plane && (k < 0 || (k == 0 && ky < 0));
            const int kk = in ? (mir ? -k : k) : 0;
            const int64_t colx = mir ? mcol : cc;
            C<T> v = base[colx + int64_t(kk + a.off_in) * a.in_ld];
            if (mir) v = conj(v);
            if (plane && k == 0 && ky == 0) v.im = T(0);
            return in ? v : zero<T>();
        };
        // adjoint: U_k + conj U_{-k} on the hyperplane (both halves); off it
        // the second load repeats the first address (a cache hit)
        auto ldk_adj = [&](int k) -> C<T> {
            const bool in = cact && k > -a.m && k < a.m;
            const int kk = in ? k : 0;
            const C<T> v = base[cc + int64_t(kk + a.off_in) * a.in_ld];
            const C<T> u = base[(plane ? mcol : cc) + int64_t((plane ? -kk : kk) + a.off_in) * a.in_ld];
            const C<T> s = plane ? v + conj(u) : v;
            return in ? s : zero<T>();
        };
        // The thread index goes through an empty asm so the per-element
        // mirror selection below stays a run-time computation.  With one
        // thread per column (G = 1) it is otherwise fully constant-folded,
        // and that folded form was observed to load wrong mirrored values
        // (caught by the G = 1 symmetrized parity cases).  The adjoint test
        // is taken once, outside the element loops, so that each loop stays
        // free of branches and its loads issue back to back.
        int tl = t;
        asm volatile("" : "+v"(tl));
        if (a.fsflags & 4) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = tl + e * G;
                up[e] = ldk_adj(k);
                un[e] = ldk_adj(k - N);
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = tl + e * G;
                up[e] = ldk(k);
                un[e] = ldk(k - N);
            }
        }
        const T h3 = T(0.86602540378443864676);
        static_for<3>([&](auto ri) {
            constexpr int R = int(decltype(ri)::value) - 1;
            const C<T> z3 = R == 0 ? C<T>{T(1), T(0)} : (R > 0 ? C<T>{T(-0.5), -h3} : C<T>{T(-0.5), h3});
            const int z = opaque_zero();
            C<T> w[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * G;
                C<T> v = up[e] + z3 * un[e];
                if constexpr (R != 0) {
                    const C<T> tw = tw3N[k + z];
                    v = R > 0 ? v * tw : mulc(v, tw);
                }
                w[e] = k == 0 ? up[e] : v;
            }
            fft<T, N, E, +1>(w, t, lds, TC, twN);
#pragma unroll
            for (int e = 0; e < E; ++e) strow(R + 1, t + e * G, w[e]);
        });
    } else if constexpr (MODE == kCenFwd) {
        C<T> ap[E], an[E];
        const T h3 = T(0.86602540378443864676);
        static_for<3>([&](auto ri) {
            constexpr int R = int(decltype(ri)::value) - 1;
            C<T> x[E];
            const int z = opaque_zero();
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = ldrow(R + 1, t + e * G + z, N);
            fft<T, N, E, -1>(x, t, lds, TC, twN);
            // zeta_3^{R} for the negative wavenumbers
            const C<T> z3p = R == 0 ? C<T>{T(1), T(0)} : (R > 0 ? C<T>{T(-0.5), h3} : C<T>{T(-0.5), -h3});
            const int z2 = opaque_zero();
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + e * G;
                C<T> v = x[e];
                if constexpr (R != 0) {
                    const C<T> tw = tw3N[k + z2];
                    v = R > 0 ? mulc(v, tw) : v * tw;  // zeta_{3N}^{-Rk}
                }
                ap[e] = R == -1 ? v : ap[e] + v;
                an[e] = R == -1 ? z3p * v : an[e] + z3p * v;
            }
        });
        const T s = T(a.scale);
        // adjoint: on the k_last = 0 hyperplane the entries the forward
        // symmetrization overwrites (k < 0, or k = 0 with ky < 0) get zero,
        // and the DC entry is halved and real
        bool plane = false;
        int ky = 0;
        if (a.fsflags & 4) {
            if (a.sym == 1) {
                plane = c == 0;
            } else if (a.sym == 2) {
                const int64_t iy = cc / a.sym_nz, iz = cc - iy * a.sym_nz;
                plane = iz == 0;
                ky = int(iy) - a.sym_offy;
            }
        }
        auto adj_edit = [&](int k, C<T> v) -> C<T> {
            if (plane && (k < 0 || (k == 0 && ky < 0))) return zero<T>();
            if (plane && k == 0 && ky == 0) return C<T>{T(0.5) * v.re, T(0)};
            return v;
        };
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * G;
            if (k < a.m) strow(0, k + a.off_out, adj_edit(k, scale(ap[e], s)));
            if (k >= 1 && k - N > -a.m) strow(0, k - N + a.off_out, adj_edit(k - N, scale(an[e], s)));
        }
        // zero slots: rows whose wavenumber lies outside |k| < m
        for (int row = t; row < a.n_out; row += G) {
            const int k = row - a.off_out;
            if (k <= -a.m || k >= a.m) strow(0, row, zero<T>());
        }
    } else if constexpr (MODE == kTerBwd) {
        // U_{j - N/2} of this thread's rows j = t + eG, with the conjugate
        // mirror of the k_last = 0 line (2D rule: column 0)
        constexpr int NH = N / 2;
        const bool plane = a.sym == 1 && c == 0;
        const C<T>* base = (const C<T>*)a.in[0] + s1 * a.in_bs + s2 * a.in_bs2 + io2;
        const C<T>* tw2N = tw2Np;
        int tl = t;
        asm volatile("" : "+v"(tl));
        C<T> x[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = tl + e * G - NH;
            const bool in = cact && k > -a.m && k < a.m;
            const bool mir = plane && k < 0;
            const int kk = in ? (mir ? -k : k) : 0;
            C<T> v = base[cc + int64_t(kk + a.off_in) * a.in_ld];
            if (mir) v = conj(v);
            if (plane && k == 0) v.im = T(0);
            x[e] = in ? v : zero<T>();
        }
        C<T> y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) y[e] = x[e];
        fft<T, N, E, +1>(y, t, lds, TC, twN);
#pragma unroll
        for (int e = 0; e < E; ++e) strow(0, t + e * G, y[e]);
        // residue 1: zeta_{2N}^{j - N/2} = -i zeta_{2N}^j
        const int z = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = muli<-1>(x[e] * tw2N[t + e * G + z]);
        fft<T, N, E, +1>(x, t, lds, TC, twN);
#pragma unroll
        for (int e = 0; e < E; ++e) strow(1, t + e * G, x[e]);
    } else if constexpr (MODE == kTerFwd) {
        constexpr int NH = N / 2;
        const C<T>* tw2N = tw2Np;
        C<T> x[E], y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = ldrow(0, t + e * G, N);
        fft<T, N, E, -1>(x, t, lds, TC, twN);
        {
            const int z = opaque_zero();
#pragma unroll
            for (int e = 0; e < E; ++e) y[e] = ldrow(1, t + e * G + z, N);
        }
        fft<T, N, E, -1>(y, t, lds, TC, twN);
        const T s = T(a.scale);
        const int z = opaque_zero();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = t + e * G, k = j - NH;
            // zeta_{2N}^{-(j - N/2)} = i conj(zeta_{2N}^j)
            const C<T> v = x[e] + muli<+1>(mulc(y[e], tw2N[j + z]));
            if (k > -a.m && k < a.m) strow(0, k + a.off_out, scale(v, s));
        }
        // zero slots: rows whose wavenumber lies outside |k| < m
        for (int row = t; row < a.n_out; row += G) {
            const int k = row - a.off_out;
            if (k <= -a.m || k >= a.m) strow(0, row, zero<T>());
        }
    } else if constexpr (MODE == kFsBwd) {
        const C<T>* tw2F = twb + tw_off(2 * a.nf);
        const int64_t m1 = a.slab_m ? a.slab_m[s1] : a.m;
        const C<T>* src = (const C<T>*)a.in[0] + (a.slab_off ? a.slab_off[s1] + s2 * a.in_bs2 : ib - cc);
        const bool rev = a.fsflags & 1, cj = a.fsflags & 2;
        C<T> x[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {  // element k = c + N1 (t + e G) of the 1D input
            const int64_t k = cc + a.ncols * int64_t(t + e * G);
            const bool ok = cact && k < m1;
            C<T> v = src[ok ? (rev ? m1 - 1 - k : k) : 0];
            if (cj) v = conj(v);
            x[e] = ok ? v : zero<T>();
        }
        // the column twiddles zeta_F^{j2 c} serve both residues: one load
        // each, contiguous across the columns of a wave
        const C<T>* twT = (const C<T>*)a.twfs + cc;
        C<T> wf[E];
#pragma unroll
        for (int e = 0; e < E; ++e) wf[e] = twT[int64_t(t + e * G) * a.ncols];
        static_for<2>([&](auto ri) {
            constexpr int R = decltype(ri)::value;
            C<T> y[E];
            const int z = opaque_zero();
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t k = cc + a.ncols * int64_t(t + e * G);
                y[e] = R ? x[e] * tw2F[k + z] : x[e];
            }
            fft<T, N, E, +1>(y, t, lds, TC, twN);
#pragma unroll
            for (int e = 0; e < E; ++e) strow(R, t + e * G, y[e] * wf[e]);
        });
    } else if constexpr (MODE == kFsFwd) {
        const C<T>* tw2F = twb + tw_off(2 * a.nf);
        C<T> acc[E];
        // the column twiddles zeta_F^{j2 c} serve both residues: one load
        // each, contiguous across the columns of a wave
        const C<T>* twT = (const C<T>*)a.twfs + cc;
        C<T> wf[E];
#pragma unroll
        for (int e = 0; e < E; ++e) wf[e] = twT[int64_t(t + e * G) * a.ncols];
        static_for<2>([&](auto ri) {
            constexpr int R = decltype(ri)::value;
            C<T> x[E];
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = mulc(ldrow(R, t + e * G, N), wf[e]);
            fft<T, N, E, -1>(x, t, lds, TC, twN);
            const int z2 = opaque_zero();
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t k = cc + a.ncols * int64_t(t + e * G);
                acc[e] = R ? acc[e] + mulc(x[e], tw2F[k + z2]) : x[e];
            }
        });
        const T s = T(a.scale);
        const int64_t m1 = a.slab_m ? a.slab_m[s1] : a.m;
        C<T>* H = (C<T>*)a.out[0] + (a.slab_off ? a.slab_off[s1] : ob - cc);
        const bool rev = a.fsflags & 1;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t k = cc + a.ncols * int64_t(t + e * G);
            if (cin && k < m1) H[rev ? m1 - 1 - k : k] = scale(acc[e], s);
        }
    } else {  // kFft
        C<T> x[E];
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = ldrow(0, t + e * G, a.n_in);
        fft<T, N, E, DIR>(x, t, lds, TC, twN);
        const T s = T(a.scale);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + e * G;
            if (k < a.n_out) strow(0, k, scale(x[e], s));
        }
    }
}

// ------------------------------------------------------------------ buffer loads
// Raw buffer loads through a buffer resource (base address, num_records in
// bytes, in scalar registers): a byte offset past num_records reads zero
// without touching memory, which gives zero padding and masked columns with
// neither a branch nor a select, so all of a thread's loads stay in one
// basic block and the waitcnt pass can count them exactly.
typedef int i32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
__device__ f32x2_t raw_buffer_load_f32x2(i32x4_t rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.v2f32");
__device__ f64x2_t raw_buffer_load_f64x2(i32x4_t rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.load.v2f64");
__device__ void raw_buffer_store_f32x2(f32x2_t v, i32x4_t rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.store.v2f32");
__device__ void raw_buffer_store_f64x2(f64x2_t v, i32x4_t rsrc, int voff, int soff, int aux)
    __asm("llvm.amdgcn.raw.buffer.store.v2f64");

constexpr uint32_t kBufRecords = 0x7fffffffu;  // bytes addressable through a resource
constexpr uint32_t kBufOff = 0x80000000u;      // an offset that reads zero / drops a write

// Resource for the wave-uniform base p.  Word 3 selects a valid 32-bit data
// format with identity swizzle, as raw loads on gfx9-family parts require.
__device__ __forceinline__ i32x4_t buf_rsrc(const void* p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    i32x4_t r;
    r.x = __builtin_amdgcn_readfirstlane(int(uint32_t(a)));
    r.y = __builtin_amdgcn_readfirstlane(int(uint32_t(a >> 32) & 0xffffu));  // stride 0
    r.z = int(kBufRecords);
    r.w = 0x00020000;
    return r;
}
template <typename T>
__device__ __forceinline__ C<T> buf_load(i32x4_t r, uint32_t off)
{
    if constexpr (sizeof(T) == 4) {
        const f32x2_t v = raw_buffer_load_f32x2(r, int(off), 0, 0);
        return C<T>{v.x, v.y};
    } else {
        const f64x2_t v = raw_buffer_load_f64x2(r, int(off), 0, 0);
        return C<T>{v.x, v.y};
    }
}
template <typename T>
__device__ __forceinline__ void buf_store(i32x4_t r, uint32_t off, C<T> v)
{
    if constexpr (sizeof(T) == 4) {
        f32x2_t w;
        w.x = v.re;
        w.y = v.im;
        raw_buffer_store_f32x2(w, r, int(off), 0, 0);
    } else {
        f64x2_t w;
        w.x = v.re;
        w.y = v.im;
        raw_buffer_store_f64x2(w, r, int(off), 0, 0);
    }
}

// ------------------------------------------------------------------ persistent form
// For long columns one tile fills the LDS of a compute unit, so a one-tile
// workgroup leaves the CU idle while it waits for its loads.  k_colpipe is
// the persistent form of kPadBwd / kPadFwd for that case: one workgroup per
// CU walks a sequence of tiles.  The backward pass issues the next tile's
// loads before the current tile's second transform; the forward pass loads
// both of its inputs up front, so the second one arrives during the first
// transform (a cross-tile prefetch there would need a third tile-sized
// register array).  Prefetched loads must not be followed by global twiddle
// loads (vector-memory loads return in order, so waiting for a twiddle would
// wait for the prefetch too), hence the stage twiddles come from a copy of
// zeta_N in LDS, and the residue shift zeta_{2N}^{t + eG} is formed as
// zeta_{2N}^t zeta_N^{eG/2}.

// zeta_N^j (j < N) from an LDS table that holds the first Q / 4 of it:
// Q = 4 the whole table, Q = 2 the first half (zeta_N^{j + N/2} = -zeta_N^j).
template <typename T, int N, int Q>
struct LdsTw {
    const C<T>* p;
    __device__ __forceinline__ LdsTw operator+(int z) const { return LdsTw{p + z}; }
    __device__ __forceinline__ C<T> operator[](int j) const
    {
        static_assert(Q == 4 || Q == 2, "LDS twiddle table: whole or half");
        if constexpr (Q == 4) {
            return p[j];
        } else {
            const C<T> v = p[j & (N / 2 - 1)];
            return (j & (N / 2)) ? C<T>{-v.re, -v.im} : v;
        }
    }
};

// Quarters of zeta_N that fit in LDS beside the exchange tile (0: none).
template <typename T>
__host__ __device__ constexpr int pipe_twq(int N)
{
    const int cs = int(sizeof(C<T>));
    const int ex = N > fft_E<T>(N) ? lpad_size(N) * col_TC<T>(N) * cs : 0;
    return ex + N * cs <= 160 * 1024 ? 4 : ex + (N / 2) * cs <= 160 * 1024 ? 2 : 0;
}
// The pipelined form pays off where the exchange tile leaves room for only
// one workgroup per CU.
template <typename T>
__host__ __device__ constexpr bool pipe_ok(int N)
{
    return N > fft_E<T>(N) && lpad_size(N) * col_TC<T>(N) * int(sizeof(C<T>)) > 80 * 1024 && pipe_twq<T>(N) > 0;
}

template <typename T, int N, int MODE>
__global__ void __launch_bounds__(col_block<T>(N))
k_colpipe(ColArgs a)
{
    static_assert(MODE == kPadBwd || MODE == kPadFwd, "pipelined pass: padded modes only");
    constexpr int E = fft_E<T>(N), G = N / E, TC = col_TC<T>(N);
    constexpr int LDSN = lpad_size(N) * TC;
    constexpr int TWQ = pipe_twq<T>(N);
    constexpr int TWN = TWQ * N / 4;
    static_assert(TWQ > 0 && G % 2 == 0, "pipelined pass needs room for the twiddle table");
    __shared__ C<T> sh[LDSN + TWN];
    static_assert(sizeof(sh) <= 160 * 1024, "LDS footprint exceeds 160 KB");

    // This workgroup's tiles: the tiles are split into 8 contiguous ranges,
    // one per XCD (workgroups are dealt to the XCDs round-robin), and the
    // workgroups of an XCD walk its range in lockstep so that neighbouring
    // tiles, which share cache lines, are in flight together.
    const int64_t ntile = (a.ncols + TC - 1) / TC;
    const int64_t total = a.nslab * ntile;
    const int64_t per = (total + 7) / 8;
    const int64_t xcd = blockIdx.x % 8, nw = gridDim.x / 8;
    const int64_t end = total < (xcd + 1) * per ? total : (xcd + 1) * per;
    const int64_t first = xcd * per + blockIdx.x / 8;
    if (first >= end) return;  // whole workgroup: no barrier is reached
    const int niter = int((end - first + nw - 1) / nw);

    const int col = threadIdx.x % TC, t = threadIdx.x / TC;
    const C<T>* twg = (const C<T>*)a.tw;
    for (int j = threadIdx.x; j < TWN; j += blockDim.x) sh[LDSN + j] = twg[tw_off(N) + j];
    const C<T> zt = twg[tw_off(2 * N) + t];  // zeta_{2N}^t
    __syncthreads();
    const LdsTw<T, N, TWQ> tw{sh + LDSN};
    C<T>* lds = sh + col;
    const int64_t in_ld = a.in_ld, out_ld = a.out_ld;

    // Tile it of the sequence: element offsets of its first column (wave
    // uniform) in the input and output arrays, and the rows this thread
    // loads and stores (0 for a column past the end, for loads also a
    // masked column or it past the sequence).  This thread's byte offsets
    // within a tile, (col + t ld) * sizeof(C<T>), are the same for every tile.
    struct Tile {
        int64_t ib, ob;
        int nr, nw;
    };
    auto tile_at = [&](int it, int nrows) {
        const int64_t q = first + int64_t(it < niter ? it : niter - 1) * nw;
        const int64_t slab = q / ntile, tile = q - slab * ntile;
        const int64_t s1 = slab / a.nsub, s2 = slab - s1 * a.nsub;
        const int64_t c = tile * TC + col;
        const bool cin = c < a.ncols;
        bool cact = cin && it < niter;
        if (a.mask_nz > 0) {
            const int64_t cc = cin ? c : 0;
            const int64_t iy = cc / a.mask_nz, iz = cc - iy * a.mask_nz;
            cact = cact && iy >= a.mask_ylo && iy < a.mask_yhi && iz < a.mask_zhi;
        }
        Tile r;
        r.nr = cact ? nrows : 0;
        r.nw = cin ? N : 0;
        r.ib = s1 * a.in_bs + s2 * a.in_bs2 + tile * TC;
        r.ob = s1 * a.out_bs + s2 * a.out_bs2 + tile * TC;
        return r;
    };
    // adjoint forms: the backward pass reads rows reversed within m (row
    // m-1-j for j < m) and/or conjugated, the forward pass writes them
    // reversed; a reversed sequence runs at a negative row step
    const bool rev = a.fsflags & 1, cj = MODE == kPadBwd && (a.fsflags & 2);
    const int64_t rt = rev ? int64_t(a.m) - 1 - t : t;  // first row of this thread (may be < 0: masked)
    const uint32_t ioff = uint32_t((col + (MODE == kPadBwd ? rt : int64_t(t)) * in_ld) * int64_t(sizeof(C<T>)));
    const uint32_t ooff = uint32_t((col + (MODE == kPadFwd ? rt : int64_t(t)) * out_ld) * int64_t(sizeof(C<T>)));
    const uint32_t istep = uint32_t((MODE == kPadBwd && rev ? -1 : 1) * int64_t(G) * in_ld * int64_t(sizeof(C<T>)));
    const uint32_t ostep = uint32_t((MODE == kPadFwd && rev ? -1 : 1) * int64_t(G) * out_ld * int64_t(sizeof(C<T>)));
    // rows t + eG of in[q] for this thread's column, zero at rows >= nr.
    // (The thread offset goes through an empty asm so the compiler forms the
    // E offsets at each use instead of hoisting all of them out of the tile
    // loop, where they would hold E registers for the whole kernel.)
    auto load = [&](C<T> (&v)[E], int q, const Tile& tl, int nr) {
        const i32x4_t rs = buf_rsrc((const C<T>*)a.in[q] + tl.ib);
        uint32_t off = ioff;
        asm volatile("" : "+v"(off));
#pragma unroll
        for (int e = 0; e < E; ++e) {
            v[e] = buf_load<T>(rs, t + e * G < nr ? off + uint32_t(e) * istep : kBufOff);
            if (cj) v[e] = conj(v[e]);
        }
    };
    // rows t + eG of out[q] where keep(e) holds
    auto store = [&](const C<T> (&v)[E], int q, const Tile& tl, auto keep) {
        const i32x4_t rs = buf_rsrc((C<T>*)a.out[q] + tl.ob);
        uint32_t off = ooff;
        asm volatile("" : "+v"(off));
#pragma unroll
        for (int e = 0; e < E; ++e)
            buf_store<T>(rs, t + e * G < tl.nw && keep(e) ? off + uint32_t(e) * ostep : kBufOff, v[e]);
    };
    // zeta_{2N}^{t + eG}
    auto shift = [&](int e) { return e == 0 ? zt : zt * tw[e * (G / 2)]; };

    // The backward loop is rotated so that the wait for a prefetched tile
    // sits inside the loop body, after a fixed number of later memory
    // operations: at a loop header the waitcnt pass would have to merge the
    // prologue's state with the back edge's and wait for everything.
    auto all = [](int) { return true; };
    Tile cur = tile_at(0, MODE == kPadBwd ? a.m : N);
    C<T> x[E];
    if constexpr (MODE == kPadBwd) {
        C<T> xn[E];
        // residue 0: FFT+(U); residue 1: FFT+(zeta_{2N}^k U_k)
        auto residue0 = [&]() {
            C<T> y[E];
#pragma unroll
            for (int e = 0; e < E; ++e) y[e] = x[e];
            fft<T, N, E, +1>(y, t, lds, TC, tw);
            store(y, 0, cur, all);
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = x[e] * shift(e);
        };
        load(x, 0, cur, cur.nr);
        residue0();
        for (int it = 0;; ++it) {
            const Tile nxt = tile_at(it + 1, a.m);
            load(xn, 0, nxt, nxt.nr);
            fft<T, N, E, +1>(x, t, lds, TC, tw);
            store(x, 1, cur, all);
            if (it + 1 >= niter) break;
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = xn[e];
            cur = nxt;
            residue0();
        }
    } else {
        // out_k = s (F0_k + zeta_{2N}^{-k} F1_k), k < m
        const T s = T(a.scale);
        const int m = a.m;
        C<T> y[E];
        for (int it = 0; it < niter; ++it) {
            load(x, 0, cur, cur.nr);
            load(y, 1, cur, cur.nr);
            fft<T, N, E, -1>(x, t, lds, TC, tw);
            fft<T, N, E, -1>(y, t, lds, TC, tw);
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = scale(x[e] + mulc(y[e], shift(e)), s);
            store(x, 0, cur, [&](int e) { return t + e * G < m; });
            cur = tile_at(it + 1, N);
        }
    }
}

}  // namespace impconv
