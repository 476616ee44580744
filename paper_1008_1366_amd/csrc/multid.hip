// multid.hip -- host side of the multi-pass convolutions.
//
// 2D (Sec. 3.1 cconv2 / Sec. 3.2 conv2) and 3D (Sec. 3.4 cconv3 and the
// centered Hermitian analogue): every outer axis is transformed with the
// implicitly padded column pass into 2 (complex) or 3 (centered) residue
// arrays held in the caller's workspace, separate from the data (Sec. 1);
// the innermost axis is convolved row by row with the fused 1D kernels; the
// outer axes are transformed back in reverse order.  Workspace layout puts
// the dot-product index i next to the innermost axis ([.. x'][i][y]), so that
// each row kernel sees uniform row and term strides.
//
// Long 1D complex convolutions use the four-step form: column pass with the
// residue shift and twiddle, cyclic row convolution, column pass back.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "colpass.hpp"
#include "launch.hpp"
#include "multid.hpp"

namespace impconv {

namespace {

size_t csize(int dt) { return dt ? 16 : 8; }

ColArgs col_args(const DevTables& tb, int dt)
{
    ColArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nsub = 1;
    a.tw = tb.tw[dt];
    a.tw3 = tb.tw3[dt];
    a.twlo = tb.twlo;
    a.ncu = tb.ncu;
    a.scale = 1.0;
    return a;
}

RowArgs row_args(const DevTables& tb, int dt)
{
    RowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tw = tb.tw[dt];
    a.tw3 = tb.tw3[dt];
    a.twlo = tb.twlo;
    a.scale = 1.0;
    return a;
}

#define HIPCHK(expr, what)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, what);     \
    } while (0)

}  // namespace

void fourstep_split(int64_t N, int64_t* N1, int64_t* N2)
{
    const int l = ilog2(N);
    *N2 = int64_t(1) << (l / 2);
    *N1 = N / *N2;
}

std::vector<int64_t> fourstep_splits(int64_t N)
{
    std::vector<int64_t> v;
    for (int64_t n2 = 16; n2 <= kColMax && n2 < N; n2 *= 2)
        if (N / n2 <= kRowMax && N / n2 >= 16) v.push_back(n2);
    return v;
}

impconv_status large1d_plan(int dt, int64_t batch, int64_t M, int64_t m, size_t* work)
{
    const int64_t N = next_pow2(m);
    int64_t N1, N2;
    fourstep_split(N, &N1, &N2);
    if (N1 > kRowMax || N2 > kColMax || 2 * N > (int64_t(1) << kTwLog))
        return fail(IMPCONV_E_UNSUPPORTED, "complex 1D convolution supports m <= 131072");
    *work = size_t(4) * batch * M * N * csize(dt);
    return IMPCONV_OK;
}

// Four-step pass sequence shared by the uniform and the ragged batches.
// f_off/m_dev: optional per-pair offsets and lengths (ragged); otherwise pair
// b starts at b * M * m and has length m.
static impconv_status fourstep(const DevTables& tb, int dt, int64_t batch, int64_t M, int64_t m,
                               int64_t N, const void* f, const void* g, void* h, void* work,
                               const int64_t* d_off, const int64_t* d_m, uint32_t flags,
                               hipStream_t s, int64_t n2 = 0)
{
    int64_t N1, N2;
    fourstep_split(N, &N1, &N2);
    if (n2 > 0) {
        N2 = n2;
        N1 = N / n2;
    }
    const size_t cs = csize(dt);
    char* w = static_cast<char*>(work);
    const size_t arr = size_t(batch) * M * N * cs;
    void* Wf[2] = {w, w + arr};
    void* Wg[2] = {w + 2 * arr, w + 3 * arr};
    const void* twfs = fs_twiddles(dt, N2, N1);
    if (!twfs) return IMPCONV_E_HIP;
    // pass 1: residue shift, column FFT (size N2), twiddle -> W[b][j2][i][k1]
    for (int q = 0; q < 2; ++q) {
        ColArgs a = col_args(tb, dt);
        a.in[0] = q ? g : f;
        a.out[0] = q ? Wg[0] : Wf[0];
        a.out[1] = q ? Wg[1] : Wf[1];
        a.nslab = batch * M;
        a.nsub = M;
        a.in_bs = M * m;
        a.in_bs2 = m;
        a.out_bs = M * N;
        a.out_bs2 = N1;
        a.ncols = N1;
        a.out_ld = M * N1;
        a.m = int(m);
        a.nf = N;
        a.twfs = twfs;
        a.slab_off = d_off;
        a.slab_m = d_m;
        a.fsflags = q == 0 ? ((flags & IMPCONV_REV_F) ? 1u : 0u) : ((flags & IMPCONV_CONJ_G) ? 2u : 0u);
        HIPCHK(launch_col(dt, int(N2), kFsBwd, 1, a, s), "four-step pass 1");
    }
    // pass 2: cyclic convolution of the rows (size N1), written in place
    for (int r = 0; r < 2; ++r) {
        RowArgs a = row_args(tb, dt);
        a.f = Wf[r];
        a.g = Wg[r];
        a.h = Wf[r];
        a.nrows = batch * N2;
        a.m = N1;
        a.m_out = N1;
        a.M = M;
        a.f_row = a.g_row = a.h_row = M * N1;
        a.f_i = a.g_i = N1;
        a.scale = 1.0;
        HIPCHK(launch_row_cyclic(dt, int(N1), a, s), "four-step pass 2");
    }
    // pass 3: twiddle, column FFT back, residue recombination, / 2N
    ColArgs a = col_args(tb, dt);
    a.in[0] = Wf[0];
    a.in[1] = Wf[1];
    a.out[0] = h;
    a.nslab = batch;
    a.in_bs = M * N;
    a.in_ld = M * N1;
    a.out_bs = m;
    a.ncols = N1;
    a.m = int(m);
    a.nf = N;
    a.twfs = twfs;
    a.slab_off = d_off;
    a.slab_m = d_m;
    a.fsflags = (flags & IMPCONV_REV_OUT) ? 1u : 0u;
    a.scale = 1.0 / double(2 * N);
    HIPCHK(launch_col(dt, int(N2), kFsFwd, 1, a, s), "four-step pass 3");
    return IMPCONV_OK;
}

impconv_status large1d_run(const DevTables& tb, int dt, int64_t batch, int64_t M, int64_t m,
                           const void* f, const void* g, void* h, void* work, uint32_t flags,
                           hipStream_t s)
{
    return fourstep(tb, dt, batch, M, m, next_pow2(m), f, g, h, work, nullptr, nullptr, flags, s);
}

impconv_status large1d_run_ragged(const DevTables& tb, int dt, int64_t count, int64_t N, int64_t maxm,
                                  const void* f, const void* g, void* h, void* work,
                                  const int64_t* d_off, const int64_t* d_m, uint32_t flags,
                                  hipStream_t s, int64_t n2)
{
    return fourstep(tb, dt, count, 1, maxm, N, f, g, h, work, d_off, d_m, flags, s, n2);
}

// ------------------------------------------------------------------ nD
namespace {

struct PlanND {
    int kind, dt, nd;
    int64_t m[3], n[3], Np[3];  // logical modes, storage extents, padded transform sizes (outer axes)
    int64_t Pe[3];              // Hermitian explicit comparator: padded sizes (last axis: NC, half the real length)
    int64_t batch, M;
    uint32_t flags;
    size_t work;
    int64_t ychunk;             // 3D: (b, x') planes per y-stage chunk
};

// 3D: the y backward pass, the innermost rows and the y forward pass run
// over chunks of the (b, x') planes, with two sets of y-residue arrays sized
// for a chunk, used by the chunks in turn.  With c chunks (fewer when there
// are fewer planes) that region is 2 / c of the full y-residue volume.
// Centered Hermitian: c = 8 keeps the 3D work memory under the explicitly
// padded method's storage (Sec. 3.4 storage counts; c = 4 would exceed it)
// while every launch still spans many planes.  Complex: the y residues are
// fewer (two per axis) and the bound holds for any c; c = 2 (256^3, batch 2:
// 2.93 -> 2.80 ms in complex64, 5.10 -> 4.79 ms in complex128 against c = 8)
// keeps the launches long and still lets one chunk's rows run beside the
// other chunk's y backward pass.
#ifndef IMPCONV_3D_YCHUNKS
#define IMPCONV_3D_YCHUNKS 8
#endif
constexpr int64_t kYChunks = IMPCONV_3D_YCHUNKS;
constexpr int64_t kYChunksComplex = 2;
int64_t y_chunk_planes(int64_t planes, int64_t chunks)
{
    return std::max<int64_t>(1, (planes + chunks - 1) / chunks);
}

impconv_status plannd(int kind, int dt, int nd, const int64_t* m, const int64_t* n, int64_t batch,
                      int64_t M, uint32_t flags, PlanND* p)
{
    if (dt != IMPCONV_C64 && dt != IMPCONV_C128) return fail(IMPCONV_E_ARG, "bad dtype");
    if (kind != IMPCONV_COMPLEX && kind != IMPCONV_HERMITIAN && kind != IMPCONV_TERNARY)
        return fail(IMPCONV_E_ARG, "nD kind must be COMPLEX, HERMITIAN or TERNARY");
    if (kind == IMPCONV_TERNARY && nd != 2) return fail(IMPCONV_E_UNSUPPORTED, "ternary nD convolutions are 2D (tconv2)");
    if (kind == IMPCONV_TERNARY && M != 1) return fail(IMPCONV_E_SIZE, "ternary convolutions take M = 1");
    if (!m || !n) return fail(IMPCONV_E_ARG, "m or n is NULL");
    if (batch < 0 || M < 1) return fail(IMPCONV_E_SIZE, "batch must be >= 0 and M >= 1");
    const uint32_t adj = IMPCONV_REV_F | IMPCONV_CONJ_G | IMPCONV_REV_OUT;
    const uint32_t known = IMPCONV_NO_SYMMETRIZE | IMPCONV_EXPLICIT_PADDED | IMPCONV_EXPLICIT_PRUNED | adj |
                           IMPCONV_HERMITIAN_ADJOINT | IMPCONV_COMPENSATED | IMPCONV_ONE_STREAM;
    if (flags & ~known) return fail(IMPCONV_E_ARG, "unsupported flag for an nD convolution");
    if ((flags & IMPCONV_COMPENSATED) && (kind != IMPCONV_COMPLEX || (flags & IMPCONV_EXPLICIT_PADDED)))
        return fail(IMPCONV_E_ARG, "COMPENSATED applies to implicit complex nD convolutions");
    if ((flags & IMPCONV_HERMITIAN_ADJOINT) &&
        (kind != IMPCONV_HERMITIAN || (flags & (IMPCONV_EXPLICIT_PADDED | IMPCONV_NO_SYMMETRIZE))))
        return fail(IMPCONV_E_ARG, "HERMITIAN_ADJOINT applies to implicit, symmetrized Hermitian nD convolutions");
    if ((flags & IMPCONV_EXPLICIT_PRUNED) && !(flags & IMPCONV_EXPLICIT_PADDED))
        return fail(IMPCONV_E_ARG, "EXPLICIT_PRUNED qualifies EXPLICIT_PADDED");
    if ((flags & adj) && (kind != IMPCONV_COMPLEX || (flags & IMPCONV_EXPLICIT_PADDED)))
        return fail(IMPCONV_E_ARG, "REV/CONJ flags apply to implicit complex nD convolutions");
    std::memset(p, 0, sizeof(*p));
    p->kind = kind; p->dt = dt; p->nd = nd; p->batch = batch; p->M = M; p->flags = flags;
    for (int d = 0; d < nd; ++d) {
        p->m[d] = m[d];
        p->n[d] = n[d];
        if (m[d] < 1) return fail(IMPCONV_E_SIZE, "m must be >= 1 on every axis");
        const bool last = d == nd - 1;
        if (kind == IMPCONV_COMPLEX) {
            if (n[d] != m[d]) return fail(IMPCONV_E_SIZE, "complex nD storage requires n == m");
        } else if (!last) {
            if (n[d] != 2 * m[d] - 1 && n[d] != 2 * m[d]) return fail(IMPCONV_E_SIZE, "centered axis needs n = 2m-1 or 2m");
        } else {
            if (n[d] != m[d] && n[d] != m[d] + 1) return fail(IMPCONV_E_SIZE, "Hermitian axis needs n = m or m+1");
        }
        p->Np[d] = next_pow2(m[d]);
        if (!last && p->Np[d] > kColMax) return fail(IMPCONV_E_UNSUPPORTED, "outer axis too long (m <= 4096)");
        if (!last && kind == IMPCONV_TERNARY && 2 * p->Np[d] > kTerColMax[dt])
            return fail(IMPCONV_E_UNSUPPORTED, dt ? "ternary outer axis too long (complex128: m <= 2048)"
                                                  : "ternary outer axis too long (complex64: m <= 4096)");
        if (last) {
            int64_t L = kind == IMPCONV_COMPLEX || kind == IMPCONV_TERNARY ? p->Np[d]
                                                                          : std::max<int64_t>(p->Np[d], 2) / 2;
            if (L > kRowMax) return fail(IMPCONV_E_UNSUPPORTED, "innermost axis too long");
        }
    }
    const size_t cs = csize(dt);
    const int R = kind == IMPCONV_COMPLEX ? 2 : 3;
    if ((flags & IMPCONV_EXPLICIT_PADDED) && kind == IMPCONV_HERMITIAN) {
        // conventional 2/3 rule: every centered axis zero padded to the power
        // of two P >= 3m - 2, the Hermitian axis to the real length
        // 2 NC >= 3m - 2 (half spectrum NC + 1); padded f and g are
        // [b][P0]([P1])[M][NC + 1]
        size_t vol = 1;
        for (int d = 0; d < nd - 1; ++d) {
            p->Pe[d] = next_pow2(std::max<int64_t>(3 * m[d] - 2, 1));
            if (p->Pe[d] > kColMax) return fail(IMPCONV_E_UNSUPPORTED, "explicit Hermitian comparator: 3m - 2 <= 4096 on the centered axes");
            vol *= size_t(p->Pe[d]);
        }
        p->Pe[nd - 1] = next_pow2(std::max<int64_t>(3 * m[nd - 1] - 2, 2)) / 2;
        if (p->Pe[nd - 1] > kRowMax) return fail(IMPCONV_E_UNSUPPORTED, "explicit Hermitian comparator: 3m - 2 <= 16384 on the last axis");
        p->work = size_t(2) * batch * M * vol * size_t(p->Pe[nd - 1] + 1) * cs;
        return IMPCONV_OK;
    }
    if ((flags & IMPCONV_EXPLICIT_PADDED) && kind == IMPCONV_COMPLEX && nd == 3) {
        // padded f and g, [b][2N0][2N1][M][2N2] (pruned: only the m2 data
        // columns of the last axis, [b][2N0][2N1][M][m2])
        const int64_t P0 = 2 * p->Np[0], P1 = 2 * p->Np[1], P2 = 2 * p->Np[2];
        if (P0 > kColMax || P1 > kColMax || P2 > kRowMax)
            return fail(IMPCONV_E_UNSUPPORTED, "explicit 3D complex comparator supports m0, m1 <= 2048, m2 <= 4096");
        p->work = size_t(2) * batch * M * P0 * P1 * ((flags & IMPCONV_EXPLICIT_PRUNED) ? m[2] : P2) * cs;
        return IMPCONV_OK;
    }
    if ((flags & IMPCONV_EXPLICIT_PADDED) && kind == IMPCONV_COMPLEX) {
        // padded f and g, [b][2N0][M][2N1] (pruned: only the m1 data columns, [b][2N0][M][m1])
        const int64_t P0 = 2 * p->Np[0], P1 = 2 * p->Np[1];
        if (P0 > kColMax || P1 > kRowMax) return fail(IMPCONV_E_UNSUPPORTED, "explicit 2D comparator supports m <= 2048 per axis");
        p->work = size_t(2) * batch * M * P0 * ((flags & IMPCONV_EXPLICIT_PRUNED) ? n[1] : P1) * cs;
        return IMPCONV_OK;
    }
    if (kind == IMPCONV_TERNARY && (flags & IMPCONV_EXPLICIT_PADDED)) {
        // padded f, g, e: [b][4 Np0][2 Np1 + 1] (x padded to 4 Np0, y real length 4 Np1)
        const int64_t P0 = 4 * p->Np[0], L = 2 * p->Np[1] + 1;
        if (P0 > kFftColMax[dt] || 2 * p->Np[1] > kRowMax)
            return fail(IMPCONV_E_UNSUPPORTED, dt ? "explicit ternary 2D comparator supports m0 <= 1024, m1 <= 4096"
                                                  : "explicit ternary 2D comparator supports m0 <= 4096, m1 <= 4096");
        p->work = size_t(3) * batch * P0 * L * cs;
    } else if (kind == IMPCONV_TERNARY) {
        // x residues of f, g, e (2 each, 2 Np0 rows); the rows write their
        // result over the residues of f unless the row kernel accumulates
        // in its output (then two more arrays)
        const int extra = row_ternary_accumulates(dt, int(p->Np[1])) ? 2 : 0;
        p->work = size_t(6 + extra) * batch * 2 * p->Np[0] * n[1] * cs;
    } else if (nd == 2) {
        // residue arrays [b][x'][i][y] for f and g
        p->work = size_t(2) * R * batch * M * p->Np[0] * n[1] * cs;
    } else {
        // x-residue arrays of f and g (the y-forward output of each plane is
        // written back into its own x-residue plane), plus two sets of
        // y-residue arrays of one chunk of planes, used by the chunks in turn
        // (the rows of one chunk run beside the y pass of the next)
        const size_t X = size_t(2) * R * batch * M * p->Np[0] * n[1] * n[2];
        const int64_t planes = batch * p->Np[0];
        p->ychunk = y_chunk_planes(planes, kind == IMPCONV_COMPLEX ? kYChunksComplex : kYChunks);
        const size_t Y = size_t(2) * R * p->ychunk * M * p->Np[1] * n[2];
        p->work = (X + 2 * Y) * cs;
    }
    return IMPCONV_OK;
}

// Outer-axis backward pass of one input array (f or g).
// src: [B][M][n0][cols], dst[r]: [B][N0][M][cols] (r < R)
impconv_status outer_bwd(const DevTables& tb, const PlanND& p, const void* src, void* const* dst,
                         int64_t nslab1, int64_t in_bs1, int64_t n0, int64_t m0, int64_t N0,
                         int64_t cols, int sym, int64_t sym_nz, int sym_offy, int sym_ny,
                         int64_t mask_nz, int mask_ylo, int mask_yhi, int mask_zhi, hipStream_t s,
                         uint32_t fsflags = 0)
{
    ColArgs a = col_args(tb, p.dt);
    a.fsflags = fsflags;
    a.in[0] = src;
    for (int r = 0; r < 3; ++r) a.out[r] = dst[r];
    a.nslab = nslab1 * p.M;
    a.nsub = p.M;
    a.in_bs = in_bs1;
    a.in_bs2 = n0 * cols;
    a.out_bs = N0 * p.M * cols;
    a.out_bs2 = cols;
    a.ncols = cols;
    a.in_ld = cols;
    a.out_ld = p.M * cols;
    a.n_in = int(n0);
    a.m = int(m0);
    a.off_in = int(n0 - m0);
    a.sym = sym;
    a.sym_nz = sym_nz;
    a.sym_offy = sym_offy;
    a.sym_ny = sym_ny;
    a.mask_nz = mask_nz;
    a.mask_ylo = mask_ylo;
    a.mask_yhi = mask_yhi;
    a.mask_zhi = mask_zhi;
    const int mode = p.kind == IMPCONV_COMPLEX ? kPadBwd : kCenBwd;
    HIPCHK(launch_col(p.dt, int(N0), mode, 1, a, s), "outer backward pass");
    return IMPCONV_OK;
}

// Outer-axis forward pass: src[r]: [B][N0][ld=ldin] -> dst [B][n0][cols]
impconv_status outer_fwd(const DevTables& tb, const PlanND& p, void* const* src, void* dst,
                         int64_t nslab, int64_t in_bs, int64_t in_ld, int64_t n0, int64_t m0,
                         int64_t N0, int64_t cols, hipStream_t s, uint32_t fsflags = 0, int sym = 0,
                         int64_t sym_nz = 0, int sym_offy = 0, int sym_ny = 0)
{
    ColArgs a = col_args(tb, p.dt);
    a.fsflags = fsflags;
    a.sym = sym;
    a.sym_nz = sym_nz;
    a.sym_offy = sym_offy;
    a.sym_ny = sym_ny;
    for (int r = 0; r < 3; ++r) a.in[r] = src[r];
    a.out[0] = dst;
    a.nslab = nslab;
    a.in_bs = in_bs;
    a.out_bs = n0 * cols;
    a.ncols = cols;
    a.in_ld = in_ld;
    a.out_ld = cols;
    a.n_out = int(n0);
    a.m = int(m0);
    a.off_out = int(n0 - m0);
    const bool cx = p.kind == IMPCONV_COMPLEX;
    a.scale = 1.0 / double((cx ? 2 : 3) * N0);
    HIPCHK(launch_col(p.dt, int(N0), cx ? kPadFwd : kCenFwd, 1, a, s), "outer forward pass");
    return IMPCONV_OK;
}

// Innermost-axis row convolutions over nrows rows, in place in f.
impconv_status inner_rows(const DevTables& tb, const PlanND& p, void* f, const void* g,
                          int64_t nrows, hipStream_t s, uint32_t rowflags = 0);

// The rows of R residue arrays: one launch over all of them where the arrays
// lie back to back (the rows then have one uniform stride), else one launch
// per residue.  Fewer, longer launches leave less of the chip idle at each
// launch's tail.
impconv_status inner_rows_residues(const DevTables& tb, const PlanND& p, void* const* f, const void* const* g,
                                   int R, int64_t nrows, hipStream_t s, uint32_t rowflags = 0)
{
    const size_t arr = size_t(nrows) * p.M * p.n[p.nd - 1] * csize(p.dt);
    bool contiguous = true;
    for (int r = 1; r < R; ++r)
        contiguous = contiguous && static_cast<const char*>(f[r]) == static_cast<const char*>(f[0]) + r * arr &&
                     static_cast<const char*>(g[r]) == static_cast<const char*>(g[0]) + r * arr;
    if (contiguous) return inner_rows(tb, p, f[0], g[0], R * nrows, s, rowflags);
    impconv_status st = IMPCONV_OK;
    for (int r = 0; r < R && !st; ++r) st = inner_rows(tb, p, f[r], g[r], nrows, s, rowflags);
    return st;
}

impconv_status inner_rows(const DevTables& tb, const PlanND& p, void* f, const void* g,
                          int64_t nrows, hipStream_t s, uint32_t rowflags)
{
    const int nd = p.nd;
    const int64_t m = p.m[nd - 1], n = p.n[nd - 1];
    RowArgs a = row_args(tb, p.dt);
    a.f = f;
    a.g = g;
    a.h = f;
    a.nrows = nrows;
    a.m = m;
    a.M = p.M;
    a.f_row = a.g_row = a.h_row = p.M * n;
    a.f_i = a.g_i = n;
    a.h_pad = n;
    a.flags = rowflags;
    hipError_t e;
    if (p.kind == IMPCONV_COMPLEX) {
        e = launch_row_complex(p.dt, int(p.Np[nd - 1]), a, s);
    } else {
        e = launch_row_hermitian(p.dt, int(std::max<int64_t>(p.Np[nd - 1], 2) / 2), a, s);
    }
    HIPCHK(e, "inner row convolution");
    return IMPCONV_OK;
}

// 2D centered Hermitian ternary convolution (Sec. 4, tconv2): the x axis
// is transformed with the ternary rule (two residues of the centered
// transform padded to 4 N0', kTerBwd), every row of each residue is
// convolved with the 1D ternary kernel, and the x axis is transformed back
// (kTerFwd).  Layouts: f, g, e, h [b][n0][n1]; residues [b][2 N0'][n1].
impconv_status run2d_ternary(int dt, int64_t batch, const int64_t* m, const int64_t* n, const void* f,
                             const void* g, const void* e, void* h, void* work, size_t wb, uint32_t flags,
                             void* stream)
{
    PlanND p;
    impconv_status st = plannd(IMPCONV_TERNARY, dt, 2, m, n, batch, 1, flags, &p);
    if (st) return st;
    if (batch == 0) return IMPCONV_OK;
    const size_t cs = csize(dt);
    if (!f || !g || !e || !h) return fail(IMPCONV_E_ARG, "null data pointer");
    for (const void* q : {f, g, e, (const void*)h})
        if (reinterpret_cast<uintptr_t>(q) % cs) return fail(IMPCONV_E_ALIGN, "data pointer misaligned");
    const int64_t n0 = n[0], n1 = n[1], m0 = m[0], m1 = m[1];
    const size_t vol = size_t(batch) * n0 * n1 * cs;
    if (bad_alias(h, vol, f, vol) || bad_alias(h, vol, g, vol) || bad_alias(h, vol, e, vol))
        return fail(IMPCONV_E_ARG, "h overlaps an input (only h == input of the same extent is allowed)");
    if (wb < p.work) return fail(IMPCONV_E_WORKSPACE, "workspace too small: need " + std::to_string(p.work) + " bytes");
    if (!work) return fail(IMPCONV_E_ARG, "work is NULL");
    if (reinterpret_cast<uintptr_t>(work) % cs) return fail(IMPCONV_E_ALIGN, "work misaligned");
    const DevTables* tbp = tables();
    if (!tbp) return IMPCONV_E_HIP;
    const DevTables& tb = *tbp;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool sym = !(flags & IMPCONV_NO_SYMMETRIZE);
    if (flags & IMPCONV_EXPLICIT_PADDED) {
        // Conventional method: f, g, e copied into zero-padded [4 N0'][2 N1' + 1]
        // arrays (k_x at row k_x mod 4 N0', so every x point of the transform is
        // a real field in y; k_y < m1 at column k_y), a full-size complex FFT
        // along x, a real cyclic triple product of length 4 N1' along y, the
        // inverse x FFT, and the crop.  No alias of |k_x| <= 3(m0-1) reaches
        // an output |k_x| < m0 since 4 N0' >= 4 m0.  The k_y = 0 line is read
        // by the c2r transform, i.e. as its Hermitian projection (the same as
        // the implicit path for symmetric input).
        const int64_t P0 = 4 * p.Np[0], NC = 2 * p.Np[1], L = NC + 1;
        const bool pruned = flags & IMPCONV_EXPLICIT_PRUNED;
        const size_t arr = size_t(batch) * P0 * L * cs;
        char* w = static_cast<char*>(work);
        void* W[3] = {w, w + arr, w + 2 * arr};
        const void* src[3] = {f, g, e};
        const int64_t r0 = n0 - m0;          // stored row of k_x = 0
        const int64_t s0 = n0 - (2 * m0 - 1);  // stored row of k_x = -m0+1
        auto rowp = [&](const void* base, int64_t row, int64_t ld) {
            return static_cast<const char*>(base) + row * ld * int64_t(cs);
        };
        for (int q = 0; q < 3; ++q) {
            // k_x >= 0 (and zero fill of the whole array), then k_x < 0 at the top
            HIPCHK(launch_copy2d(dt, rowp(src[q], r0, n1), W[q], batch, 1, n0 * n1, 0, n1, P0 * L, 0, L, m0, m1,
                                 P0, L, s), "explicit pad");
            HIPCHK(launch_copy2d(dt, rowp(src[q], s0, n1), (void*)rowp(W[q], P0 - m0 + 1, L), batch, 1, n0 * n1, 0,
                                 n1, P0 * L, 0, L, m0 - 1, m1, m0 - 1, L, s), "explicit pad");
            ColArgs a = col_args(tb, dt);
            a.in[0] = a.out[0] = W[q];
            a.nslab = batch;
            a.in_bs = a.out_bs = P0 * L;
            a.ncols = pruned ? m1 : L;  // pruned: the all-zero columns k_y >= m1 stay zero
            a.in_ld = a.out_ld = L;
            a.n_in = a.n_out = int(P0);
            HIPCHK(launch_col(dt, int(P0), kFft, 1, a, s), "explicit x FFT");
        }
        RowArgs ra = row_args(tb, dt);
        ra.f = W[0]; ra.g = W[1]; ra.e = W[2]; ra.h = W[0];
        ra.nrows = batch * P0;
        ra.m = pruned ? m1 : L;
        ra.m_out = m1;
        ra.M = 1;
        ra.f_row = ra.g_row = ra.e_row = ra.h_row = L;
        ra.scale = 1.0 / double(2 * NC);
        HIPCHK(launch_row_realcyclic(dt, int(NC), ra, s), "explicit y triple product");
        ColArgs a = col_args(tb, dt);
        a.in[0] = a.out[0] = W[0];
        a.nslab = batch;
        a.in_bs = a.out_bs = P0 * L;
        a.ncols = m1;
        a.in_ld = a.out_ld = L;
        a.n_in = a.n_out = int(P0);
        a.scale = 1.0 / double(P0);
        HIPCHK(launch_col(dt, int(P0), kFft, -1, a, s), "explicit inverse x FFT");
        HIPCHK(launch_copy2d(dt, W[0], (void*)rowp(h, r0, n1), batch, 1, P0 * L, 0, L, n0 * n1, 0, n1, m0, m1, m0,
                             n1, s), "explicit crop");
        HIPCHK(launch_copy2d(dt, rowp(W[0], P0 - m0 + 1, L), (void*)rowp(h, s0, n1), batch, 1, P0 * L, 0, L,
                             n0 * n1, 0, n1, m0 - 1, m1, m0 - 1, n1, s), "explicit crop");
        if (s0 > 0)  // zero slot row k_x = -m0
            HIPCHK(launch_copy2d(dt, h, h, batch, 1, 0, 0, 0, n0 * n1, 0, n1, 0, 0, 1, n1, s), "zero slot");
        return IMPCONV_OK;
    }
    const int64_t P0 = 2 * p.Np[0];  // x transform size (residues of the 4 N0' padding)
    const size_t arr = size_t(batch) * P0 * n1 * cs;
    char* w = static_cast<char*>(work);
    void* X[3][2];
    for (int q = 0; q < 3; ++q)
        for (int r = 0; r < 2; ++r) X[q][r] = w + (2 * q + r) * arr;
    void* Q[2] = {X[0][0], X[0][1]};
    if (row_ternary_accumulates(dt, int(p.Np[1]))) {
        Q[0] = w + 6 * arr;
        Q[1] = w + 7 * arr;
    }
    const void* src[3] = {f, g, e};
    for (int q = 0; q < 3; ++q) {
        ColArgs a = col_args(tb, dt);
        a.in[0] = src[q];
        a.out[0] = X[q][0];
        a.out[1] = X[q][1];
        a.nslab = batch;
        a.in_bs = n0 * n1;
        a.out_bs = P0 * n1;
        a.ncols = n1;
        a.in_ld = a.out_ld = n1;
        a.n_in = int(n0);
        a.m = int(m0);
        a.off_in = int(n0 - m0);
        a.sym = sym ? 1 : 0;
        a.mask_nz = n1;  // columns k_y < m1 carry data; k_y = m1 is a zero slot
        a.mask_ylo = 0;
        a.mask_yhi = 1;
        a.mask_zhi = int(m1);
        HIPCHK(launch_col(dt, int(P0), kTerBwd, 1, a, s), "ternary x backward pass");
    }
    for (int r = 0; r < 2; ++r) {
        RowArgs a = row_args(tb, dt);
        a.f = X[0][r];
        a.g = X[1][r];
        a.e = X[2][r];
        a.h = Q[r];
        a.nrows = batch * P0;
        a.m = m1;
        a.M = 1;
        a.f_row = a.g_row = a.e_row = a.h_row = n1;
        a.h_pad = n1;
        HIPCHK(launch_row_ternary(dt, int(p.Np[1]), a, s), "ternary row convolutions");
    }
    ColArgs a = col_args(tb, dt);
    a.in[0] = Q[0];
    a.in[1] = Q[1];
    a.out[0] = h;
    a.nslab = batch;
    a.in_bs = P0 * n1;
    a.out_bs = n0 * n1;
    a.ncols = n1;
    a.in_ld = a.out_ld = n1;
    a.n_out = int(n0);
    a.m = int(m0);
    a.off_out = int(n0 - m0);
    a.mask_nz = n1;
    a.mask_ylo = 0;
    a.mask_yhi = 1;
    a.mask_zhi = int(m1);
    a.scale = 1.0 / double(2 * P0);
    HIPCHK(launch_col(dt, int(P0), kTerFwd, 1, a, s), "ternary x forward pass");
    return IMPCONV_OK;
}


// Conventional centered Hermitian nD comparator (Secs. 3.2, 3.4 timing
// comparisons): f and g copied into zero-padded arrays, every centered axis
// of length P >= 3m - 2 (wavenumber k at index k mod P, so each line of the
// transform is a real field in the last axis), the last axis as the half
// spectrum of a real length 2 NC >= 3m - 2; full-size complex FFTs along the
// centered axes, real cyclic products (M-dot) along the last axis, inverse
// FFTs, crop.  No alias of |k| <= 2(m - 1) reaches an output |k| < m.  The
// k_last = 0 hyperplane is read by the real transforms, i.e. as its
// Hermitian projection (equal to the implicit path's reading for symmetric
// input).  pruned: no transform of a column that is all zero -- the x FFTs
// run over the data rows of y and the data columns of the last axis only,
// the y FFTs over the data columns, the inverse x FFT over the rows the crop
// keeps.
impconv_status run_herm_explicit(const DevTables& tb, const PlanND& p, const void* f, const void* g, void* h,
                                 char* w, hipStream_t s, bool pruned)
{
    const int nd = p.nd, dt = p.dt;
    const int64_t B = p.batch, M = p.M;
    const size_t cs = csize(dt);
    const int64_t NC = p.Pe[nd - 1], L = NC + 1;
    const int64_t m2 = p.m[nd - 1], n2 = p.n[nd - 1];
    const int64_t P0 = p.Pe[0], P1 = nd == 3 ? p.Pe[1] : 1;
    const int64_t m0 = p.m[0], n0 = p.n[0], m1 = nd == 3 ? p.m[1] : 1, n1 = nd == 3 ? p.n[1] : 1;
    const int64_t vol = P0 * P1;                      // padded centered points
    const size_t arr = size_t(B) * vol * M * L * cs;  // one padded input
    void* W[2] = {w, w + arr};
    const void* src[2] = {f, g};
    auto at = [&](const void* base, int64_t elems) {
        return static_cast<const char*>(base) + elems * int64_t(cs);
    };
    auto atw = [&](void* base, int64_t elems) { return static_cast<char*>(base) + elems * int64_t(cs); };
    // centered index ranges: (first stored row, first padded row, count) for k >= 0 and k < 0
    struct Seg { int64_t src0, dst0, cnt; };
    auto segs = [](int64_t m, int64_t n, int64_t P) {
        std::vector<Seg> v;
        v.push_back({n - m, 0, m});                      // k = 0..m-1
        if (m > 1) v.push_back({n - 2 * m + 1, P - m + 1, m - 1});  // k = -m+1..-1
        return v;
    };
    const auto sx = segs(m0, n0, P0);
    const auto sy = nd == 3 ? segs(m1, n1, P1) : std::vector<Seg>{{0, 0, 1}};
    const int64_t sin_b = M * n0 * n1 * n2, sin_i = n0 * n1 * n2;   // input strides: batch, term
    for (int q = 0; q < 2; ++q) {
        // zero the padded array, then copy the (x, y) blocks of k_last < m
        HIPCHK(launch_copy2d(dt, W[q], W[q], 1, 1, 0, 0, 0, 0, 0, L, 0, 0, B * vol * M, L, s), "explicit zero");
        for (int64_t b = 0; b < B; ++b)
            for (const Seg& X : sx)
                for (const Seg& Y : sy) {
                    // per x row (nb) and term (nsub): a block of Y.cnt rows x m2 columns
                    const void* sp = at(src[q], b * sin_b + (X.src0 * n1 + Y.src0) * n2);
                    void* dp = atw(W[q], ((b * P0 + X.dst0) * P1 + Y.dst0) * M * L);
                    HIPCHK(launch_copy2d(dt, sp, dp, X.cnt * M, M, n1 * n2, sin_i, n2, P1 * M * L, L, M * L, Y.cnt, m2,
                                         Y.cnt, m2, s), "explicit pad");
                }
        // FFT along x over the columns (y', i, z) of each batch entry
        if (!pruned) {
            ColArgs a = col_args(tb, dt);
            a.in[0] = a.out[0] = W[q];
            a.nslab = B;
            a.in_bs = a.out_bs = vol * M * L;
            a.ncols = P1 * M * L;
            a.in_ld = a.out_ld = P1 * M * L;
            a.n_in = a.n_out = int(P0);
            HIPCHK(launch_col(dt, int(P0), kFft, 1, a, s), "explicit x FFT");
        } else {
            // slabs (b, y' data row, i), columns z < m2: (y', i) sit at (y' M + i) L
            for (const Seg& Y : sy) {
                ColArgs a = col_args(tb, dt);
                a.in[0] = a.out[0] = atw(W[q], Y.dst0 * M * L);
                a.nslab = B * Y.cnt * M;
                a.nsub = Y.cnt * M;
                a.in_bs = a.out_bs = vol * M * L;
                a.in_bs2 = a.out_bs2 = L;
                a.ncols = m2;
                a.in_ld = a.out_ld = P1 * M * L;
                a.n_in = a.n_out = int(P0);
                HIPCHK(launch_col(dt, int(P0), kFft, 1, a, s), "explicit x FFT");
            }
        }
        if (nd == 3) {
            // FFT along y in every (b, x') plane; pruned: slabs (b x', i), columns z < m2
            ColArgs c = col_args(tb, dt);
            c.in[0] = c.out[0] = W[q];
            c.nslab = B * P0 * (pruned ? M : 1);
            c.nsub = pruned ? M : 1;
            c.in_bs = c.out_bs = P1 * M * L;
            c.in_bs2 = c.out_bs2 = pruned ? L : 0;
            c.ncols = pruned ? m2 : M * L;
            c.in_ld = c.out_ld = M * L;
            c.n_in = c.n_out = int(P1);
            HIPCHK(launch_col(dt, int(P1), kFft, 1, c, s), "explicit y FFT");
        }
    }
    // real cyclic products along the last axis, summed over the M terms, into term 0 of W[0]
    RowArgs ra = row_args(tb, dt);
    ra.f = W[0]; ra.g = W[1]; ra.h = W[0];
    ra.nrows = B * vol;
    ra.m = pruned ? m2 : L;  // the entries from m2 on are zero
    ra.m_out = m2;
    ra.M = M;
    ra.f_row = ra.g_row = ra.h_row = M * L;
    ra.f_i = ra.g_i = L;
    ra.scale = 1.0 / double(2 * NC);
    HIPCHK(launch_row_realcyclic(dt, int(NC), ra, s), "explicit last-axis products");
    if (nd == 3) {
        ColArgs c = col_args(tb, dt);
        c.in[0] = c.out[0] = W[0];
        c.nslab = B * P0;
        c.in_bs = c.out_bs = P1 * M * L;
        c.ncols = m2;
        c.in_ld = c.out_ld = M * L;
        c.n_in = c.n_out = int(P1);
        c.scale = 1.0 / double(P1);
        HIPCHK(launch_col(dt, int(P1), kFft, -1, c, s), "explicit inverse y FFT");
    }
    // inverse x FFT of term 0: slabs (b, y'), columns z < m2, rows x' (stride
    // P1 M L); pruned: only the y' rows the crop keeps
    const std::vector<Seg> yall{{0, 0, P1}};
    for (const Seg& Y : pruned ? sy : yall) {
        ColArgs a = col_args(tb, dt);
        a.in[0] = a.out[0] = atw(W[0], Y.dst0 * M * L);
        a.nslab = B * Y.cnt;
        a.nsub = Y.cnt;
        a.in_bs = a.out_bs = vol * M * L;
        a.in_bs2 = a.out_bs2 = M * L;
        a.ncols = m2;
        a.in_ld = a.out_ld = P1 * M * L;
        a.n_in = a.n_out = int(P0);
        a.scale = 1.0 / double(P0);
        HIPCHK(launch_col(dt, int(P0), kFft, -1, a, s), "explicit inverse x FFT");
    }
    // crop into h (zero slots and the Hermitian slot column stay zero)
    HIPCHK(launch_copy2d(dt, h, h, 1, 1, 0, 0, 0, 0, 0, n2, 0, 0, B * n0 * n1, n2, s), "explicit zero output");
    for (int64_t b = 0; b < B; ++b)
        for (const Seg& X : sx)
            for (const Seg& Y : sy) {
                const void* sp = at(W[0], ((b * P0 + X.dst0) * P1 + Y.dst0) * M * L);
                void* dp = static_cast<char*>(h) + ((b * n0 + X.src0) * n1 + Y.src0) * n2 * int64_t(cs);
                HIPCHK(launch_copy2d(dt, sp, dp, X.cnt, 1, P1 * M * L, 0, M * L, n1 * n2, 0, n2, Y.cnt, m2, Y.cnt,
                                     m2, s), "explicit crop");
            }
    return IMPCONV_OK;
}

// Conventional 3D complex comparator (Sec. 3.4 timing comparison): inputs
// zero padded to P_d = 2 N_d per axis (N_d = 2^ceil(log2 m_d)), full-size
// FFTs along x, y and z, product summed over the M terms, inverse
// transforms, crop.  Padded arrays W[q] are [b][P0][P1][M][Z], Z = P2.
// Pruned: the padding is never materialized and no all-zero column is
// transformed -- the x FFTs read the m0 stored rows of the m1 x m2 data
// columns straight from f and g, the y FFTs run on the m2 data columns of
// every x' plane, the z rows read their m2 data entries (zero beyond, Z =
// m2 stored) and keep m2 outputs, and the inverse y / x FFTs produce only
// the m1 / m0 rows the crop keeps, the last one writing h directly.
impconv_status run_complex3d_explicit(const DevTables& tb, const PlanND& p, const void* f, const void* g,
                                      void* h, char* w, hipStream_t s, bool pruned)
{
    const int dt = p.dt;
    const int64_t B = p.batch, M = p.M;
    const size_t cs = csize(dt);
    const int64_t m0 = p.m[0], m1 = p.m[1], m2 = p.m[2];
    const int64_t P0 = 2 * p.Np[0], P1 = 2 * p.Np[1], P2 = 2 * p.Np[2];
    const int64_t Z = pruned ? m2 : P2;                 // stored last-axis entries of W
    const int64_t plane = P1 * M * Z;                   // one x' plane of W
    const size_t arr = size_t(B) * P0 * plane * cs;     // one padded input
    void* W[2] = {w, w + arr};
    const void* src[2] = {f, g};
    const int64_t sin_i = m0 * m1 * m2, sin_b = M * sin_i;  // input strides: term, batch
    auto atw = [&](void* base, int64_t elems) { return static_cast<char*>(base) + elems * int64_t(cs); };
    auto atc = [&](const void* base, int64_t elems) { return static_cast<const char*>(base) + elems * int64_t(cs); };
    for (int q = 0; q < 2; ++q) {
        if (!pruned) {
            HIPCHK(launch_copy2d(dt, W[q], W[q], 1, 1, 0, 0, 0, 0, 0, Z, 0, 0, B * P0 * P1 * M, Z, s), "explicit zero");
            // per batch entry: slabs (x < m0, i), blocks of m1 rows (y) x m2 columns (z)
            for (int64_t b = 0; b < B; ++b)
                HIPCHK(launch_copy2d(dt, atc(src[q], b * sin_b), atw(W[q], b * P0 * plane), m0 * M, M, m1 * m2, sin_i, m2,
                                     plane, Z, M * Z, m1, m2, m1, m2, s), "explicit pad");
            // x FFT over every (y', i, z) column of each batch entry
            ColArgs a = col_args(tb, dt);
            a.in[0] = a.out[0] = W[q];
            a.nslab = B;
            a.in_bs = a.out_bs = P0 * plane;
            a.ncols = plane;
            a.in_ld = a.out_ld = plane;
            a.n_in = a.n_out = int(P0);
            HIPCHK(launch_col(dt, int(P0), kFft, 1, a, s), "explicit x FFT");
        } else {
            // x FFT of the data columns (y < m1, z < m2) read from the input:
            // per batch entry, slabs (i, y), columns z
            for (int64_t b = 0; b < B; ++b) {
                ColArgs a = col_args(tb, dt);
                a.in[0] = atc(src[q], b * sin_b);
                a.out[0] = atw(W[q], b * P0 * plane);
                a.nslab = M * m1;
                a.nsub = m1;
                a.in_bs = sin_i;
                a.in_bs2 = m2;
                a.out_bs = Z;
                a.out_bs2 = M * Z;
                a.ncols = m2;
                a.in_ld = m1 * m2;
                a.out_ld = plane;
                a.n_in = int(m0);
                a.n_out = int(P0);
                HIPCHK(launch_col(dt, int(P0), kFft, 1, a, s), "explicit x FFT");
            }
        }
        // y FFT in every (b, x') plane over its (i, z) columns (pruned: the m1
        // data rows in, P1 rows out)
        ColArgs c = col_args(tb, dt);
        c.in[0] = c.out[0] = W[q];
        c.nslab = B * P0;
        c.in_bs = c.out_bs = plane;
        c.ncols = M * Z;
        c.in_ld = c.out_ld = M * Z;
        c.n_in = int(pruned ? m1 : P1);
        c.n_out = int(P1);
        HIPCHK(launch_col(dt, int(P1), kFft, 1, c, s), "explicit y FFT");
    }
    // z rows: cyclic convolution of length P2, summed over the M terms, into term 0 of W[0]
    RowArgs ra = row_args(tb, dt);
    ra.f = W[0]; ra.g = W[1]; ra.h = W[0];
    ra.nrows = B * P0 * P1;
    ra.m = Z;
    ra.m_out = pruned ? m2 : P2;
    ra.M = M;
    ra.f_row = ra.g_row = ra.h_row = M * Z;
    ra.f_i = ra.g_i = Z;
    ra.scale = 1.0 / double(P0 * P1 * P2);
    HIPCHK(launch_row_cyclic(dt, int(P2), ra, s), "explicit z rows");
    // inverse y FFT of term 0 in every (b, x') plane, columns z < m2 (the
    // ones the crop keeps); pruned: only the m1 rows the crop keeps
    ColArgs c = col_args(tb, dt);
    c.in[0] = c.out[0] = W[0];
    c.nslab = B * P0;
    c.in_bs = c.out_bs = plane;
    c.ncols = m2;
    c.in_ld = c.out_ld = M * Z;
    c.n_in = int(P1);
    c.n_out = int(pruned ? m1 : P1);
    HIPCHK(launch_col(dt, int(P1), kFft, -1, c, s), "explicit inverse y FFT");
    // inverse x FFT of term 0: per batch entry, slabs y < m1, columns z < m2;
    // pruned: m0 rows straight into h, else in place and cropped after
    for (int64_t b = 0; b < B; ++b) {
        ColArgs a = col_args(tb, dt);
        void* wb = atw(W[0], b * P0 * plane);
        a.in[0] = wb;
        a.out[0] = pruned ? static_cast<void*>(static_cast<char*>(h) + b * m0 * m1 * m2 * int64_t(cs)) : wb;
        a.nslab = m1;
        a.in_bs = M * Z;
        a.out_bs = pruned ? m2 : M * Z;
        a.ncols = m2;
        a.in_ld = plane;
        a.out_ld = pruned ? m1 * m2 : plane;
        a.n_in = int(P0);
        a.n_out = int(m0);
        HIPCHK(launch_col(dt, int(P0), kFft, -1, a, s), "explicit inverse x FFT");
    }
    if (!pruned) {
        // crop: rows (b, x < m0) of m1 x m2 blocks of term 0
        for (int64_t b = 0; b < B; ++b)
            HIPCHK(launch_copy2d(dt, atw(W[0], b * P0 * plane), static_cast<char*>(h) + b * m0 * m1 * m2 * int64_t(cs), m0,
                                 1, plane, 0, M * Z, m1 * m2, 0, m2, m1, m2, m1, m2, s), "explicit crop");
    }
    return IMPCONV_OK;
}

impconv_status runnd(int kind, int dt, int nd, int64_t batch, int64_t M, const int64_t* m,
                     const int64_t* n, const void* f, const void* g, void* h, void* work, size_t wb,
                     uint32_t flags, void* stream)
{
    if (kind == IMPCONV_TERNARY) return fail(IMPCONV_E_ARG, "ternary 2D convolutions use impconv_conv2d_ternary");
    PlanND p;
    impconv_status st = plannd(kind, dt, nd, m, n, batch, M, flags, &p);
    if (st) return st;
    if (batch == 0) return IMPCONV_OK;
    const size_t cs = csize(dt);
    if (!f || !g || !h) return fail(IMPCONV_E_ARG, "null data pointer");
    for (const void* q : {f, g, (const void*)h})
        if (reinterpret_cast<uintptr_t>(q) % cs) return fail(IMPCONV_E_ALIGN, "data pointer misaligned");
    size_t vol = 1;
    for (int d = 0; d < nd; ++d) vol *= size_t(n[d]);
    const size_t nin = batch * M * vol * cs, nout = batch * vol * cs;
    if (bad_alias(h, nout, f, nin) || bad_alias(h, nout, g, nin))
        return fail(IMPCONV_E_ARG, "h overlaps an input (only h == input of the same extent is allowed)");
    if (wb < p.work) return fail(IMPCONV_E_WORKSPACE, "workspace too small: need " + std::to_string(p.work) + " bytes");
    if (!work) return fail(IMPCONV_E_ARG, "work is NULL");
    if (reinterpret_cast<uintptr_t>(work) % cs) return fail(IMPCONV_E_ALIGN, "work misaligned");
    const DevTables* tbp = tables();
    if (!tbp) return IMPCONV_E_HIP;
    const DevTables& tb = *tbp;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool herm = kind == IMPCONV_HERMITIAN;
    const int R = herm ? 3 : 2;
    const bool sym = herm && !(flags & IMPCONV_NO_SYMMETRIZE);
    char* w = static_cast<char*>(work);

    if ((flags & IMPCONV_EXPLICIT_PADDED) && herm)
        return run_herm_explicit(tb, p, f, g, h, w, s, flags & IMPCONV_EXPLICIT_PRUNED);
    if ((flags & IMPCONV_EXPLICIT_PADDED) && nd == 3)
        return run_complex3d_explicit(tb, p, f, g, h, w, s, flags & IMPCONV_EXPLICIT_PRUNED);
    if ((flags & IMPCONV_EXPLICIT_PADDED) && (flags & IMPCONV_EXPLICIT_PRUNED)) {
        // Pruned conventional method: the padded transforms with the zero
        // padding fused into the loads and no transform of an all-zero
        // column -- x FFTs of size 2N0 read the m0 stored rows of each of the
        // m1 data columns straight from f and g, the rows of size 2N1 read
        // their m1 data entries (zero beyond) and keep the m1 cropped outputs,
        // and the inverse x FFT writes the m0 cropped rows straight to h.
        const int64_t P0 = 2 * p.Np[0], P1 = 2 * p.Np[1], m0 = m[0], m1 = m[1];
        const size_t arr = size_t(batch) * M * P0 * m1 * cs;
        void* Fp = w;
        void* Gp = w + arr;
        for (int q = 0; q < 2; ++q) {
            ColArgs a = col_args(tb, dt);
            a.in[0] = q ? g : f;
            a.out[0] = q ? Gp : Fp;
            a.nslab = batch * M;
            a.nsub = M;
            a.in_bs = M * m0 * m1;
            a.in_bs2 = m0 * m1;
            a.in_ld = m1;
            a.out_bs = P0 * M * m1;
            a.out_bs2 = m1;
            a.out_ld = M * m1;
            a.ncols = m1;
            a.n_in = int(m0);
            a.n_out = int(P0);
            HIPCHK(launch_col(dt, int(P0), kFft, 1, a, s), "pruned column FFT");
        }
        RowArgs ra = row_args(tb, dt);
        ra.f = Fp; ra.g = Gp; ra.h = Fp;
        ra.nrows = batch * P0;
        ra.m = m1;
        ra.m_out = m1;
        ra.M = M;
        ra.f_row = ra.g_row = ra.h_row = M * m1;
        ra.f_i = ra.g_i = m1;
        ra.scale = 1.0 / double(P0 * P1);
        HIPCHK(launch_row_cyclic(dt, int(P1), ra, s), "pruned row convolution");
        ColArgs a = col_args(tb, dt);
        a.in[0] = Fp;
        a.out[0] = h;
        a.nslab = batch;
        a.in_bs = P0 * M * m1;
        a.in_ld = M * m1;
        a.out_bs = m0 * m1;
        a.out_ld = m1;
        a.ncols = m1;
        a.n_in = int(P0);
        a.n_out = int(m0);
        HIPCHK(launch_col(dt, int(P0), kFft, -1, a, s), "pruned inverse column FFT");
        return IMPCONV_OK;
    }
    if (flags & IMPCONV_EXPLICIT_PADDED) {
        // Conventional method (Sec. 1): copy the inputs into zero-padded
        // 2N0 x 2N1 arrays, transform both axes at the padded size, multiply,
        // transform back, crop.  Same FFT kernels as the implicit path.
        const int64_t P0 = 2 * p.Np[0], P1 = 2 * p.Np[1], m0 = m[0], m1 = m[1];
        const size_t arr = size_t(batch) * M * P0 * P1 * cs;
        void* Fp = w;
        void* Gp = w + arr;
        const int64_t slab = P0 * M * P1;
        for (int q = 0; q < 2; ++q)
            HIPCHK(launch_copy2d(dt, q ? g : f, q ? Gp : Fp, batch * M, M, M * m0 * m1, m0 * m1, m1, slab, P1,
                                 M * P1, m0, m1, P0, P1, s), "explicit pad");
        for (int q = 0; q < 2; ++q) {
            ColArgs a = col_args(tb, dt);
            a.in[0] = q ? Gp : Fp;
            a.out[0] = q ? Gp : Fp;
            a.nslab = batch * M;
            a.nsub = M;
            a.in_bs = a.out_bs = slab;
            a.in_bs2 = a.out_bs2 = P1;
            a.ncols = P1;
            a.in_ld = a.out_ld = M * P1;
            a.n_in = int(P0);
            a.n_out = int(P0);
            HIPCHK(launch_col(dt, int(P0), kFft, 1, a, s), "explicit column FFT");
        }
        RowArgs ra = row_args(tb, dt);
        ra.f = Fp; ra.g = Gp; ra.h = Fp;
        ra.nrows = batch * P0;
        ra.m = P1;
        ra.m_out = P1;
        ra.M = M;
        ra.f_row = ra.g_row = ra.h_row = M * P1;
        ra.f_i = ra.g_i = P1;
        ra.scale = 1.0 / double(P0 * P1);
        HIPCHK(launch_row_cyclic(dt, int(P1), ra, s), "explicit row convolution");
        ColArgs a = col_args(tb, dt);
        a.in[0] = Fp;
        a.out[0] = Fp;
        a.nslab = batch;
        a.in_bs = a.out_bs = slab;
        a.ncols = P1;
        a.in_ld = a.out_ld = M * P1;
        a.n_in = int(P0);
        a.n_out = int(m0);
        HIPCHK(launch_col(dt, int(P0), kFft, -1, a, s), "explicit inverse column FFT");
        HIPCHK(launch_copy2d(dt, Fp, h, batch, 1, slab, 0, M * P1, m0 * m1, 0, m1, m0, m1, m0, m1, s),
               "explicit crop");
        return IMPCONV_OK;
    }

    // adjoint forms (complex): f reversed along every axis (the first pass of
    // each outer axis and the row loads), g conjugated once (in the x pass),
    // the output reversed along every axis (row stores and the forward
    // passes of the outer axes)
    // compensated twiddle products (complex): bit 8 of every column pass,
    // kComp in the rows
    const uint32_t cb = (flags & IMPCONV_COMPENSATED) ? 8u : 0u;
    const uint32_t fs_f = ((flags & IMPCONV_REV_F) ? 1u : 0u) | cb;
    const uint32_t fs_g = ((flags & IMPCONV_CONJ_G) ? 2u : 0u) | cb;
    const uint32_t fs_o = ((flags & IMPCONV_REV_OUT) ? 1u : 0u) | cb;
    const uint32_t rowfl = ((flags & IMPCONV_REV_F) ? kRevF : 0u) | ((flags & IMPCONV_REV_OUT) ? kRevOut : 0u) |
                           ((flags & IMPCONV_COMPENSATED) ? kComp : 0u);
    // adjoint form (Hermitian): the k_last = 0 hyperplane of f enters as
    // f_k + conj f_{-k} in the first outer pass, and the last outer pass
    // edits that hyperplane of the output; the inner passes are unchanged
    const uint32_t ha = (flags & IMPCONV_HERMITIAN_ADJOINT) ? 4u : 0u;
    if (nd == 2) {
        const int64_t N0 = p.Np[0], n0 = n[0], n1 = n[1], m0 = m[0], m1 = m[1];
        const size_t arr = size_t(batch) * M * N0 * n1 * cs;
        void* Wf[3] = {w, w + arr, w + 2 * arr};
        void* Wg[3] = {w + R * arr, w + (R + 1) * arr, w + (R + 2) * arr};
        if (!herm) { Wf[2] = Wf[1]; Wg[2] = Wg[1]; }
        // Hermitian: columns y < m1 carry data (slot m1 is a zero slot); k_y = 0 is column 0
        const int64_t mask_nz = herm ? n1 : 0;
        if ((st = outer_bwd(tb, p, f, Wf, batch, M * n0 * n1, n0, m0, N0, n1, sym ? 1 : 0, 0, 0, 0,
                            mask_nz, 0, 1, int(m1), s, fs_f | ha))) return st;
        if ((st = outer_bwd(tb, p, g, Wg, batch, M * n0 * n1, n0, m0, N0, n1, sym ? 1 : 0, 0, 0, 0,
                            mask_nz, 0, 1, int(m1), s, fs_g))) return st;
        if ((st = inner_rows_residues(tb, p, Wf, Wg, R, batch * N0, s, rowfl))) return st;
        if ((st = outer_fwd(tb, p, Wf, h, batch, N0 * M * n1, M * n1, n0, m0, N0, n1, s, fs_o | ha,
                            ha ? 1 : 0))) return st;
        return IMPCONV_OK;
    }
    // 3D (Sec. 3.4): x backward pass into the x-residue arrays Xf[rx], Xg[rx]
    // ([b][x'][i][y][z]); then, per x residue and per chunk of (b, x')
    // planes, the y backward pass into the chunk's y-residue arrays
    // ([plane][y'][i][z]), the z rows (M-dot, in place in Yf), and the y
    // forward pass, whose result ([plane][y][z]) overwrites term 0 of the
    // plane in Xf[rx] (every element of the plane has been read by then);
    // last, the x forward pass over term 0 of the three Xf[rx].
    const int64_t N0 = p.Np[0], N1 = p.Np[1];
    const int64_t n0 = n[0], n1 = n[1], n2 = n[2], m0 = m[0], m1 = m[1], m2 = m[2];
    const int64_t plane = M * n1 * n2;                            // elements of one x-residue plane
    const size_t xa = size_t(batch) * N0 * plane * cs;            // one x-residue array
    const int64_t nplanes = batch * N0;
    const int64_t P = p.ychunk;                                   // planes per chunk
    const size_t ya = size_t(P) * M * N1 * n2 * cs;               // one y-residue array of a chunk
    void* Xf[3]; void* Xg[3];
    for (int r = 0; r < 3; ++r) {
        Xf[r] = w + (r < R ? r : R - 1) * xa;
        Xg[r] = w + (R + (r < R ? r : R - 1)) * xa;
    }
    char* yb = w + 2 * R * xa;
    void* Yf[3]; void* Yg[3];    // y-residue set 0
    void* Yf1[3]; void* Yg1[3];  // y-residue set 1
    for (int ry = 0; ry < 3; ++ry) {
        const int rr = ry < R ? ry : R - 1;
        Yf[ry] = yb + size_t(rr) * ya;
        Yg[ry] = yb + size_t(R + rr) * ya;
        Yf1[ry] = yb + size_t(2 * R + rr) * ya;
        Yg1[ry] = yb + size_t(3 * R + rr) * ya;
    }
    // x pass over columns (y, z): valid columns skip the zero slots of y and z
    const int ylo = herm ? int(n1 - (2 * m1 - 1)) : 0;
    const int64_t mask_nz = herm ? n2 : 0;
    if ((st = outer_bwd(tb, p, f, Xf, batch, M * n0 * n1 * n2, n0, m0, N0, n1 * n2, sym ? 2 : 0, n2,
                        int(n1 - m1), int(n1), mask_nz, ylo, int(n1), int(m2), s, fs_f | ha))) return st;
    if ((st = outer_bwd(tb, p, g, Xg, batch, M * n0 * n1 * n2, n0, m0, N0, n1 * n2, sym ? 2 : 0, n2,
                        int(n1 - m1), int(n1), mask_nz, ylo, int(n1), int(m2), s, fs_g))) return st;
    // y backward pass of np planes: slabs (plane, i) of [n1][n2] -> [plane][y'][i][n2]
    // src2/dst2: a second input and its residue arrays, at the same element
    // distance from src/dst for every residue, transformed in the same
    // launch (slabs np M .. 2 np M)
    auto ypass = [&](const void* src, void* const* dst, int64_t np, uint32_t fsf, hipStream_t q,
                     const void* src2 = nullptr, void* const* dst2 = nullptr) -> impconv_status {
        ColArgs c = col_args(tb, dt);
        c.fsflags = fsf;
        c.in[0] = src;
        for (int r = 0; r < 3; ++r) c.out[r] = dst[r];
        c.nslab = np * M;
        if (src2) {
            c.nslab2 = np * M;
            c.nslab = 2 * np * M;
            c.in2_off = (static_cast<const char*>(src2) - static_cast<const char*>(src)) / int64_t(cs);
            c.out2_off = (static_cast<char*>(dst2[0]) - static_cast<char*>(dst[0])) / int64_t(cs);
        }
        c.nsub = M;
        c.in_bs = M * n1 * n2;
        c.in_bs2 = n1 * n2;
        c.out_bs = N1 * M * n2;
        c.out_bs2 = n2;
        c.ncols = n2;
        c.in_ld = n2;
        c.out_ld = M * n2;
        c.n_in = int(n1);
        c.m = int(m1);
        c.off_in = int(n1 - m1);
        if (herm) { c.mask_nz = n2; c.mask_ylo = 0; c.mask_yhi = 1; c.mask_zhi = int(m2); }
        HIPCHK(launch_col(dt, int(N1), herm ? kCenBwd : kPadBwd, 1, c, q), "y backward pass");
        return IMPCONV_OK;
    };
    // rows and y forward pass of np planes from y-residue set Y into the
    // planes' term 0 in Xf[rx] at xf
    auto rows_fwd = [&](void* const* YF, void* const* YG, char* xf, int64_t np, hipStream_t q) -> impconv_status {
        // one launch over the R residues (3D Hermitian 512^2 x 257, M = 3:
        // complex64 10.23 -> 9.95 ms per step; complex128, with the twiddle
        // tables in LDS, 17.14 -> 16.72 ms against one launch per residue)
        const impconv_status st2 = inner_rows_residues(tb, p, YF, YG, R, np * N1, q, rowfl);
        if (st2) return st2;
        // y forward: [plane][y'][i = 0][n2] (R residues) -> term 0 of the plane in Xf[rx]
        ColArgs c = col_args(tb, dt);
        for (int r = 0; r < 3; ++r) c.in[r] = YF[r];
        c.out[0] = xf;
        c.nslab = np;
        c.in_bs = N1 * M * n2;
        c.out_bs = plane;
        c.ncols = n2;
        c.in_ld = M * n2;
        c.out_ld = n2;
        c.n_out = int(n1);
        c.m = int(m1);
        c.off_out = int(n1 - m1);
        c.scale = 1.0 / double((herm ? 3 : 2) * N1);
        c.fsflags = fs_o;
        HIPCHK(launch_col(dt, int(N1), herm ? kCenFwd : kPadFwd, 1, c, q), "y forward pass");
        return IMPCONV_OK;
    };
    // Chunk j runs its y backward passes on the caller's stream s into
    // y-residue set j mod 2, and its rows and y forward pass on the device's
    // first auxiliary stream, so that the rows of chunk j (latency-bound)
    // overlap the y backward pass of chunk j + 1 (bandwidth-bound).  Events:
    // pipe[b] = set b filled (s -> aux), pipe[2 + b] = set b consumed (aux -> s).
    // The two streams touch disjoint memory: chunk j's y forward pass writes
    // term 0 of chunk j's planes, the y pass of chunk j + 1 reads chunk j + 1's.
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail(hipErrorInvalidDevice, "hipGetDevice");
    // IMPCONV_ONE_STREAM: every launch in order on s (no fork, no events)
    const bool one = (p.flags & IMPCONV_ONE_STREAM) != 0;
    DevLanes* L = one ? nullptr : device_lanes(dev);
    if (!one && !L) return IMPCONV_E_HIP;
    std::unique_lock<std::mutex> lanes_lock;
    if (!one) lanes_lock = std::unique_lock<std::mutex>(L->mu);
    hipStream_t q = one ? s : L->aux[0];
    if (!one) {
        hipError_t e = hipEventRecord(L->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(q, L->fork, 0);
        if (e != hipSuccess) return hip_fail(e, "3D fork");
    }
    int64_t j = 0;
    for (int rx = 0; rx < R && !st; ++rx) {
        for (int64_t p0 = 0; p0 < nplanes && !st; p0 += P, ++j) {
            const int64_t np = std::min(P, nplanes - p0);
            const int bset = int(j & 1);
            char* xf = static_cast<char*>(Xf[rx]) + size_t(p0) * plane * cs;
            const char* xg = static_cast<const char*>(Xg[rx]) + size_t(p0) * plane * cs;
            void* const* YF = bset ? Yf1 : Yf;
            void* const* YG = bset ? Yg1 : Yg;
            hipError_t e = hipSuccess;
            if (!one && j >= 2) e = hipStreamWaitEvent(s, L->pipe[2 + bset], 0);
            if (e != hipSuccess) { st = hip_fail(e, "3D pipeline wait"); break; }
            // the passes of f and g in one launch where they share their
            // flags and the residue arrays of g sit at one distance from
            // those of f (3D Hermitian 512^2 x 257, M = 3: twice as many
            // workgroups per launch, a shorter tail; 16.64 -> 16.23 ms)
            const bool pair = fs_f == cb && static_cast<char*>(YG[1]) - static_cast<char*>(YF[1]) ==
                                                        static_cast<char*>(YG[0]) - static_cast<char*>(YF[0]) &&
                              static_cast<char*>(YG[2]) - static_cast<char*>(YF[2]) ==
                                  static_cast<char*>(YG[0]) - static_cast<char*>(YF[0]);
            if (pair) {
                if ((st = ypass(xf, YF, np, fs_f, s, xg, YG))) break;
            } else {
                if ((st = ypass(xf, YF, np, fs_f, s))) break;
                if ((st = ypass(xg, YG, np, cb, s))) break;
            }
            if (!one) {
                e = hipEventRecord(L->pipe[bset], s);
                if (e == hipSuccess) e = hipStreamWaitEvent(q, L->pipe[bset], 0);
                if (e != hipSuccess) { st = hip_fail(e, "3D pipeline event"); break; }
            }
            if ((st = rows_fwd(YF, YG, xf, np, q))) break;
            if (!one && (e = hipEventRecord(L->pipe[2 + bset], q)) != hipSuccess) {
                st = hip_fail(e, "3D pipeline event");
                break;
            }
        }
    }
    // join, also after a failure part way: s waits for everything queued on q
    if (!one) {
        hipError_t e = hipEventRecord(L->join[0], q);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, L->join[0], 0);
        if (e != hipSuccess && !st) st = hip_fail(e, "3D join");
    }
    if (st) return st;
    // x forward: term 0 of Xf[rx], [b][x'][(i = 0) y z] -> h [b][n0][n1 n2]
    PlanND px = p;
    px.M = 1;
    if ((st = outer_fwd(tb, px, Xf, h, batch, N0 * plane, plane, n0, m0, N0, n1 * n2, s, fs_o | ha,
                        ha ? 2 : 0, n2, int(n1 - m1), int(n1)))) return st;
    return IMPCONV_OK;
}

}  // namespace
}  // namespace impconv

using namespace impconv;

extern "C" {

impconv_status impconv_convnd_workspace(int kind, int dtype, int ndim, const int64_t* m,
                                        const int64_t* n, int64_t batch, int64_t M, uint32_t flags,
                                        size_t* bytes)
{
    if (!bytes) return fail(IMPCONV_E_ARG, "bytes is NULL");
    if (ndim != 2 && ndim != 3) return fail(IMPCONV_E_ARG, "ndim must be 2 or 3");
    PlanND p;
    impconv_status st = plannd(kind, dtype, ndim, m, n, batch, M, flags, &p);
    if (st) return st;
    *bytes = p.work;
    return IMPCONV_OK;
}

impconv_status impconv_conv2d(int kind, int dtype, int64_t batch, int64_t M, const int64_t* m,
                              const int64_t* n, const void* f, const void* g, void* h, void* work,
                              size_t work_bytes, uint32_t flags, void* stream)
{
    return runnd(kind, dtype, 2, batch, M, m, n, f, g, h, work, work_bytes, flags, stream);
}

impconv_status impconv_conv3d(int kind, int dtype, int64_t batch, int64_t M, const int64_t* m,
                              const int64_t* n, const void* f, const void* g, void* h, void* work,
                              size_t work_bytes, uint32_t flags, void* stream)
{
    return runnd(kind, dtype, 3, batch, M, m, n, f, g, h, work, work_bytes, flags, stream);
}

impconv_status impconv_conv2d_ternary(int dtype, int64_t batch, const int64_t* m, const int64_t* n,
                                      const void* f, const void* g, const void* e, void* h, void* work,
                                      size_t work_bytes, uint32_t flags, void* stream)
{
    return run2d_ternary(dtype, batch, m, n, f, g, e, h, work, work_bytes, flags, stream);
}

}  // extern "C"
