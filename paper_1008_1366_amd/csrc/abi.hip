// abi.cpp -- the extern "C" entry points of libimpconv: argument checks on
// the host, workspace sizing, and the launch sequence of each convolution.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "launch.hpp"
#include "multid.hpp"
#include "runtime.hpp"

namespace impconv {

namespace {
thread_local std::string g_err;
}

impconv_status fail(impconv_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

impconv_status hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return IMPCONV_E_HIP;
}

namespace {

size_t csize(int dt) { return dt ? 16 : 8; }

bool aligned(const void* p, int dt) { return (reinterpret_cast<uintptr_t>(p) % csize(dt)) == 0; }

impconv_status check_dtype(int dt)
{
    if (dt != IMPCONV_C64 && dt != IMPCONV_C128) return fail(IMPCONV_E_ARG, "dtype must be IMPCONV_C64 or IMPCONV_C128");
    return IMPCONV_OK;
}

impconv_status check_ptrs(int dt, std::initializer_list<const void*> ps)
{
    for (const void* p : ps) {
        if (!p) return fail(IMPCONV_E_ARG, "null data pointer");
        if (!aligned(p, dt)) return fail(IMPCONV_E_ALIGN, "data pointer not aligned to its complex element size");
    }
    return IMPCONV_OK;
}

hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

// ------------------------------------------------------------------ 1D plans
struct Plan1D {
    int kind, dt;
    int64_t batch, M, m;
    uint32_t flags;
    int64_t N;        // FFT size of the fused kernel (complex: N >= m; Hermitian: NC; ternary: NN)
    bool explicit_;   // comparator path
    int64_t Ne;       // explicit: padded transform size
    size_t work;      // bytes
    int64_t np;       // complex, general p/q rule: block size (0: the 1/2 rule at size N)
    int pq_p, pq_q;   // blocks and residues of the p/q rule
};

// ---------------------------------------------------- general p/q padding
// Sec. 2.4 with the inputs zero-extended to P blocks of NP (P NP >= m) and
// q = ceil((2m - 1) / NP) residues, so that q NP >= 2m - 1 and the cyclic
// convolution of length q NP has no wrap-around onto k < m.
bool pq_rule(int dt, int64_t m, int64_t np, int64_t* P, int64_t* q)
{
    if (np < 1 || (np & (np - 1)) || np > (dt ? kPqMax / 2 : kPqMax)) return false;
    *P = (m + np - 1) / np;
    *q = (2 * m - 1 + np - 1) / np;
    return *P >= 2 && *P <= kPqMaxP;
}

// Relative cost per row, calibrated on MI355X: transform volume times
// (log2 size + per-element work).  The p/q kernel re-reads its P blocks for
// every residue and keeps P output blocks live (half the elements per
// thread of the 1/2-rule kernel), which costs it ~1.5x (P = 2) / ~1.75x
// (P = 3) per unit of volume; the 1/2 rule pays ~1.5x where it needs the
// multi-pass path (N > kRowMax) or, in complex128, the register-bound
// N = kRowMax kernel.
double cost_half_rule(int dt, int64_t m)
{
    const int64_t N = next_pow2(m);
    const double c = 2.0 * double(N) * (std::log2(double(N)) + 2.0);
    return (N > kRowMax || (dt && N == kRowMax)) ? 1.5 * c : c;
}
double cost_pq_rule(int64_t np, int64_t P, int64_t q)
{
    return double(q) * double(np) * (std::log2(double(np)) + 2.0 + double(P)) * (1.0 + 0.25 * double(P));
}

// Block size of the cheapest p/q rule for m, or 0 if the 1/2 rule at the
// power-of-two size is cheaper.
int64_t pq_auto(int dt, int64_t m)
{
    int64_t best = 0;
    double bc = cost_half_rule(dt, m);
    for (int64_t np = 1; np <= kPqMax; np *= 2) {
        int64_t P, q;
        if (!pq_rule(dt, m, np, &P, &q)) continue;
        const double c = cost_pq_rule(np, P, q);
        if (c < bc) { bc = c; best = np; }
    }
    return best;
}

// np_req (complex only): -1 automatic, 0 the 1/2 rule at N = 2^ceil(log2 m),
// > 0 the p/q rule with that block size (np >= m: the 1/2 rule at size np).
impconv_status plan1d(int kind, int dt, int64_t batch, int64_t M, int64_t m, uint32_t flags, Plan1D* p,
                      int64_t np_req = -1)
{
    impconv_status st = check_dtype(dt);
    if (st) return st;
    if (m < 1) return fail(IMPCONV_E_SIZE, "m must be >= 1");
    if (batch < 0) return fail(IMPCONV_E_SIZE, "batch must be >= 0");
    if (M < 1) return fail(IMPCONV_E_SIZE, "M must be >= 1");
    const uint32_t known = IMPCONV_EXPLICIT_PADDED | IMPCONV_EXPLICIT_PRUNED | IMPCONV_REV_F | IMPCONV_CONJ_G |
                           IMPCONV_REV_OUT | IMPCONV_HERMITIAN_ADJOINT | IMPCONV_COMPENSATED;
    if (flags & ~known) return fail(IMPCONV_E_ARG, "unknown flag bits for a 1D convolution");
    if ((flags & IMPCONV_EXPLICIT_PRUNED) && (kind != IMPCONV_COMPLEX || !(flags & IMPCONV_EXPLICIT_PADDED)))
        return fail(IMPCONV_E_ARG, "EXPLICIT_PRUNED qualifies EXPLICIT_PADDED (complex 1D)");
    if ((flags & IMPCONV_COMPENSATED) && (kind != IMPCONV_COMPLEX || (flags & IMPCONV_EXPLICIT_PADDED)))
        return fail(IMPCONV_E_ARG, "COMPENSATED applies to the implicit complex convolution");
    const bool adj = flags & (IMPCONV_REV_F | IMPCONV_CONJ_G | IMPCONV_REV_OUT | IMPCONV_HERMITIAN_ADJOINT);
    if ((flags & (IMPCONV_REV_F | IMPCONV_CONJ_G | IMPCONV_REV_OUT)) && kind != IMPCONV_COMPLEX)
        return fail(IMPCONV_E_ARG, "REV/CONJ flags apply to complex convolutions only");
    if ((flags & IMPCONV_HERMITIAN_ADJOINT) && kind != IMPCONV_HERMITIAN)
        return fail(IMPCONV_E_ARG, "HERMITIAN_ADJOINT applies to Hermitian convolutions only");
    *p = Plan1D{kind, dt, batch, M, m, flags, 0, bool(flags & IMPCONV_EXPLICIT_PADDED), 0, 0, 0, 0, 0};
    if (p->explicit_ && adj) return fail(IMPCONV_E_ARG, "REV/CONJ flags are not accepted with EXPLICIT_PADDED");
    const size_t cs = csize(dt);
    if (kind == IMPCONV_COMPLEX) {
        p->N = next_pow2(m);
        if (!p->explicit_) {
            if (flags & IMPCONV_COMPENSATED) {
                // compensated products: the 1/2-rule row kernel only
                if (np_req > 0 && np_req != p->N) return fail(IMPCONV_E_ARG, "COMPENSATED takes the 1/2 rule");
                if (p->N > kRowMax) return fail(IMPCONV_E_UNSUPPORTED, "COMPENSATED supports m <= 8192");
                return IMPCONV_OK;
            }
            if (np_req < 0) np_req = pq_auto(dt, m);
            if (np_req > 0) {
                if (np_req >= m && np_req <= kRowMax && (np_req & (np_req - 1)) == 0) {
                    p->N = np_req;  // P = 1: the 1/2 rule at size np
                    return IMPCONV_OK;
                }
                if (np_req == p->N) np_req = 0;  // the 1/2 rule at N, multi-pass above kRowMax
            }
            if (np_req > 0) {
                int64_t P, q;
                if (!pq_rule(dt, m, np_req, &P, &q))
                    return fail(IMPCONV_E_SIZE, "p/q rule: np must be a power of two <= " +
                                                    std::to_string(dt ? kPqMax / 2 : kPqMax) +
                                                    " with ceil(m / np) <= " + std::to_string(kPqMaxP));
                p->np = np_req;
                p->pq_p = int(P);
                p->pq_q = int(q);
                return IMPCONV_OK;
            }
            if (p->N > kRowMax) return large1d_plan(p->dt, batch, M, m, &p->work) ;
        } else {
            p->Ne = 2 * p->N;
            if (p->Ne > kRowMax) return fail(IMPCONV_E_UNSUPPORTED, "explicit complex comparator supports m <= 4096");
            // pruned form: the zero padding is read, not stored; no workspace
            p->work = (flags & IMPCONV_EXPLICIT_PRUNED) ? 0 : size_t(batch) * (2 * M + 1) * p->Ne * cs;
        }
    } else if (kind == IMPCONV_HERMITIAN) {
        int64_t N = next_pow2(m);
        if (N < 2) N = 2;
        p->N = N / 2;
        if (!p->explicit_) {
            if (p->N > kRowMax) return fail(IMPCONV_E_UNSUPPORTED, "Hermitian convolution supports m <= 16384");
        } else {
            // conventional 2/3 rule: real transform length 2^ceil(log2(3m-2)), half spectrum + 1
            int64_t Ne = next_pow2(std::max<int64_t>(3 * m - 2, 2));
            p->Ne = Ne;
            if (Ne / 2 > kRowMax) return fail(IMPCONV_E_UNSUPPORTED, "explicit Hermitian comparator supports m <= 5462");
            p->work = size_t(batch) * (2 * M + 1) * (Ne / 2 + 1) * cs;
        }
    } else if (kind == IMPCONV_TERNARY) {
        p->N = next_pow2(m);
        if (!p->explicit_) {
            if (p->N > kRowMax) return fail(IMPCONV_E_UNSUPPORTED, "ternary convolution supports m <= 8192");
        } else {
            // conventional: real transform length 2^ceil(log2(4m-3)) (no wave beating of
            // three factors), half spectrum + 1 per padded row of f, g, e and h
            const int64_t Ne = next_pow2(std::max<int64_t>(4 * m - 3, 2));
            p->Ne = Ne;
            if (Ne / 2 > kRowMax) return fail(IMPCONV_E_UNSUPPORTED, "explicit ternary comparator supports m <= 4096");
            p->work = size_t(batch) * 4 * (Ne / 2 + 1) * cs;
        }
    } else {
        return fail(IMPCONV_E_ARG, "unknown kind");
    }
    return IMPCONV_OK;
}

RowArgs row_args(const DevTables* tb, int dt)
{
    RowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tw = tb->tw[dt];
    a.tw3 = tb->tw3[dt];
    a.twlo = tb->twlo;
    return a;
}

}  // namespace

// Device-side preparation of a 1D convolution that its execution would
// otherwise do on first use: the column twiddle table of the three-pass form
// (complex lengths whose power-of-two size exceeds kRowMax, 1/2 rule).
impconv_status conv1d_prepare(int kind, int dt, int64_t batch, int64_t M, int64_t m, uint32_t flags)
{
    if (kind != IMPCONV_COMPLEX) return IMPCONV_OK;
    Plan1D p;
    impconv_status st = plan1d(kind, dt, batch, M, m, flags, &p);
    if (st) return st;
    if (p.explicit_ || p.np != 0 || p.N <= kRowMax) return IMPCONV_OK;
    int64_t N1, N2;
    fourstep_split(p.N, &N1, &N2);
    return fs_twiddles(dt, N2, N1) ? IMPCONV_OK : IMPCONV_E_HIP;
}

}  // namespace impconv

using namespace impconv;

extern "C" {

int impconv_version(void) { return 10000; }

const char* impconv_status_string(int s)
{
    switch (s) {
        case IMPCONV_OK: return "ok";
        case IMPCONV_E_ARG: return "invalid argument";
        case IMPCONV_E_SIZE: return "invalid size";
        case IMPCONV_E_WORKSPACE: return "workspace too small";
        case IMPCONV_E_ALIGN: return "misaligned pointer";
        case IMPCONV_E_UNSUPPORTED: return "unsupported size or mode";
        case IMPCONV_E_HIP: return "HIP error";
        default: return "unknown status";
    }
}

const char* impconv_last_error(void) { return g_err.c_str(); }

impconv_status impconv_init(void)
{
    if (!tables()) return IMPCONV_E_HIP;
    return noalloc_setup();
}

impconv_status impconv_conv1d_workspace(int kind, int dtype, int64_t batch, int64_t M, int64_t m,
                                        uint32_t flags, size_t* bytes)
{
    if (!bytes) return fail(IMPCONV_E_ARG, "bytes is NULL");
    Plan1D p;
    impconv_status st = plan1d(kind, dtype, batch, M, m, flags, &p);
    if (st) return st;
    *bytes = p.work;
    return IMPCONV_OK;
}

static impconv_status run1d(int kind, int dtype, int64_t batch, int64_t M, int64_t m, const void* f,
                            const void* g, const void* e, void* h, void* work, size_t wb,
                            uint32_t flags, void* stream, int64_t np_req = -1)
{
    Plan1D p;
    impconv_status st = plan1d(kind, dtype, batch, M, m, flags, &p, np_req);
    if (st) return st;
    if (batch == 0) return IMPCONV_OK;
    const int dt = dtype;
    st = kind == IMPCONV_TERNARY ? check_ptrs(dt, {f, g, e, h}) : check_ptrs(dt, {f, g, h});
    if (st) return st;
    const size_t cs = csize(dt);
    const size_t nin = size_t(batch) * (kind == IMPCONV_TERNARY ? 1 : M) * m * cs, nout = size_t(batch) * m * cs;
    if (bad_alias(h, nout, f, nin) || bad_alias(h, nout, g, nin) || (e && bad_alias(h, nout, e, nin)))
        return fail(IMPCONV_E_ARG, "h overlaps an input (only h == input of the same extent is allowed)");
    if (wb < p.work) return fail(IMPCONV_E_WORKSPACE, "workspace too small: need " + std::to_string(p.work) + " bytes");
    if (p.work && !work) return fail(IMPCONV_E_ARG, "work is NULL");
    if (p.work && !aligned(work, dt)) return fail(IMPCONV_E_ALIGN, "work not aligned");
    const DevTables* tb = tables();
    if (!tb) return IMPCONV_E_HIP;
    hipStream_t s = S(stream);
    hipError_t err = hipSuccess;

    if (kind == IMPCONV_COMPLEX && !p.explicit_ && p.np == 0 && p.N > kRowMax)
        return large1d_run(*tb, dt, batch, M, m, f, g, h, work, flags, s);

    RowArgs a = row_args(tb, dt);
    a.nrows = batch;
    a.m = m;
    a.M = M;
    a.flags = flags & (kRevF | kConjG | kRevOut | kHermAdj | kComp);
    if (!p.explicit_) {
        a.f = f; a.g = g; a.e = e; a.h = h;
        if (kind == IMPCONV_TERNARY) {
            a.f_row = a.g_row = a.e_row = a.h_row = m;
            err = launch_row_ternary(dt, int(p.N), a, s);
        } else {
            a.f_row = a.g_row = M * m;
            a.f_i = a.g_i = m;
            a.h_row = m;
            if (kind == IMPCONV_COMPLEX && p.np > 0) {
                const int64_t Nq = p.pq_q * p.np;
                a.q = p.pq_q;
                a.twq = (Nq & (Nq - 1)) == 0 ? static_cast<const void*>(static_cast<const char*>(tb->tw[dt]) + tw_off(Nq) * cs)
                                             : static_cast<const void*>(static_cast<const char*>(tb->twq[dt]) + twq_off(p.pq_q, p.np) * cs);
                err = launch_row_pq(dt, int(p.np), p.pq_p, a, s);
            } else {
                err = kind == IMPCONV_COMPLEX ? launch_row_complex(dt, int(p.N), a, s)
                                              : launch_row_hermitian(dt, int(p.N), a, s);
            }
        }
        if (err != hipSuccess) return hip_fail(err, "row kernel launch");
        return IMPCONV_OK;
    }
    if (kind == IMPCONV_COMPLEX && (flags & IMPCONV_EXPLICIT_PRUNED)) {
        // Explicit comparator with the padding fused into the loads: one
        // size-2N cyclic convolution per row reads f and g (zero beyond m)
        // and writes the first m outputs.
        a.f = f; a.g = g; a.h = h;
        a.f_row = a.g_row = M * m;
        a.f_i = a.g_i = m;
        a.h_row = m;
        a.m_out = m;
        a.scale = 1.0 / double(p.Ne);
        err = launch_row_cyclic(dt, int(p.Ne), a, s);
        if (err != hipSuccess) return hip_fail(err, "explicit pruned launch");
        return IMPCONV_OK;
    }
    // Explicit comparator: materialize zero-padded copies in the workspace,
    // transform at the padded size, multiply, transform back, crop.
    const int64_t L = kind == IMPCONV_COMPLEX ? p.Ne : p.Ne / 2 + 1;  // padded row length
    char* w = static_cast<char*>(work);
    void* fp = w;
    void* gp = w + size_t(batch) * M * L * cs;
    void* hp = w + size_t(batch) * 2 * M * L * cs;
    void* ep = w + size_t(batch) * 3 * M * L * cs;  // ternary (M = 1)
    if ((err = launch_pad_rows(dt, f, fp, batch * M, m, m, L, s)) != hipSuccess) return hip_fail(err, "pad");
    if ((err = launch_pad_rows(dt, g, gp, batch * M, m, m, L, s)) != hipSuccess) return hip_fail(err, "pad");
    if (kind == IMPCONV_TERNARY && (err = launch_pad_rows(dt, e, ep, batch, m, m, L, s)) != hipSuccess)
        return hip_fail(err, "pad");
    a.f = fp; a.g = gp; a.h = hp;
    if (kind == IMPCONV_TERNARY) {
        a.e = ep;
        a.e_row = L;
    }
    a.f_row = a.g_row = M * L;
    a.f_i = a.g_i = L;
    a.h_row = L;
    if (kind == IMPCONV_COMPLEX) {
        a.m = L;
        a.m_out = L;
        a.scale = 1.0 / double(p.Ne);
        err = launch_row_cyclic(dt, int(p.Ne), a, s);
    } else {
        a.m = L;
        a.m_out = L;
        a.scale = 1.0 / double(p.Ne);
        err = launch_row_realcyclic(dt, int(p.Ne / 2), a, s);
    }
    if (err != hipSuccess) return hip_fail(err, "explicit transform");
    if ((err = launch_pad_rows(dt, hp, h, batch, L, m, m, s)) != hipSuccess) return hip_fail(err, "crop");
    return IMPCONV_OK;
}

impconv_status impconv_conv1d_complex(int dtype, int64_t batch, int64_t M, int64_t m, const void* f,
                                      const void* g, void* h, void* work, size_t work_bytes,
                                      uint32_t flags, void* stream)
{
    return run1d(IMPCONV_COMPLEX, dtype, batch, M, m, f, g, nullptr, h, work, work_bytes, flags, stream);
}

impconv_status impconv_conv1d_complex_pq(int dtype, int64_t batch, int64_t M, int64_t m, int64_t np,
                                         const void* f, const void* g, void* h, void* work,
                                         size_t work_bytes, uint32_t flags, void* stream)
{
    if (np < 0) return fail(IMPCONV_E_SIZE, "np must be >= 0");
    if (flags & IMPCONV_EXPLICIT_PADDED) return fail(IMPCONV_E_ARG, "the p/q rule is an implicit method");
    return run1d(IMPCONV_COMPLEX, dtype, batch, M, m, f, g, nullptr, h, work, work_bytes, flags, stream,
                 np == 0 ? -1 : np);
}

impconv_status impconv_conv1d_complex_pq_workspace(int dtype, int64_t batch, int64_t M, int64_t m, int64_t np,
                                                   size_t* bytes)
{
    if (!bytes) return fail(IMPCONV_E_ARG, "bytes is NULL");
    if (np < 0) return fail(IMPCONV_E_SIZE, "np must be >= 0");
    Plan1D p;
    impconv_status st = plan1d(IMPCONV_COMPLEX, dtype, batch, M, m, 0, &p, np == 0 ? -1 : np);
    if (st) return st;
    *bytes = p.work;
    return IMPCONV_OK;
}

impconv_status impconv_conv1d_complex_rule(int dtype, int64_t m, int64_t* np, int* p, int* q)
{
    if (!np || !p || !q) return fail(IMPCONV_E_ARG, "null output pointer");
    Plan1D pl;
    impconv_status st = plan1d(IMPCONV_COMPLEX, dtype, 1, 1, m, 0, &pl);
    if (st) return st;
    *np = pl.np;
    *p = pl.np ? pl.pq_p : 1;
    *q = pl.np ? pl.pq_q : 2;
    return IMPCONV_OK;
}

impconv_status impconv_conv1d_hermitian(int dtype, int64_t batch, int64_t M, int64_t m, const void* f,
                                        const void* g, void* h, void* work, size_t work_bytes,
                                        uint32_t flags, void* stream)
{
    return run1d(IMPCONV_HERMITIAN, dtype, batch, M, m, f, g, nullptr, h, work, work_bytes, flags, stream);
}

impconv_status impconv_conv1d_ternary(int dtype, int64_t batch, int64_t m, const void* f, const void* g,
                                      const void* e, void* h, void* work, size_t work_bytes,
                                      uint32_t flags, void* stream)
{
    return run1d(IMPCONV_TERNARY, dtype, batch, 1, m, f, g, e, h, work, work_bytes, flags, stream);
}

}  // extern "C"
