/*
 * impconv_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct FP64 direct summations of the convolution
 * sums that the implicitly dealiased method (Bowman & Roberts, "Efficient
 * dealiased convolutions without padding") reaches exactly, up to rounding
 * order.  No FFT, no blocking, no fusion: every function is the definition
 * written out as nested loops, so a reader can check it against the paper by
 * eye.  Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg
 * may load this library; the product path never does.
 *
 * Complex numbers are C99 `double complex`, i.e. interleaved (re, im) FP64,
 * which is also the memory layout of numpy complex128.
 *
 * Citations name the paper's sections and equations:
 *   Sec. 1        -- dealiased linear convolution as an explicitly padded cyclic one
 *   Sec. 2.1      -- complex 1D sum  h_k = sum_{p=0..k} f_p g_{k-p}, k < m
 *   Sec. 2.2      -- centered data of length 2m-1, origin at index m-1
 *   Sec. 2.3      -- centered Hermitian sum over p = k-m+1 .. m-1, with U_{-k} = conj U_k
 *   Sec. 3.1/3.3  -- 2D and 3D complex convolutions (componentwise origin at 0)
 *   Sec. 3.2/3.4  -- 2D and 3D centered Hermitian convolutions
 *   Sec. 3.3      -- M-vector inputs: f*g read as sum_i f_i*g_i
 *   Sec. 4        -- centered ternary sum over p+q+r = k (1D tconv; nD over the
 *                    box, the 2D case being tconv2)
 *   Concluding remarks -- the Hermitian symmetry of the k_last = 0 line/plane
 *                    is enforced by the convolution routine itself.
 *
 * Where the paper is silent the readings are:
 *   - Im f_0 of a Hermitian input is ignored (a real-valued field has a real
 *     mean); more generally the k_last = 0 hyperplane is replaced by its
 *     Hermitian projection when symmetrization is off, and by the conjugate
 *     mirror of its authoritative half when it is on.
 *   - Authoritative half of the k_last = 0 hyperplane: the first nonzero
 *     leading wavenumber is positive (2D: k_x > 0; 3D: k_x > 0, or k_x = 0 and
 *     k_y > 0).
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex dc;

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------------------
 * Complex 1D (Sec. 2.1): h_k = sum_{i<M} sum_{p=0}^{k} f_{i,p} g_{i,k-p},
 * k = 0..m-1.  Layout f[b][i][p], g[b][i][p], h[b][k].
 * ------------------------------------------------------------------------- */
void orc_conv1d_complex(int64_t m, int64_t M, int64_t batch,
                        const dc *f, const dc *g, dc *h)
{
    #pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t b = 0; b < batch; ++b)
        for (int64_t k = 0; k < m; ++k) {
            dc s = 0;
            for (int64_t i = 0; i < M; ++i) {
                const dc *fi = f + (b * M + i) * m;
                const dc *gi = g + (b * M + i) * m;
                for (int64_t p = 0; p <= k; ++p) s += fi[p] * gi[k - p];
            }
            h[b * m + k] = s;
        }
}

/* Ragged batch of complex 1D pairs: pair j has length ms[j] and starts at
 * element offs[j] of the packed f, g and h arrays. */
void orc_conv1d_complex_ragged(int64_t npairs, const int64_t *ms, const int64_t *offs,
                               const dc *f, const dc *g, dc *h)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < npairs; ++j) {
        const int64_t m = ms[j];
        const dc *fj = f + offs[j], *gj = g + offs[j];
        dc *hj = h + offs[j];
        for (int64_t k = 0; k < m; ++k) {
            dc s = 0;
            for (int64_t p = 0; p <= k; ++p) s += fj[p] * gj[k - p];
            hj[k] = s;
        }
    }
}

/* Adjoint of the complex 1D sum with respect to each input (not in the paper;
 * derived from the definition above).  With gh = dL/dRe h + i dL/dIm h:
 *   grad_f[p] = sum_{k=p}^{m-1} gh_k conj(g_{k-p})
 *   grad_g[q] = sum_{k=q}^{m-1} gh_k conj(f_{k-q})                          */
void orc_grad_conv1d_complex(int64_t m, const dc *f, const dc *g, const dc *gh,
                             dc *grad_f, dc *grad_g)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < m; ++p) {
        dc sf = 0, sg = 0;
        for (int64_t k = p; k < m; ++k) {
            sf += gh[k] * conj(g[k - p]);
            sg += gh[k] * conj(f[k - p]);
        }
        grad_f[p] = sf;
        grad_g[p] = sg;
    }
}

/* ---------------------------------------------------------------------------
 * Centered 1D (Sec. 2.2): inputs of length 2m-1 with the Fourier origin at
 * index m-1; h_k = sum_p f_p g_{k-p} over |p| <= m-1, |k-p| <= m-1, for
 * |k| <= m-1.  This is the operation the centered outer-axis passes of the
 * multidimensional convolutions perform along one axis.
 * ------------------------------------------------------------------------- */
void orc_conv1d_centered(int64_t m, const dc *f, const dc *g, dc *h)
{
    const int64_t o = m - 1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = -(m - 1); k <= m - 1; ++k) {
        dc s = 0;
        for (int64_t p = -(m - 1); p <= m - 1; ++p) {
            const int64_t q = k - p;
            if (q < -(m - 1) || q > m - 1) continue;
            s += f[p + o] * g[q + o];
        }
        h[k + o] = s;
    }
}

/* Value of the full Hermitian-extended 1D sequence at wavenumber p, from the
 * stored non-negative half u[0..m-1] (Sec. 2.3: U_{-k} = conj U_k; Im U_0 is
 * dropped). */
static dc herm1(const dc *u, int64_t p)
{
    if (p == 0) return creal(u[0]);
    if (p > 0) return u[p];
    return conj(u[-p]);
}

/* ---------------------------------------------------------------------------
 * Centered Hermitian 1D (Sec. 2.3):
 *   h_k = sum_{i<M} sum_{p=k-m+1}^{m-1} F_i(p) G_i(k-p),  k = 0..m-1,
 * with F, G the Hermitian extensions of the stored halves.
 * ------------------------------------------------------------------------- */
void orc_conv1d_hermitian(int64_t m, int64_t M, int64_t batch,
                          const dc *f, const dc *g, dc *h)
{
    #pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t b = 0; b < batch; ++b)
        for (int64_t k = 0; k < m; ++k) {
            dc s = 0;
            for (int64_t i = 0; i < M; ++i) {
                const dc *fi = f + (b * M + i) * m;
                const dc *gi = g + (b * M + i) * m;
                for (int64_t p = k - m + 1; p <= m - 1; ++p)
                    s += herm1(fi, p) * herm1(gi, k - p);
            }
            h[b * m + k] = s;
        }
}

/* ---------------------------------------------------------------------------
 * Centered Hermitian ternary 1D (Sec. 4):
 *   h_k = sum_{p,q,r in [-m+1, m-1], p+q+r = k} F(p) G(q) E(r),  k = 0..m-1.
 * Direct O(m^3).
 * ------------------------------------------------------------------------- */
void orc_conv1d_ternary(int64_t m, int64_t batch, const dc *f, const dc *g,
                        const dc *e, dc *h)
{
    #pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int64_t b = 0; b < batch; ++b)
        for (int64_t k = 0; k < m; ++k) {
            const dc *fb = f + b * m, *gb = g + b * m, *eb = e + b * m;
            dc s = 0;
            for (int64_t p = -(m - 1); p <= m - 1; ++p) {
                const dc fp = herm1(fb, p);
                for (int64_t q = -(m - 1); q <= m - 1; ++q) {
                    const int64_t r = k - p - q;
                    if (r < -(m - 1) || r > m - 1) continue;
                    s += fp * herm1(gb, q) * herm1(eb, r);
                }
            }
            h[b * m + k] = s;
        }
}

/* Same ternary sum evaluated only at the output indices ks[0..npts-1]. */
void orc_conv1d_ternary_at(int64_t m, const dc *f, const dc *g, const dc *e, int64_t npts,
                           const int64_t *ks, dc *out)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < npts; ++j) {
        const int64_t k = ks[j];
        dc s = 0;
        for (int64_t p = -(m - 1); p <= m - 1; ++p) {
            const dc fp = herm1(f, p);
            for (int64_t q = -(m - 1); q <= m - 1; ++q) {
                const int64_t r = k - p - q;
                if (r < -(m - 1) || r > m - 1) continue;
                s += fp * herm1(g, q) * herm1(e, r);
            }
        }
        out[j] = s;
    }
}

/* ---------------------------------------------------------------------------
 * Multidimensional helpers.  Arrays are C-ordered, last axis contiguous
 * (Sec. 3.1: y is the stride-one direction).  ndim is 1, 2 or 3.
 * ------------------------------------------------------------------------- */
static void unflatten(int ndim, const int64_t *ext, int64_t lin, int64_t *idx)
{
    for (int d = ndim - 1; d >= 0; --d) { idx[d] = lin % ext[d]; lin /= ext[d]; }
}

/* Complex nD (Secs. 3.1 and 3.3): h_k = sum_i sum_{0 <= p <= k componentwise}
 * f_{i,p} g_{i,k-p}, 0 <= k_d < m_d.  Layout f[i][x][y][z], h[x][y][z]. */
static dc cnd_point(int ndim, const int64_t *m, int64_t M, const dc *f, const dc *g,
                    const int64_t *k)
{
    /* unused trailing axes get k = 0 and stride 0, so one triple loop serves 1D..3D */
    int64_t vol = 1, st[3] = {0, 0, 0}, kk[3] = {0, 0, 0};
    for (int d = 0; d < ndim; ++d) vol *= m[d];
    int64_t s = 1;
    for (int d = ndim - 1; d >= 0; --d) { st[d] = s; s *= m[d]; kk[d] = k[d]; }
    dc acc = 0;
    for (int64_t i = 0; i < M; ++i) {
        const dc *fi = f + i * vol, *gi = g + i * vol;
        for (int64_t p0 = 0; p0 <= kk[0]; ++p0)
            for (int64_t p1 = 0; p1 <= kk[1]; ++p1)
                for (int64_t p2 = 0; p2 <= kk[2]; ++p2) {
                    const int64_t a = p0 * st[0] + p1 * st[1] + p2 * st[2];
                    const int64_t c = (kk[0] - p0) * st[0] + (kk[1] - p1) * st[1]
                                    + (kk[2] - p2) * st[2];
                    acc += fi[a] * gi[c];
                }
    }
    return acc;
}

void orc_convnd_complex(int ndim, const int64_t *m, int64_t M, const dc *f, const dc *g, dc *h)
{
    int64_t vol = 1;
    for (int d = 0; d < ndim; ++d) vol *= m[d];
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t lin = 0; lin < vol; ++lin) {
        int64_t k[3];
        unflatten(ndim, m, lin, k);
        h[lin] = cnd_point(ndim, m, M, f, g, k);
    }
}

/* Same sum evaluated only at npts output points pts[j][0..ndim-1]. */
void orc_convnd_complex_at(int ndim, const int64_t *m, int64_t M, const dc *f, const dc *g,
                           int64_t npts, const int64_t *pts, dc *out)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < npts; ++j) out[j] = cnd_point(ndim, m, M, f, g, pts + j * ndim);
}

/* ---------------------------------------------------------------------------
 * Centered Hermitian nD (Secs. 3.2 and 3.4).  Logical box
 * B = prod_d [-m_d+1, m_d-1]; the stored half is k_last >= 0.
 * Storage: leading (centered) axes have n_d in {2m_d-1, 2m_d} and wavenumber
 * k at index k + (n_d - m_d) (for n_d = 2m_d, index 0 is a zero slot); the
 * last axis has n in {m, m+1} and wavenumber k at index k (index m, if
 * present, is a zero slot).
 * ------------------------------------------------------------------------- */
typedef struct {
    int ndim;
    int64_t m[3], n[3], off[3], st[3], vol;
    int sym;
} hlay;

static void hlay_init(hlay *L, int ndim, const int64_t *m, const int64_t *n, int sym)
{
    L->ndim = ndim;
    L->sym = sym;
    for (int d = 0; d < 3; ++d) { L->m[d] = 1; L->n[d] = 1; L->off[d] = 0; }
    for (int d = 0; d < ndim; ++d) {
        L->m[d] = m[d];
        L->n[d] = n[d];
        L->off[d] = (d < ndim - 1) ? n[d] - m[d] : 0;
    }
    L->st[ndim - 1] = 1;
    for (int d = ndim - 2; d >= 0; --d) L->st[d] = L->st[d + 1] * L->n[d + 1];
    L->vol = 1;
    for (int d = 0; d < ndim; ++d) L->vol *= L->n[d];
}

static int in_box(const hlay *L, const int64_t *p)
{
    for (int d = 0; d < L->ndim; ++d)
        if (p[d] < -(L->m[d] - 1) || p[d] > L->m[d] - 1) return 0;
    return 1;
}

static int64_t hidx(const hlay *L, const int64_t *p)
{
    int64_t a = 0;
    for (int d = 0; d < L->ndim; ++d) a += (p[d] + L->off[d]) * L->st[d];
    return a;
}

/* Full-array value at p (p in B) of the field whose stored half is u. */
static dc hval(const hlay *L, const dc *u, const int64_t *p)
{
    const int nd = L->ndim;
    int64_t q[3];
    for (int d = 0; d < nd; ++d) q[d] = -p[d];
    if (p[nd - 1] > 0) return u[hidx(L, p)];
    if (p[nd - 1] < 0) return conj(u[hidx(L, q)]);
    /* k_last = 0 hyperplane */
    if (!L->sym) return 0.5 * (u[hidx(L, p)] + conj(u[hidx(L, q)]));
    int sgn = 0;
    for (int d = 0; d < nd - 1 && sgn == 0; ++d) sgn = (p[d] > 0) - (p[d] < 0);
    if (sgn > 0) return u[hidx(L, p)];
    if (sgn < 0) return conj(u[hidx(L, q)]);
    return creal(u[hidx(L, p)]); /* DC */
}

/* Compensated (Kahan) accumulation: s + x with the rounding error of each
 * addition carried in c.  The 3D sums reach ~10^8 terms per output, where
 * plain accumulation would leave an error of order 1e-12 in the reference
 * itself (compiled without FMA contraction or reassociation). */
static inline void kahan_add(dc *s, dc *c, dc x)
{
    const dc y = x - *c;
    const dc t = *s + y;
    *c = (t - *s) - y;
    *s = t;
}

static dc hnd_point(const hlay *L, int64_t M, const dc *f, const dc *g, const int64_t *k)
{
    const int nd = L->ndim;
    int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < nd; ++d) {
        const int64_t a = L->m[d] - 1;
        lo[d] = (k[d] - a > -a) ? k[d] - a : -a;
        hi[d] = (k[d] + a < a) ? k[d] + a : a;
    }
    dc s = 0, c = 0;
    for (int64_t i = 0; i < M; ++i) {
        const dc *fi = f + i * L->vol, *gi = g + i * L->vol;
        int64_t p[3] = {0, 0, 0}, q[3] = {0, 0, 0};
        for (p[0] = lo[0]; p[0] <= hi[0]; ++p[0])
            for (p[1] = lo[1]; p[1] <= hi[1]; ++p[1])
                for (p[2] = lo[2]; p[2] <= hi[2]; ++p[2]) {
                    for (int d = 0; d < nd; ++d) q[d] = k[d] - p[d];
                    if (!in_box(L, p) || !in_box(L, q)) continue;
                    kahan_add(&s, &c, hval(L, fi, p) * hval(L, gi, q));
                }
    }
    return s;
}

/* Full output in the storage layout (zero slots written as 0). */
void orc_convnd_hermitian(int ndim, const int64_t *m, const int64_t *n, int64_t M, int sym,
                          const dc *f, const dc *g, dc *h)
{
    hlay L;
    hlay_init(&L, ndim, m, n, sym);
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t lin = 0; lin < L.vol; ++lin) {
        int64_t idx[3], k[3];
        unflatten(ndim, L.n, lin, idx);
        for (int d = 0; d < ndim; ++d) k[d] = idx[d] - L.off[d];
        if (!in_box(&L, k) || k[ndim - 1] < 0) { h[lin] = 0; continue; }
        h[lin] = hnd_point(&L, M, f, g, k);
    }
}

/* Sampled outputs at logical wavenumbers pts[j][0..ndim-1] (k_last >= 0). */
void orc_convnd_hermitian_at(int ndim, const int64_t *m, const int64_t *n, int64_t M, int sym,
                             const dc *f, const dc *g, int64_t npts, const int64_t *pts, dc *out)
{
    hlay L;
    hlay_init(&L, ndim, m, n, sym);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < npts; ++j) out[j] = hnd_point(&L, M, f, g, pts + j * ndim);
}

/* The full Hermitian-extended field over the box B, as a dense array of
 * extents (2m_d - 1) with wavenumber k at index k + m_d - 1 (used by tests to
 * hand the same field to library routines). */
void orc_hermitian_expand(int ndim, const int64_t *m, const int64_t *n, int sym,
                          const dc *u, dc *full)
{
    hlay L;
    hlay_init(&L, ndim, m, n, sym);
    int64_t fe[3] = {1, 1, 1};
    for (int d = 0; d < ndim; ++d) fe[d] = 2 * m[d] - 1;
    int64_t vol = 1;
    for (int d = 0; d < ndim; ++d) vol *= fe[d];
    for (int64_t lin = 0; lin < vol; ++lin) {
        int64_t idx[3], p[3];
        unflatten(ndim, fe, lin, idx);
        for (int d = 0; d < ndim; ++d) p[d] = idx[d] - (m[d] - 1);
        full[lin] = hval(&L, u, p);
    }
}

/* ---------------------------------------------------------------------------
 * Centered Hermitian nD ternary sum (Sec. 4; tconv2 for ndim = 2):
 *   h_k = sum_{p in B} sum_{q in B, k-p-q in B} f_p g_q e_{k-p-q},
 * for k in B with k_last >= 0, the full fields built from the stored halves
 * exactly as for the binary sum above (same storage layout, same reading of
 * the k_last = 0 hyperplane).  Zero slots of h are written as 0.
 * ------------------------------------------------------------------------- */
typedef struct {
    int ndim;
    int64_t a[3], fe[3], fst[3];
    const dc *F, *G, *E;
} tfull;

static int64_t tfidx(const tfull *T, const int64_t *p)
{
    int64_t x = 0;
    for (int d = 0; d < T->ndim; ++d) x += (p[d] + T->a[d]) * T->fst[d];
    return x;
}

static dc tnd_point(const tfull *T, const int64_t *k)
{
    const int nd = T->ndim;
    int64_t p[3] = {0, 0, 0}, q[3] = {0, 0, 0}, r[3] = {0, 0, 0};
    int64_t plo[3] = {0, 0, 0}, phi[3] = {0, 0, 0};
    for (int d = 0; d < nd; ++d) { plo[d] = -T->a[d]; phi[d] = T->a[d]; }
    dc s = 0;
    for (p[0] = plo[0]; p[0] <= phi[0]; ++p[0])
        for (p[1] = plo[1]; p[1] <= phi[1]; ++p[1])
            for (p[2] = plo[2]; p[2] <= phi[2]; ++p[2]) {
                /* q and r = k - p - q both in the box */
                int64_t qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
                int empty = 0;
                for (int d = 0; d < nd; ++d) {
                    const int64_t c = k[d] - p[d], a = T->a[d];
                    qlo[d] = (c - a > -a) ? c - a : -a;
                    qhi[d] = (c + a < a) ? c + a : a;
                    if (qlo[d] > qhi[d]) empty = 1;
                }
                if (empty) continue;
                const dc fp = T->F[tfidx(T, p)];
                dc t = 0;
                for (q[0] = qlo[0]; q[0] <= qhi[0]; ++q[0])
                    for (q[1] = qlo[1]; q[1] <= qhi[1]; ++q[1])
                        for (q[2] = qlo[2]; q[2] <= qhi[2]; ++q[2]) {
                            for (int d = 0; d < nd; ++d) r[d] = k[d] - p[d] - q[d];
                            t += T->G[tfidx(T, q)] * T->E[tfidx(T, r)];
                        }
                s += fp * t;
            }
    return s;
}

static int tfull_init(tfull *T, int ndim, const int64_t *m, const int64_t *n, int sym, const dc *f,
                      const dc *g, const dc *e, dc **buf)
{
    T->ndim = ndim;
    int64_t vol = 1;
    for (int d = 0; d < 3; ++d) { T->a[d] = 0; T->fe[d] = 1; }
    for (int d = 0; d < ndim; ++d) { T->a[d] = m[d] - 1; T->fe[d] = 2 * m[d] - 1; vol *= T->fe[d]; }
    T->fst[2] = 1;
    T->fst[1] = T->fe[2];
    T->fst[0] = T->fe[1] * T->fe[2];
    if (ndim == 2) { T->fst[1] = 1; T->fst[0] = T->fe[1]; }
    if (ndim == 1) T->fst[0] = 1;
    *buf = (dc *)malloc(3 * vol * sizeof(dc));
    if (!*buf) return -1;
    orc_hermitian_expand(ndim, m, n, sym, f, *buf);
    orc_hermitian_expand(ndim, m, n, sym, g, *buf + vol);
    orc_hermitian_expand(ndim, m, n, sym, e, *buf + 2 * vol);
    T->F = *buf;
    T->G = *buf + vol;
    T->E = *buf + 2 * vol;
    return 0;
}

/* Full output in the storage layout. */
int orc_convnd_ternary(int ndim, const int64_t *m, const int64_t *n, int sym, const dc *f,
                       const dc *g, const dc *e, dc *h)
{
    hlay L;
    hlay_init(&L, ndim, m, n, sym);
    tfull T;
    dc *buf = NULL;
    if (tfull_init(&T, ndim, m, n, sym, f, g, e, &buf)) return -1;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t lin = 0; lin < L.vol; ++lin) {
        int64_t idx[3], k[3];
        unflatten(ndim, L.n, lin, idx);
        for (int d = 0; d < ndim; ++d) k[d] = idx[d] - L.off[d];
        if (!in_box(&L, k) || k[ndim - 1] < 0) { h[lin] = 0; continue; }
        h[lin] = tnd_point(&T, k);
    }
    free(buf);
    return 0;
}

/* Sampled outputs at logical wavenumbers pts[j][0..ndim-1] (k in B,
 * k_last >= 0). */
int orc_convnd_ternary_at(int ndim, const int64_t *m, const int64_t *n, int sym, const dc *f,
                          const dc *g, const dc *e, int64_t npts, const int64_t *pts, dc *out)
{
    tfull T;
    dc *buf = NULL;
    if (tfull_init(&T, ndim, m, n, sym, f, g, e, &buf)) return -1;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < npts; ++j) out[j] = tnd_point(&T, pts + j * ndim);
    free(buf);
    return 0;
}
