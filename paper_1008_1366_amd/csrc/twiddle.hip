// twiddle.hip -- FP64 roots of unity for the FFT stages and the residue
// shifts (Sec. 2.1 discussion of the zeta_N^k factors).  The paper builds
// them from two short tables with one complex multiply; on the GPU the full
// per-size tables cost only ~16 MB of HBM and one cached load per use, so
// they are stored directly: tw_N[j] = zeta_N^j for every power-of-two N up to
// 2^18 (concatenated, tw_N at offset N - 1), zeta_{3N}^j, j < N, for the
// 2/3-rule shifts, and zeta_{q NP}^j, j < q NP, for the general p/q rule.
// Each value is computed in long double with the argument reduced exactly
// (integer j mod denom, folded into the first octant) and rounded once to
// double; the complex64 tables round those doubles to float, and for the
// compensated products a second complex64 table holds the rounded remainder.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "cx.hpp"
#include "runtime.hpp"

namespace impconv {

// zeta_denom^j = exp(2 pi i j / denom) for j = 0..count-1, FP64, interleaved.
void gen_roots(int64_t denom, int64_t count, double* out)
{
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int64_t j = 0; j < count; ++j) {
        // exact reduction in units of 1/(8 denom) of a turn: P = 8 (j mod denom),
        // quadrant q = P / (2 denom), angle = q pi/2 + 2 pi b / (8 denom)
        const int64_t D = 8 * denom;
        const int64_t P = 8 * (j % denom);
        const int64_t q = P / (2 * denom);
        const int64_t b = P - q * 2 * denom;
        long double c, s;
        if (b <= denom) {  // within the first octant of the quadrant
            long double th = two_pi * (long double)b / (long double)D;
            c = cosl(th);
            s = sinl(th);
        } else {  // use complement: angle' = pi/2 - angle
            long double th = two_pi * (long double)(2 * denom - b) / (long double)D;
            c = sinl(th);
            s = cosl(th);
        }
        long double re, im;
        switch (q & 3) {
            case 0: re = c; im = s; break;
            case 1: re = -s; im = c; break;
            case 2: re = -c; im = -s; break;
            default: re = s; im = -c; break;
        }
        out[2 * j] = (double)re;
        out[2 * j + 1] = (double)im;
    }
}

int64_t twq_off(int q, int64_t NP)
{
    int64_t off = 0;
    for (int qq : kTwqList) {
        for (int l = 0; l <= kTwqLog; ++l) {
            const int64_t n = int64_t(1) << l;
            if (qq == q && n == NP) return off;
            off += qq * n;
        }
    }
    return -1;
}

namespace {

std::mutex g_mu;
DevTables g_tab[64];
bool g_have[64];

// Low parts of a table for the compensated complex64 products:
// lo = float(w - double(float(w))) per component.
std::vector<double> low_parts(const std::vector<double>& src)
{
    std::vector<double> lo(src.size());
    for (size_t i = 0; i < src.size(); ++i) lo[i] = (double)(float)(src[i] - (double)(float)src[i]);
    return lo;
}

template <typename T>
hipError_t upload(const std::vector<double>& src, const void** dst)
{
    const size_t n = src.size() / 2;
    std::vector<C<T>> host(n);
    for (size_t i = 0; i < n; ++i) host[i] = C<T>{(T)src[2 * i], (T)src[2 * i + 1]};
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(C<T>));
    if (e != hipSuccess) return e;
    e = hipMemcpy(p, host.data(), n * sizeof(C<T>), hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(p); return e; }
    *dst = p;
    return hipSuccess;
}

}  // namespace

const DevTables* tables()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= 64) {
        hip_fail(e == hipSuccess ? hipErrorInvalidDevice : e, "hipGetDevice");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_have[dev]) return &g_tab[dev];
    // zeta_N^j for N = 2^0 .. 2^kTwLog, concatenated at offset N - 1
    std::vector<double> tw(2 * ((int64_t(1) << (kTwLog + 1)) - 1));
    for (int l = 0; l <= kTwLog; ++l) {
        const int64_t N = int64_t(1) << l;
        gen_roots(N, N, tw.data() + 2 * (N - 1));
    }
    std::vector<double> tw3(2 * ((int64_t(1) << (kTw3Log + 1)) - 1));
    for (int l = 0; l <= kTw3Log; ++l) {
        const int64_t N = int64_t(1) << l;
        gen_roots(3 * N, N, tw3.data() + 2 * (N - 1));
    }
    std::vector<double> twq;
    for (int q : kTwqList) {
        for (int l = 0; l <= kTwqLog; ++l) {
            const int64_t NP = int64_t(1) << l;
            const size_t at = twq.size();
            twq.resize(at + 2 * q * NP);
            gen_roots(q * NP, q * NP, twq.data() + at);
        }
    }
    DevTables t{};
    if ((e = hipDeviceGetAttribute(&t.ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) {
        hip_fail(e, "hipDeviceGetAttribute");
        return nullptr;
    }
    if ((e = upload<float>(tw, &t.tw[0])) != hipSuccess ||
        (e = upload<double>(tw, &t.tw[1])) != hipSuccess ||
        (e = upload<float>(tw3, &t.tw3[0])) != hipSuccess ||
        (e = upload<double>(tw3, &t.tw3[1])) != hipSuccess ||
        (e = upload<float>(twq, &t.twq[0])) != hipSuccess ||
        (e = upload<double>(twq, &t.twq[1])) != hipSuccess ||
        (e = upload<float>(low_parts(tw), &t.twlo)) != hipSuccess ||
        (e = upload<float>(low_parts(tw3), &t.tw3lo)) != hipSuccess) {
        hip_fail(e, "twiddle table upload");
        return nullptr;
    }
    g_tab[dev] = t;
    g_have[dev] = true;
    return &g_tab[dev];
}

// zeta_F^{j2 c} stored at [j2][c] (j2 < N2, c < N1, F = N1 N2): the column
// twiddles of the four-step passes, laid out so that the loads of a wave
// (consecutive columns c) are contiguous instead of j2 elements apart.  The
// values are the FP64 roots (rounded to float for complex64), as in the
// zeta_F table.  Created once per device, dtype and split, on first use.
const void* fs_twiddles(int dt, int64_t N2, int64_t N1)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        hip_fail(e, "hipGetDevice");
        return nullptr;
    }
    static std::map<std::tuple<int, int, int64_t, int64_t>, const void*> cache;
    std::lock_guard<std::mutex> lk(g_mu);
    const auto key = std::make_tuple(dev, dt, N2, N1);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const int64_t F = N1 * N2;
    std::vector<double> roots(2 * F), t(2 * F);
    gen_roots(F, F, roots.data());
    for (int64_t j2 = 0; j2 < N2; ++j2)
        for (int64_t c = 0; c < N1; ++c) {
            const int64_t idx = (j2 * c) % F;
            t[2 * (j2 * N1 + c)] = roots[2 * idx];
            t[2 * (j2 * N1 + c) + 1] = roots[2 * idx + 1];
        }
    const void* p = nullptr;
    e = dt ? upload<double>(t, &p) : upload<float>(t, &p);
    if (e != hipSuccess) {
        hip_fail(e, "four-step twiddle table upload");
        return nullptr;
    }
    cache[key] = p;
    return p;
}

// ------------------------------------------------------------------ timing
namespace {
struct Rec {
    std::string name;
    hipEvent_t a, b;
};
std::mutex t_mu;
std::atomic<bool> t_on{false};  // read by launches on any thread
std::vector<Rec> t_recs;
thread_local hipEvent_t t_pending = nullptr;

hipEvent_t new_event()
{
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool timing_on() { return t_on.load(); }

void timing_begin(hipStream_t s)
{
    if (!t_on.load()) return;
    t_pending = new_event();
    if (t_pending) (void)hipEventRecord(t_pending, s);
}

void timing_end(const char* name, hipStream_t s)
{
    if (!t_on.load() || !t_pending) return;
    hipEvent_t b = new_event();
    if (!b) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(t_mu);
    t_recs.push_back({name, t_pending, b});
    t_pending = nullptr;
}

}  // namespace impconv

extern "C" {

void impconv_timing_enable(int on)
{
    impconv::t_on.store(on != 0);
}

// Waits for the recorded events, writes a JSON array of per-kernel aggregates
// {"name", "count", "total_ms", "min_ms", "max_ms"} into buf (NUL-terminated,
// truncated to cap), releases the events and returns the full length.
size_t impconv_timing_report(char* buf, size_t cap)
{
    using namespace impconv;
    std::vector<Rec> recs;
    {
        std::lock_guard<std::mutex> lk(t_mu);
        recs.swap(t_recs);
    }
    struct Agg { int64_t n = 0; double tot = 0, mn = 1e300, mx = 0; };
    std::vector<std::pair<std::string, Agg>> aggs;
    for (auto& r : recs) {
        float ms = 0;
        (void)hipEventSynchronize(r.b);
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
        Agg* g = nullptr;
        for (auto& p : aggs)
            if (p.first == r.name) g = &p.second;
        if (!g) {
            aggs.push_back({r.name, Agg{}});
            g = &aggs.back().second;
        }
        g->n++;
        g->tot += ms;
        g->mn = std::min(g->mn, double(ms));
        g->mx = std::max(g->mx, double(ms));
    }
    std::string s = "[";
    char tmp[512];
    for (size_t i = 0; i < aggs.size(); ++i) {
        const auto& a = aggs[i].second;
        snprintf(tmp, sizeof(tmp), "%s{\"name\": \"%s\", \"count\": %lld, \"total_ms\": %.6f, \"min_ms\": %.6f, \"max_ms\": %.6f}",
                 i ? ", " : "", aggs[i].first.c_str(), (long long)a.n, a.tot, a.mn, a.mx);
        s += tmp;
    }
    s += "]";
    if (buf && cap) {
        const size_t n = std::min(cap - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return s.size();
}

}  // extern "C"
