// ragged.hip -- batches of complex 1D convolutions of uneven lengths.
//
// The plan groups the pairs by FFT size N = next_pow2(m) ("size classes"),
// copies each class's (offset, length) descriptors to the device once, and at
// execution issues one launch per class: the fused row kernel for classes
// with N <= kRowMax (each workgroup group reads its pair's offset and length
// from the descriptor arrays), the three four-step passes for longer ones.
// Classes are issued longest first so the long multi-pass classes start
// while the GPU is empty.  Execution performs no allocation, copy or
// synchronization, so it can be captured in a hipGraph.
#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "colpass.hpp"
#include "launch.hpp"
#include "multid.hpp"

using namespace impconv;

struct impconv_ragged_plan {
    int dt;
    int64_t npairs;
    int64_t extent;  // elements the packed arrays must hold: max(offset + m)
    struct Class {
        int64_t N, count, maxm;
        const int64_t* d_off;
        const int64_t* d_m;
    };
    std::vector<Class> classes;
    void* dmem;
    size_t work;
    int device;
};

namespace {
#define HIPCHK(expr, what)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(e_, what);     \
    } while (0)
}  // namespace

extern "C" {

impconv_status impconv_ragged_plan_create(int dtype, int64_t npairs, const int64_t* m_host,
                                          const int64_t* offset_host, impconv_ragged_plan** plan)
{
    if (!plan) return fail(IMPCONV_E_ARG, "plan is NULL");
    *plan = nullptr;
    if (dtype != IMPCONV_C64 && dtype != IMPCONV_C128) return fail(IMPCONV_E_ARG, "bad dtype");
    if (npairs < 0) return fail(IMPCONV_E_SIZE, "npairs must be >= 0");
    if (npairs > 0 && (!m_host || !offset_host)) return fail(IMPCONV_E_ARG, "null descriptor array");
    const size_t cs = dtype ? 16 : 8;
    std::map<int64_t, std::vector<int64_t>> byN;  // N -> pair indices
    std::vector<std::pair<int64_t, int64_t>> spans;
    int64_t extent = 0;
    for (int64_t j = 0; j < npairs; ++j) {
        const int64_t m = m_host[j], o = offset_host[j];
        if (m < 1) return fail(IMPCONV_E_SIZE, "pair length must be >= 1");
        if (o < 0) return fail(IMPCONV_E_ARG, "negative pair offset");
        if (next_pow2(m) > (int64_t(1) << 17)) return fail(IMPCONV_E_UNSUPPORTED, "pair length > 131072");
        byN[next_pow2(m)].push_back(j);
        spans.push_back({o, o + m});
        extent = std::max(extent, o + m);
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return fail(IMPCONV_E_ARG, "pairs overlap in the packed arrays");
    if (!tables()) return IMPCONV_E_HIP;
    auto* p = new impconv_ragged_plan();
    p->dt = dtype;
    p->npairs = npairs;
    p->extent = extent;
    p->dmem = nullptr;
    p->work = 0;
    (void)hipGetDevice(&p->device);
    std::vector<int64_t> host;
    struct Pending { int64_t N, count, maxm; size_t off_at, m_at; };
    std::vector<Pending> pend;
    for (auto it = byN.rbegin(); it != byN.rend(); ++it) {  // longest class first
        const auto& idx = it->second;
        Pending q{it->first, int64_t(idx.size()), 0, host.size(), 0};
        for (int64_t j : idx) host.push_back(offset_host[j]);
        q.m_at = host.size();
        for (int64_t j : idx) {
            host.push_back(m_host[j]);
            q.maxm = std::max(q.maxm, m_host[j]);
        }
        pend.push_back(q);
        if (q.N > kRowMax) p->work = std::max(p->work, size_t(4) * q.count * q.N * cs);
    }
    if (!host.empty()) {
        hipError_t e = hipMalloc(&p->dmem, host.size() * sizeof(int64_t));
        if (e == hipSuccess) e = hipMemcpy(p->dmem, host.data(), host.size() * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (p->dmem) (void)hipFree(p->dmem);
            delete p;
            return hip_fail(e, "ragged descriptor upload");
        }
    }
    const int64_t* d = static_cast<const int64_t*>(p->dmem);
    for (const auto& q : pend) p->classes.push_back({q.N, q.count, q.maxm, d + q.off_at, d + q.m_at});
    *plan = p;
    return IMPCONV_OK;
}

impconv_status impconv_ragged_workspace(const impconv_ragged_plan* plan, size_t* bytes)
{
    if (!plan || !bytes) return fail(IMPCONV_E_ARG, "null argument");
    *bytes = plan->work;
    return IMPCONV_OK;
}

impconv_status impconv_ragged_execute(const impconv_ragged_plan* p, const void* f, const void* g,
                                      void* h, void* work, size_t work_bytes, uint32_t flags,
                                      void* stream)
{
    if (!p) return fail(IMPCONV_E_ARG, "plan is NULL");
    const uint32_t known = IMPCONV_REV_F | IMPCONV_CONJ_G | IMPCONV_REV_OUT;
    if (flags & ~known) return fail(IMPCONV_E_ARG, "unsupported flag for a ragged batch");
    if (p->npairs == 0) return IMPCONV_OK;
    const size_t cs = p->dt ? 16 : 8;
    for (const void* q : {f, g, (const void*)h}) {
        if (!q) return fail(IMPCONV_E_ARG, "null data pointer");
        if (reinterpret_cast<uintptr_t>(q) % cs) return fail(IMPCONV_E_ALIGN, "data pointer misaligned");
    }
    const size_t bytes = size_t(p->extent) * cs;
    auto ov = [](const void* a, const void* b, size_t n) {
        const char* x = (const char*)a; const char* y = (const char*)b;
        return x < y + n && y < x + n;
    };
    if (ov(h, f, bytes) || ov(h, g, bytes)) return fail(IMPCONV_E_ARG, "h overlaps an input");
    if (work_bytes < p->work) return fail(IMPCONV_E_WORKSPACE, "workspace too small: need " + std::to_string(p->work) + " bytes");
    if (p->work && !work) return fail(IMPCONV_E_ARG, "work is NULL");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != p->device) return fail(IMPCONV_E_ARG, "plan was created on another device");
    const DevTables* tb = tables();
    if (!tb) return IMPCONV_E_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (const auto& c : p->classes) {
        if (c.N <= kRowMax) {
            RowArgs a;
            std::memset(&a, 0, sizeof(a));
            a.tw = tb->tw[p->dt];
            a.tw3 = tb->tw3[p->dt];
            a.f = f; a.g = g; a.h = h;
            a.nrows = c.count;
            a.m = c.maxm;
            a.M = 1;
            a.row_off = c.d_off;
            a.row_m = c.d_m;
            a.flags = flags & (kRevF | kConjG | kRevOut);
            HIPCHK(launch_row_complex(p->dt, int(c.N), a, s), "ragged row class");
        } else {
            impconv_status st = large1d_run_ragged(*tb, p->dt, c.count, c.N, c.maxm, f, g, h, work,
                                                   c.d_off, c.d_m, flags, s);
            if (st) return st;
        }
    }
    return IMPCONV_OK;
}

impconv_status impconv_ragged_plan_destroy(impconv_ragged_plan* plan)
{
    if (!plan) return IMPCONV_OK;
    if (plan->dmem) (void)hipFree(plan->dmem);
    delete plan;
    return IMPCONV_OK;
}

}  // extern "C"
