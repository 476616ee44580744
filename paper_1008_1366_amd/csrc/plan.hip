// plan.hip -- the descriptor-based plan API (one entry point for every kind
// and dimension) and the one-shot ragged wrapper with its plan cache.
//
// A plan validates a descriptor once, creates the device's twiddle tables
// and fixes the workspace size; executing it dispatches to the 1D, 2D or 3D
// convolution of its kind.  Plans hold no data-sized memory.
#include <algorithm>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "multid.hpp"
#include "runtime.hpp"

struct impconv_plan {
    impconv_desc d;
    size_t work;
};

namespace {

using namespace impconv;

impconv_status validate(const impconv_desc* d, size_t* work)
{
    if (!d) return fail(IMPCONV_E_ARG, "desc is NULL");
    if (d->ndim < 1 || d->ndim > 3) return fail(IMPCONV_E_ARG, "ndim must be 1, 2 or 3");
    if (d->kind != IMPCONV_COMPLEX && d->kind != IMPCONV_HERMITIAN && d->kind != IMPCONV_TERNARY)
        return fail(IMPCONV_E_ARG, "bad kind");
    if (d->ndim == 1)
        return impconv_conv1d_workspace(d->kind, d->dtype, d->batch, d->kind == IMPCONV_TERNARY ? 1 : d->M,
                                        d->m[0], d->flags, work);
    if (d->kind == IMPCONV_TERNARY && d->ndim != 2)
        return fail(IMPCONV_E_UNSUPPORTED, "ternary convolutions are 1D or 2D in this build");
    return impconv_convnd_workspace(d->kind, d->dtype, d->ndim, d->m, d->n, d->batch,
                                    d->kind == IMPCONV_TERNARY ? 1 : d->M, d->flags, work);
}

// One-shot ragged wrapper: plans keyed by device, dtype and the descriptor
// arrays, the most recently used kept first.
struct CachedRagged {
    int device, dtype;
    std::vector<int64_t> m, off;
    impconv_ragged_plan* plan;
};
std::mutex c_mu;
std::deque<CachedRagged> c_plans;
constexpr size_t kCacheMax = 16;

// The caller holds c_mu until it has finished with *out: another thread's
// lookup may evict (destroy) any plan it did not just return.
impconv_status cached_ragged(int dtype, int64_t npairs, const int64_t* m_host, const int64_t* off_host,
                             impconv_ragged_plan** out)
{
    if (npairs < 0) return fail(IMPCONV_E_SIZE, "npairs must be >= 0");
    if (npairs > 0 && (!m_host || !off_host)) return fail(IMPCONV_E_ARG, "null descriptor array");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    for (auto it = c_plans.begin(); it != c_plans.end(); ++it) {
        if (it->device == dev && it->dtype == dtype && int64_t(it->m.size()) == npairs &&
            std::equal(it->m.begin(), it->m.end(), m_host) && std::equal(it->off.begin(), it->off.end(), off_host)) {
            CachedRagged hit = *it;
            c_plans.erase(it);
            c_plans.push_front(hit);
            *out = hit.plan;
            return IMPCONV_OK;
        }
    }
    impconv_ragged_plan* p = nullptr;
    impconv_status st = impconv_ragged_plan_create(dtype, npairs, m_host, off_host, &p);
    if (st) return st;
    c_plans.push_front({dev, dtype, std::vector<int64_t>(m_host, m_host + npairs),
                        std::vector<int64_t>(off_host, off_host + npairs), p});
    while (c_plans.size() > kCacheMax) {
        // (destroying a plan waits for its own executions still in flight)
        (void)impconv_ragged_plan_destroy(c_plans.back().plan);
        c_plans.pop_back();
    }
    *out = p;
    return IMPCONV_OK;
}

}  // namespace

extern "C" {

impconv_status impconv_plan_create(impconv_plan** plan, const impconv_desc* desc)
{
    if (!plan) return fail(IMPCONV_E_ARG, "plan is NULL");
    *plan = nullptr;
    size_t work = 0;
    impconv_status st = validate(desc, &work);
    if (st) return st;
    if ((st = impconv_init())) return st;
    if (desc->ndim == 1 && (st = conv1d_prepare(desc->kind, desc->dtype, desc->batch, desc->M, desc->m[0],
                                                desc->flags)))
        return st;
    auto* p = new impconv_plan();
    p->d = *desc;
    p->work = work;
    *plan = p;
    return IMPCONV_OK;
}

impconv_status impconv_workspace_bytes(const impconv_plan* plan, size_t* bytes)
{
    if (!plan || !bytes) return fail(IMPCONV_E_ARG, "null argument");
    *bytes = plan->work;
    return IMPCONV_OK;
}

impconv_status impconv_execute(const impconv_plan* plan, const void* f, const void* g, const void* e, void* h,
                               void* work, size_t work_bytes, void* stream)
{
    if (!plan) return fail(IMPCONV_E_ARG, "plan is NULL");
    const impconv_desc& d = plan->d;
    if ((d.kind == IMPCONV_TERNARY) != (e != nullptr))
        return fail(IMPCONV_E_ARG, d.kind == IMPCONV_TERNARY ? "ternary plan needs e" : "e is only for ternary plans");
    if (d.ndim == 1) {
        switch (d.kind) {
            case IMPCONV_COMPLEX:
                return impconv_conv1d_complex(d.dtype, d.batch, d.M, d.m[0], f, g, h, work, work_bytes, d.flags, stream);
            case IMPCONV_HERMITIAN:
                return impconv_conv1d_hermitian(d.dtype, d.batch, d.M, d.m[0], f, g, h, work, work_bytes, d.flags, stream);
            default:
                return impconv_conv1d_ternary(d.dtype, d.batch, d.m[0], f, g, e, h, work, work_bytes, d.flags, stream);
        }
    }
    if (d.ndim == 2 && d.kind == IMPCONV_TERNARY)
        return impconv_conv2d_ternary(d.dtype, d.batch, d.m, d.n, f, g, e, h, work, work_bytes, d.flags, stream);
    if (d.ndim == 2)
        return impconv_conv2d(d.kind, d.dtype, d.batch, d.M, d.m, d.n, f, g, h, work, work_bytes, d.flags, stream);
    return impconv_conv3d(d.kind, d.dtype, d.batch, d.M, d.m, d.n, f, g, h, work, work_bytes, d.flags, stream);
}

impconv_status impconv_plan_destroy(impconv_plan* plan)
{
    delete plan;
    return IMPCONV_OK;
}

impconv_status impconv_conv1d_complex_ragged_workspace(int dtype, int64_t npairs, const int64_t* m_host,
                                                       const int64_t* offset_host, size_t* bytes)
{
    if (!bytes) return fail(IMPCONV_E_ARG, "bytes is NULL");
    impconv_ragged_plan* p = nullptr;
    std::lock_guard<std::mutex> lk(c_mu);
    impconv_status st = cached_ragged(dtype, npairs, m_host, offset_host, &p);
    if (st) return st;
    return impconv_ragged_workspace(p, bytes);
}

impconv_status impconv_conv1d_complex_ragged(int dtype, int64_t npairs, const int64_t* m_host,
                                             const int64_t* offset_host, const void* f, const void* g, void* h,
                                             void* work, size_t work_bytes, uint32_t flags, void* stream)
{
    impconv_ragged_plan* p = nullptr;
    // held through the execution's enqueue, so that no other call evicts p
    std::lock_guard<std::mutex> lk(c_mu);
    impconv_status st = cached_ragged(dtype, npairs, m_host, offset_host, &p);
    if (st) return st;
    return impconv_ragged_execute(p, f, g, h, work, work_bytes, flags, stream);
}

}  // extern "C"
