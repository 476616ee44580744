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
//
// Autotuning (impconv_ragged_plan_autotune, outside any capture): for every
// four-step class the plan times each supported split N = N1 x N2 (the row
// and column FFT sizes, hence the radix schedule of both passes) on
// temporary arrays of the plan's packed shape and keeps the fastest.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
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
        int64_t n2;                       // four-step column length (0: default split)
        std::vector<std::pair<int64_t, double>> tuned;  // (n2, ms) measured by the autotuner
        int lane;                         // stream lane: 0 the caller's stream, 1.. the auxiliary ones
        size_t work_off;                  // four-step classes: byte offset of their work arrays
    };
    std::vector<Class> classes;
    void* dmem;
    size_t work;
    int device;
    // Completion events, one per stream the plan was executed on, recorded
    // after each execution's join: destruction waits for these (the work
    // that reads the plan's descriptor arrays) rather than for the device.
    std::map<hipStream_t, hipEvent_t> done;
    // held while an execution (or the autotuner) enqueues its work or
    // changes the schedule, and by destruction
    std::mutex mu;
};

namespace {
constexpr int kRaggedLanes = 4;  // the caller's stream and three auxiliary streams

// The size classes of a plan run concurrently: the caller's stream forks to
// three auxiliary streams through an event and joins them back at the end,
// so the short fused classes overlap the long multi-pass ones (one launch of
// a short class fills only part of the chip).  The auxiliary streams
// (default priority) and the fork / join events belong to the device, not to
// a plan: they are created once, on the first plan of the device, and kept
// until the process ends, so that creating and destroying plans creates and
// destroys no streams.  `mu` serializes the executions that enqueue through
// them (the events are re-recorded by every execution).
struct Lanes {
    hipStream_t aux[kRaggedLanes - 1];
    hipEvent_t fork;
    hipEvent_t join[kRaggedLanes - 1];
    std::mutex mu;
};
std::mutex g_lanes_mu;
Lanes* g_lanes[64];

Lanes* device_lanes(int dev)
{
    if (dev < 0 || dev >= 64) {
        hip_fail(hipErrorInvalidDevice, "ragged streams");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_lanes_mu);
    if (g_lanes[dev]) return g_lanes[dev];
    auto* L = new Lanes();
    int streams = 0, joins = 0;
    hipError_t e = hipEventCreateWithFlags(&L->fork, hipEventDisableTiming);
    if (e != hipSuccess) L->fork = nullptr;
    for (int l = 0; l < kRaggedLanes - 1 && e == hipSuccess; ++l) {
        e = hipStreamCreateWithFlags(&L->aux[l], hipStreamNonBlocking);
        if (e != hipSuccess) break;
        ++streams;
        e = hipEventCreateWithFlags(&L->join[l], hipEventDisableTiming);
        if (e == hipSuccess) ++joins;
    }
    if (e != hipSuccess) {
        // (nothing has used them yet: safe to release)
        for (int l = 0; l < streams; ++l) (void)hipStreamDestroy(L->aux[l]);
        for (int l = 0; l < joins; ++l) (void)hipEventDestroy(L->join[l]);
        if (L->fork) (void)hipEventDestroy(L->fork);
        delete L;
        hip_fail(e, "ragged streams");
        return nullptr;
    }
    g_lanes[dev] = L;
    return L;
}

// Destroys a plan that was never executed (creation failed part way).
void free_unused(impconv_ragged_plan* p)
{
    if (p->dmem) (void)hipFree(p->dmem);
    delete p;
}
}  // namespace

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
    if (!device_lanes(p->device)) {
        delete p;
        return IMPCONV_E_HIP;
    }
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
    // lanes: longest class first, each to the lane with the least estimated
    // work (pairs x N log N); the four-step classes get work arrays of their
    // own, since classes on different lanes run at the same time
    double load[kRaggedLanes] = {0, 0, 0, 0};
    for (const auto& q : pend) {
        int lane = 0;
        for (int l = 1; l < kRaggedLanes; ++l)
            if (load[l] < load[lane]) lane = l;
        load[lane] += double(q.count) * double(q.N) * std::log2(double(q.N) + 1.0) * (q.N > kRowMax ? 3.0 : 1.0);
        size_t off = 0;
        if (q.N > kRowMax) {
            off = p->work;
            p->work += size_t(4) * q.count * q.N * cs;
        }
        p->classes.push_back({q.N, q.count, q.maxm, d + q.off_at, d + q.m_at, 0, {}, lane, off});
    }
    // the four-step classes' column twiddle tables are created here, so that
    // executing the plan allocates nothing (and may be captured)
    for (const auto& q : pend) {
        if (q.N <= kRowMax) continue;
        int64_t N1, N2;
        fourstep_split(q.N, &N1, &N2);
        if (!fs_twiddles(dtype, N2, N1)) {
            free_unused(p);
            return IMPCONV_E_HIP;
        }
    }
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
    const uint32_t known = IMPCONV_REV_F | IMPCONV_CONJ_G | IMPCONV_REV_OUT | IMPCONV_ONE_STREAM;
    if (flags & ~known) return fail(IMPCONV_E_ARG, "unsupported flag for a ragged batch");
    const bool one = (flags & IMPCONV_ONE_STREAM) != 0;
    flags &= ~IMPCONV_ONE_STREAM;
    if (p->npairs == 0) return IMPCONV_OK;
    const size_t cs = p->dt ? 16 : 8;
    for (const void* q : {f, g, (const void*)h}) {
        if (!q) return fail(IMPCONV_E_ARG, "null data pointer");
        if (reinterpret_cast<uintptr_t>(q) % cs) return fail(IMPCONV_E_ALIGN, "data pointer misaligned");
    }
    const size_t bytes = size_t(p->extent) * cs;
    if (bad_alias(h, bytes, f, bytes) || bad_alias(h, bytes, g, bytes))
        return fail(IMPCONV_E_ARG, "h overlaps an input (only h == f or h == g is allowed)");
    if (work_bytes < p->work) return fail(IMPCONV_E_WORKSPACE, "workspace too small: need " + std::to_string(p->work) + " bytes");
    if (p->work && !work) return fail(IMPCONV_E_ARG, "work is NULL");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != p->device) return fail(IMPCONV_E_ARG, "plan was created on another device");
    const DevTables* tb = tables();
    if (!tb) return IMPCONV_E_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Lanes* L = device_lanes(p->device);
    if (!L) return IMPCONV_E_HIP;
    auto* pm = const_cast<impconv_ragged_plan*>(p);
    // lock order: the plan, then the device's lanes
    std::lock_guard<std::mutex> lk(pm->mu);
    std::unique_lock<std::mutex> lanes_lock(L->mu, std::defer_lock);
    impconv_status st = IMPCONV_OK;
    bool forked = false;
    if (!one) {
        // fork: every auxiliary stream waits for the work queued on s so far
        lanes_lock.lock();
        hipError_t e = hipEventRecord(L->fork, s);
        for (int l = 0; l < kRaggedLanes - 1 && e == hipSuccess; ++l) e = hipStreamWaitEvent(L->aux[l], L->fork, 0);
        if (e != hipSuccess) return hip_fail(e, "ragged fork");
        forked = true;
    }
    for (const auto& c : p->classes) {
        hipStream_t cs_ = one || c.lane == 0 ? s : L->aux[c.lane - 1];
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
            const hipError_t e = launch_row_complex(p->dt, int(c.N), a, cs_);
            if (e != hipSuccess) st = hip_fail(e, "ragged row class");
        } else {
            st = large1d_run_ragged(*tb, p->dt, c.count, c.N, c.maxm, f, g, h,
                                    static_cast<char*>(work) + c.work_off, c.d_off, c.d_m, flags, cs_, c.n2);
        }
        if (st) break;
    }
    // join, also after a failed launch: s waits for every auxiliary stream,
    // so that nothing of this call is left unordered with what s does next
    // (and a capture sees every forked stream rejoin)
    if (forked) {
        for (int l = 0; l < kRaggedLanes - 1; ++l) {
            hipError_t e = hipEventRecord(L->join[l], L->aux[l]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, L->join[l], 0);
            if (e != hipSuccess && !st) st = hip_fail(e, "ragged join");
        }
    }
    // completion of this execution on s, for destruction
    hipEvent_t& dn = pm->done[s];
    hipError_t e = dn ? hipSuccess : hipEventCreateWithFlags(&dn, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(dn, s);
    if (e != hipSuccess && !st) st = hip_fail(e, "ragged completion event");
    return st;
}

impconv_status impconv_ragged_plan_autotune(impconv_ragged_plan* p, void* stream)
{
    if (!p) return fail(IMPCONV_E_ARG, "plan is NULL");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != p->device) return fail(IMPCONV_E_ARG, "plan was created on another device");
    std::lock_guard<std::mutex> lk(p->mu);  // no execution enqueues while the schedule changes
    bool any = false;
    for (const auto& c : p->classes) any = any || c.N > kRowMax;
    if (!any) return IMPCONV_OK;
    const DevTables* tb = tables();
    if (!tb) return IMPCONV_E_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t cs = p->dt ? 16 : 8;
    const size_t bytes = size_t(p->extent) * cs;
    void *f = nullptr, *g = nullptr, *h = nullptr, *w = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    impconv_status st = IMPCONV_OK;
    auto cleanup = [&]() {
        // kernels already launched on s may still use the arrays (also
        // after a failure part way): wait for them before freeing
        (void)hipStreamSynchronize(s);
        for (void* q : {f, g, h, w})
            if (q) (void)hipFree(q);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t e = hipMalloc(&f, bytes);
    if (e == hipSuccess) e = hipMalloc(&g, bytes);
    if (e == hipSuccess) e = hipMalloc(&h, bytes);
    if (e == hipSuccess) e = hipMalloc(&w, std::max<size_t>(p->work, 256));
    if (e == hipSuccess) e = hipMemsetAsync(f, 0, bytes, s);
    if (e == hipSuccess) e = hipMemsetAsync(g, 0, bytes, s);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "autotune buffers");
    }
    for (auto& c : p->classes) {
        if (c.N <= kRowMax) continue;
        c.tuned.clear();
        double best = 1e30;
        int64_t best_n2 = 0;
        for (int64_t n2 : fourstep_splits(c.N)) {
            constexpr int reps = 3;
            for (int r = 0; r <= reps && !st; ++r) {
                if (r == 1 && (e = hipEventRecord(e0, s)) != hipSuccess) st = hip_fail(e, "autotune event");
                if (!st) st = large1d_run_ragged(*tb, p->dt, c.count, c.N, c.maxm, f, g, h, w, c.d_off, c.d_m, 0, s, n2);
            }
            float ms = 0;
            if (!st && (e = hipEventRecord(e1, s)) != hipSuccess) st = hip_fail(e, "autotune event");
            if (!st && (e = hipEventSynchronize(e1)) != hipSuccess) st = hip_fail(e, "autotune sync");
            if (!st && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) st = hip_fail(e, "autotune timing");
            if (st) break;
            const double t = double(ms) / reps;
            c.tuned.push_back({n2, t});
            if (t < best) {
                best = t;
                best_n2 = n2;
            }
        }
        if (st) break;
        c.n2 = best_n2;
    }
    cleanup();
    return st;
}

impconv_status impconv_ragged_plan_schedule(const impconv_ragged_plan* p, char* buf, size_t cap, size_t* len)
{
    if (!p || !len) return fail(IMPCONV_E_ARG, "null argument");
    std::string js = "[";
    for (size_t i = 0; i < p->classes.size(); ++i) {
        const auto& c = p->classes[i];
        int64_t N1 = 0, N2 = 0;
        if (c.N > kRowMax) {
            fourstep_split(c.N, &N1, &N2);
            if (c.n2) {
                N2 = c.n2;
                N1 = c.N / c.n2;
            }
        }
        js += (i ? "," : "") + std::string("{\"N\":") + std::to_string(c.N) + ",\"pairs\":" + std::to_string(c.count) +
              ",\"method\":\"" + (c.N <= kRowMax ? "fused" : "four-step") + "\"" +
              ",\"stream\":" + std::to_string(c.lane);
        if (c.N > kRowMax) {
            js += ",\"N1\":" + std::to_string(N1) + ",\"N2\":" + std::to_string(N2) + ",\"tuned_ms\":{";
            for (size_t j = 0; j < c.tuned.size(); ++j) {
                char t[64];
                std::snprintf(t, sizeof(t), "%s\"%lld\":%.5f", j ? "," : "", (long long)c.tuned[j].first, c.tuned[j].second);
                js += t;
            }
            js += "}";
        }
        js += "}";
    }
    js += "]";
    *len = js.size();
    if (buf && cap > 0) {
        const size_t n = std::min(cap - 1, js.size());
        std::memcpy(buf, js.data(), n);
        buf[n] = 0;
    }
    return IMPCONV_OK;
}

impconv_status impconv_ragged_plan_destroy(impconv_ragged_plan* plan)
{
    if (!plan) return IMPCONV_OK;
    {
        // Executions still in flight read the plan's descriptor arrays: wait
        // for the completion event each stream recorded after its last
        // execution (a host wait on those points of those streams only; the
        // device's auxiliary streams are not the plan's and stay).
        std::lock_guard<std::mutex> lk(plan->mu);
        for (auto& kv : plan->done) {
            (void)hipEventSynchronize(kv.second);
            (void)hipEventDestroy(kv.second);
        }
        plan->done.clear();
    }
    int cur = -1;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    if (have_cur && cur != plan->device) (void)hipSetDevice(plan->device);
    if (plan->dmem) (void)hipFree(plan->dmem);
    if (have_cur && cur != plan->device) (void)hipSetDevice(cur);
    delete plan;
    return IMPCONV_OK;
}

}  // extern "C"
