// ragged.hip -- batches of complex 1D convolutions of uneven lengths.
//
// The plan groups the pairs by FFT size N = next_pow2(m) ("size classes"),
// copies each class's (offset, length) descriptors to the device once, and at
// execution launches:
//  - the fused classes (N <= kRowMax) together in one persistent launch that
//    drains a work queue of items, longest class first (queue.hpp), or, if
//    the autotuner finds that faster, one launch of the fused row kernel per
//    class (each workgroup group reads its pair's offset and length from the
//    descriptor arrays);
//  - the longer classes as the three four-step passes each.
// The four-step classes run on auxiliary streams beside the fused work.
// Execution performs no allocation, copy or synchronization, so it can be
// captured in a hipGraph.
//
// Autotuning (impconv_ragged_plan_autotune, outside any capture) times, on
// temporary arrays of the plan's packed shape: for every four-step class each
// supported split N = N1 x N2 (the radix schedule of both passes); for every
// fused class in the queue both supported values-per-thread E (the radix
// schedule and the number of pairs per item); then the fused classes as one
// queue launch against one launch per class.  Each class's winner is kept in
// the process-wide schedule cache under (architecture, variant, dtype, N), so
// a later plan with a class of the same key takes it without timing.
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
#include "queue.hpp"
#include "schedule.hpp"

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
        int E;                            // fused classes in the queue: values per thread
        bool queued;                      // fused class the queue kernel can run
        std::vector<std::pair<int64_t, double>> tuned;  // (n2 or E, ms) measured by the autotuner
        const char* source;               // where the schedule came from: "default", "timed", "cache"
        int lane;                         // stream lane: 0 the caller's stream, 1.. the auxiliary ones
        size_t work_off;                  // four-step classes: byte offset of their work arrays
    };
    std::vector<Class> classes;
    void* dmem;        // descriptor arrays, then the queue's class table
    size_t qtab_off;   // byte offset of the class table in dmem
    int nq;            // classes in the queue
    bool use_queue;    // fused classes: one persistent launch (else one launch per class)
    int grid;          // workgroups of the queue launch
    int ncu;
    std::vector<std::pair<int, double>> tuned_queue;  // (1 queue / 0 one launch per class, ms)
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
constexpr int kRaggedLanes = kAuxStreams + 1;  // the caller's stream and the auxiliary streams

// The size classes of a plan run concurrently: the caller's stream forks to
// the device's three auxiliary streams (runtime.hpp DevLanes) through an
// event and joins them back at the end, so the short fused classes overlap
// the long multi-pass ones (one launch of a short class fills only part of
// the chip).
using Lanes = DevLanes;

// Destroys a plan that was never executed (creation failed part way).
void free_unused(impconv_ragged_plan* p)
{
    if (p->dmem) (void)hipFree(p->dmem);
    delete p;
}

// Bytes at the start of the work memory that hold the queue's counter.
constexpr size_t kQueueCtrBytes = 256;

// Class records of the queued classes in the plan's order (longest N first),
// with their item counts under the current E.
std::vector<QueueClass> queue_table(const impconv_ragged_plan* p, int64_t* nitems)
{
    std::vector<QueueClass> t;
    int64_t items = 0;
    for (const auto& c : p->classes) {
        if (!c.queued) continue;
        const int64_t per = queue_pairs(int(c.N), c.E);
        items += (c.count + per - 1) / per;
        t.push_back({c.d_off, c.d_m, c.count, c.maxm, items, int32_t(c.N), int32_t(c.E)});
    }
    if (nitems) *nitems = items;
    return t;
}

// Copies the class table to the device (synchronous: at creation and after
// autotuning, outside any capture) and sizes the queue launch.
hipError_t upload_queue_table(impconv_ragged_plan* p)
{
    int64_t items = 0;
    const std::vector<QueueClass> t = queue_table(p, &items);
    p->grid = int(std::max<int64_t>(1, std::min<int64_t>(items, p->ncu)));
    if (t.empty()) return hipSuccess;
    return hipMemcpy(static_cast<char*>(p->dmem) + p->qtab_off, t.data(), t.size() * sizeof(QueueClass),
                     hipMemcpyHostToDevice);
}

// Stream lanes: with the queue, its launch (all queued classes) on lane 0;
// every other class, longest first, on the lane with the least estimated
// work (pairs x N log N, x3 for the three four-step passes).
void assign_lanes(impconv_ragged_plan* p)
{
    double load[kRaggedLanes] = {0, 0, 0, 0};
    auto cost = [](const impconv_ragged_plan::Class& c) {
        return double(c.count) * double(c.N) * std::log2(double(c.N) + 1.0) * (c.N > kRowMax ? 3.0 : 1.0);
    };
    const bool q = p->use_queue && p->nq > 0;
    if (q)
        for (auto& c : p->classes)
            if (c.queued) {
                c.lane = 0;
                load[0] += cost(c);
            }
    for (auto& c : p->classes) {
        if (q && c.queued) continue;
        int lane = 0;
        for (int l = 1; l < kRaggedLanes; ++l)
            if (load[l] < load[lane]) lane = l;
        c.lane = lane;
        load[lane] += cost(c);
    }
}

// The fused classes as one queue launch (queue = true) or one launch per
// class, all on stream s; the four-step classes are not touched.
impconv_status run_fused(const impconv_ragged_plan* p, const DevTables& tb, const RowArgs& base, bool queue,
                         const QueueClass* qtab, unsigned* ctr, int grid, hipStream_t s)
{
    if (queue) {
        const hipError_t e = launch_row_queue(p->dt, base, qtab, p->nq, ctr, grid, s);
        return e == hipSuccess ? IMPCONV_OK : hip_fail(e, "ragged queue launch");
    }
    for (const auto& c : p->classes) {
        if (!c.queued) continue;
        RowArgs a = base;
        a.nrows = c.count;
        a.m = c.maxm;
        a.row_off = c.d_off;
        a.row_m = c.d_m;
        const hipError_t e = launch_row_complex(p->dt, int(c.N), a, s);
        if (e != hipSuccess) return hip_fail(e, "ragged row class");
    }
    return IMPCONV_OK;
}

RowArgs ragged_row_args(const DevTables& tb, int dt, const void* f, const void* g, void* h, uint32_t flags)
{
    RowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tw = tb.tw[dt];
    a.tw3 = tb.tw3[dt];
    a.f = f;
    a.g = g;
    a.h = h;
    a.M = 1;
    a.flags = flags & (kRevF | kConjG | kRevOut);
    return a;
}
}  // namespace

namespace impconv {
namespace {
std::mutex g_lanes_mu;
DevLanes* g_lanes[64];
}  // namespace

DevLanes* device_lanes(int dev)
{
    if (dev < 0 || dev >= 64) {
        hip_fail(hipErrorInvalidDevice, "auxiliary streams");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_lanes_mu);
    if (g_lanes[dev]) return g_lanes[dev];
    auto* L = new DevLanes();
    std::vector<hipEvent_t> evs;
    int streams = 0;
    hipError_t e = hipSuccess;
    for (int l = 0; l < kAuxStreams && e == hipSuccess; ++l) {
        e = hipStreamCreateWithFlags(&L->aux[l], hipStreamNonBlocking);
        if (e == hipSuccess) ++streams;
    }
    hipEvent_t* slots[] = {&L->fork, &L->join[0], &L->join[1], &L->join[2],
                           &L->pipe[0], &L->pipe[1], &L->pipe[2], &L->pipe[3]};
    for (hipEvent_t* ev : slots) {
        if (e != hipSuccess) break;
        e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e == hipSuccess) evs.push_back(*ev);
    }
    if (e != hipSuccess) {
        // (nothing has used them yet: safe to release)
        for (int l = 0; l < streams; ++l) (void)hipStreamDestroy(L->aux[l]);
        for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
        delete L;
        hip_fail(e, "auxiliary streams");
        return nullptr;
    }
    g_lanes[dev] = L;
    return L;
}
}  // namespace impconv

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
    // queued classes: fused, and the queue kernel runs their default E
    int nq = 0;
    for (const auto& q : pend)
        if (q.N <= kRowMax && queue_supports(dtype, int(q.N), queue_default_E(dtype, int(q.N)))) ++nq;
    // device memory: the descriptors, then the queue's class table
    const size_t desc_bytes = host.size() * sizeof(int64_t);
    p->qtab_off = (desc_bytes + 15) / 16 * 16;
    const size_t dbytes = p->qtab_off + size_t(nq) * sizeof(QueueClass);
    if (dbytes > 0) {
        hipError_t e = hipMalloc(&p->dmem, dbytes);
        if (e == hipSuccess && desc_bytes)
            e = hipMemcpy(p->dmem, host.data(), desc_bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (p->dmem) (void)hipFree(p->dmem);
            delete p;
            return hip_fail(e, "ragged descriptor upload");
        }
    }
    const int64_t* d = static_cast<const int64_t*>(p->dmem);
    // the queue's counter at the start of the work memory; the four-step
    // classes get work arrays of their own after it, since classes on
    // different lanes run at the same time
    p->work = nq > 0 ? kQueueCtrBytes : 0;
    for (const auto& q : pend) {
        size_t off = 0;
        if (q.N > kRowMax) {
            off = p->work;
            p->work += size_t(4) * q.count * q.N * cs;
        }
        const bool queued = q.N <= kRowMax && queue_supports(dtype, int(q.N), queue_default_E(dtype, int(q.N)));
        p->classes.push_back({q.N, q.count, q.maxm, d + q.off_at, d + q.m_at, 0,
                              q.N <= kRowMax ? queue_default_E(dtype, int(q.N)) : 0, queued, {}, "default", 0, off});
    }
    p->nq = nq;
    p->use_queue = nq > 0;
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || ncu < 1)
            ncu = 256;
        p->ncu = ncu;
    }
    assign_lanes(p);
    {
        const hipError_t e = upload_queue_table(p);
        if (e != hipSuccess) {
            free_unused(p);
            return hip_fail(e, "ragged queue table upload");
        }
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
    if (reinterpret_cast<uintptr_t>(work) % 16) return fail(IMPCONV_E_ALIGN, "work misaligned (16 bytes)");
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
    const bool queue = p->use_queue && p->nq > 0;
    if (queue) {
        // every queued class in one persistent launch, on lane 0
        st = run_fused(p, *tb, ragged_row_args(*tb, p->dt, f, g, h, flags), true,
                       reinterpret_cast<const QueueClass*>(static_cast<const char*>(p->dmem) + p->qtab_off),
                       static_cast<unsigned*>(work), p->grid, s);
    }
    for (const auto& c : p->classes) {
        if (st) break;
        if (queue && c.queued) continue;
        hipStream_t cs_ = one || c.lane == 0 ? s : L->aux[c.lane - 1];
        if (c.N <= kRowMax) {
            RowArgs a = ragged_row_args(*tb, p->dt, f, g, h, flags);
            a.nrows = c.count;
            a.m = c.maxm;
            a.row_off = c.d_off;
            a.row_m = c.d_m;
            const hipError_t e = launch_row_complex(p->dt, int(c.N), a, cs_);
            if (e != hipSuccess) st = hip_fail(e, "ragged row class");
        } else {
            st = large1d_run_ragged(*tb, p->dt, c.count, c.N, c.maxm, f, g, h,
                                    static_cast<char*>(work) + c.work_off, c.d_off, c.d_m, flags, cs_, c.n2);
        }
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
    if (p->classes.empty()) return IMPCONV_OK;
    const DevTables* tb = tables();
    if (!tb) return IMPCONV_E_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t cs = p->dt ? 16 : 8;
    const size_t bytes = size_t(p->extent) * cs;
    const std::string arch = device_arch();
    void *f = nullptr, *g = nullptr, *h = nullptr, *w = nullptr, *qt = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    impconv_status st = IMPCONV_OK;
    auto cleanup = [&]() {
        // kernels already launched on s may still use the arrays (also
        // after a failure part way): wait for them before freeing
        (void)hipStreamSynchronize(s);
        for (void* q : {f, g, h, w, qt})
            if (q) (void)hipFree(q);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t e = hipMalloc(&f, bytes);
    if (e == hipSuccess) e = hipMalloc(&g, bytes);
    if (e == hipSuccess) e = hipMalloc(&h, bytes);
    if (e == hipSuccess) e = hipMalloc(&w, std::max<size_t>(p->work, 256));
    if (e == hipSuccess) e = hipMalloc(&qt, sizeof(QueueClass));
    if (e == hipSuccess) e = hipMemsetAsync(f, 0, bytes, s);
    if (e == hipSuccess) e = hipMemsetAsync(g, 0, bytes, s);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "autotune buffers");
    }
    // mean time of `reps` runs of fn after one untimed run
    auto time_ms = [&](auto&& fn, double* ms_out) -> impconv_status {
        constexpr int reps = 3;
        for (int r = 0; r <= reps; ++r) {
            if (r == 1 && (e = hipEventRecord(e0, s)) != hipSuccess) return hip_fail(e, "autotune event");
            impconv_status q = fn();
            if (q) return q;
        }
        float ms = 0;
        if ((e = hipEventRecord(e1, s)) != hipSuccess) return hip_fail(e, "autotune event");
        if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "autotune sync");
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return hip_fail(e, "autotune timing");
        *ms_out = double(ms) / reps;
        return IMPCONV_OK;
    };
    const RowArgs base = ragged_row_args(*tb, p->dt, f, g, h, 0);
    unsigned* ctr = static_cast<unsigned*>(w);
    for (auto& c : p->classes) {
        if (st) break;
        if (c.N > kRowMax) {
            // four-step class: the split N = N1 x N2
            int64_t n2 = 0;
            if (sched_lookup(arch, "fourstep", p->dt, c.N, &n2, nullptr)) {
                c.n2 = n2;
                c.source = "cache";
                continue;
            }
            c.tuned.clear();
            double best = 1e30;
            int64_t best_n2 = 0;
            for (int64_t cand : fourstep_splits(c.N)) {
                double t = 0;
                st = time_ms([&]() {
                    return large1d_run_ragged(*tb, p->dt, c.count, c.N, c.maxm, f, g, h,
                                              static_cast<char*>(w) + c.work_off, c.d_off, c.d_m, 0, s, cand);
                }, &t);
                if (st) break;
                c.tuned.push_back({cand, t});
                if (t < best) {
                    best = t;
                    best_n2 = cand;
                }
            }
            if (st) break;
            c.n2 = best_n2;
            c.source = "timed";
            sched_store(arch, "fourstep", p->dt, c.N, best_n2, best);
        } else if (c.queued) {
            // fused class in the queue: values per thread (radix schedule,
            // pairs per item), timed as a queue of this class alone
            int64_t E = 0;
            if (sched_lookup(arch, "fused", p->dt, c.N, &E, nullptr) && queue_supports(p->dt, int(c.N), int(E))) {
                c.E = int(E);
                c.source = "cache";
                continue;
            }
            c.tuned.clear();
            const int e0c = queue_default_E(p->dt, int(c.N));
            double best = 1e30;
            int best_E = e0c;
            for (int cand : {e0c, e0c / 2}) {
                if (!queue_supports(p->dt, int(c.N), cand)) continue;
                const int64_t per = queue_pairs(int(c.N), cand);
                const int64_t items = (c.count + per - 1) / per;
                const QueueClass one{c.d_off, c.d_m, c.count, c.maxm, items, int32_t(c.N), int32_t(cand)};
                if ((e = hipMemcpy(qt, &one, sizeof(one), hipMemcpyHostToDevice)) != hipSuccess) {
                    st = hip_fail(e, "autotune queue table");
                    break;
                }
                const int grid = int(std::max<int64_t>(1, std::min<int64_t>(items, p->ncu)));
                double t = 0;
                st = time_ms([&]() {
                    const hipError_t le = launch_row_queue(p->dt, base, static_cast<const QueueClass*>(qt), 1, ctr,
                                                           grid, s);
                    return le == hipSuccess ? IMPCONV_OK : hip_fail(le, "ragged queue launch");
                }, &t);
                if (st) break;
                c.tuned.push_back({cand, t});
                if (t < best) {
                    best = t;
                    best_E = cand;
                }
            }
            if (st) break;
            c.E = best_E;
            c.source = "timed";
            sched_store(arch, "fused", p->dt, c.N, best_E, best);
        }
    }
    // the fused classes as one queue launch against one launch per class
    if (!st && p->nq > 0) {
        if ((e = upload_queue_table(p)) != hipSuccess) st = hip_fail(e, "ragged queue table upload");
        p->tuned_queue.clear();
        double tq = 0, tl = 0;
        const QueueClass* qtab = reinterpret_cast<const QueueClass*>(static_cast<const char*>(p->dmem) + p->qtab_off);
        if (!st) st = time_ms([&]() { return run_fused(p, *tb, base, true, qtab, ctr, p->grid, s); }, &tq);
        if (!st) st = time_ms([&]() { return run_fused(p, *tb, base, false, qtab, ctr, p->grid, s); }, &tl);
        if (!st) {
            p->tuned_queue = {{1, tq}, {0, tl}};
            p->use_queue = tq <= tl;
        }
    }
    assign_lanes(p);
    cleanup();
    return st;
}

impconv_status impconv_ragged_plan_set_fused(impconv_ragged_plan* p, int queue, int elems)
{
    if (!p) return fail(IMPCONV_E_ARG, "plan is NULL");
    if (queue != 0 && queue != 1) return fail(IMPCONV_E_ARG, "queue must be 0 or 1");
    if (elems < 0) return fail(IMPCONV_E_ARG, "elems must be >= 0");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != p->device) return fail(IMPCONV_E_ARG, "plan was created on another device");
    std::lock_guard<std::mutex> lk(p->mu);
    for (auto& c : p->classes) {
        if (!c.queued) continue;
        const int e = elems ? elems : queue_default_E(p->dt, int(c.N));
        if (queue_supports(p->dt, int(c.N), e)) {
            c.E = e;
            c.source = "set";
        }
    }
    p->use_queue = queue == 1 && p->nq > 0;
    assign_lanes(p);
    const hipError_t e = upload_queue_table(p);
    return e == hipSuccess ? IMPCONV_OK : hip_fail(e, "ragged queue table upload");
}

impconv_status impconv_ragged_plan_schedule(const impconv_ragged_plan* p, char* buf, size_t cap, size_t* len)
{
    if (!p || !len) return fail(IMPCONV_E_ARG, "null argument");
    const bool queue = p->use_queue && p->nq > 0;
    std::string js = std::string("{\"fused_launch\":\"") + (queue ? "queue" : "per-class") + "\"";
    if (queue) js += ",\"queue_grid\":" + std::to_string(p->grid);
    if (!p->tuned_queue.empty()) {
        char t[128];
        std::snprintf(t, sizeof(t), ",\"fused_tuned_ms\":{\"queue\":%.5f,\"per-class\":%.5f}",
                      p->tuned_queue[0].second, p->tuned_queue[1].second);
        js += t;
    }
    js += ",\"classes\":[";
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
        const char* method = c.N > kRowMax ? "four-step" : (queue && c.queued ? "queue" : "fused");
        js += (i ? "," : "") + std::string("{\"N\":") + std::to_string(c.N) + ",\"pairs\":" + std::to_string(c.count) +
              ",\"method\":\"" + method + "\"" + ",\"stream\":" + std::to_string(c.lane) +
              ",\"source\":\"" + c.source + "\"";
        if (c.N > kRowMax) js += ",\"N1\":" + std::to_string(N1) + ",\"N2\":" + std::to_string(N2);
        else js += ",\"E\":" + std::to_string(c.E);
        if (!c.tuned.empty()) {
            js += ",\"tuned_ms\":{";
            for (size_t j = 0; j < c.tuned.size(); ++j) {
                char t[64];
                std::snprintf(t, sizeof(t), "%s\"%lld\":%.5f", j ? "," : "", (long long)c.tuned[j].first, c.tuned[j].second);
                js += t;
            }
            js += "}";
        }
        js += "}";
    }
    js += "]}";
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
