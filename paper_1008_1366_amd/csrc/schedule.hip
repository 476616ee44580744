// schedule.hip -- process-wide cache of autotuned schedules.
//
// The autotuner of ragged plans (ragged.hip) times the candidate schedules
// of each size class and records the winner here, keyed by (device
// architecture, variant, dtype, FFT size N):
//   variant "fused":    values per thread E of the fused row code in the
//                       persistent work queue;
//   variant "fourstep": column length N2 of the split N = N1 x N2 of the
//                       three-pass form.
// A later plan with a class of the same key takes the recorded choice
// without timing it again.  The cache can be exported as JSON and imported
// (merged) in another process, so that the timing is paid once per machine.
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "runtime.hpp"
#include "schedule.hpp"

namespace impconv {
namespace {
using Key = std::tuple<std::string, std::string, int, int64_t>;  // arch, variant, dtype, N
struct Val {
    int64_t choice;
    double ms;
};
std::mutex s_mu;
std::map<Key, Val> s_cache;

// "key": value pairs of one flat JSON object (strings or numbers)
bool parse_object(const char* p, const char* end, std::map<std::string, std::string>* kv)
{
    while (p < end) {
        while (p < end && *p != '"') ++p;
        if (p >= end) break;
        const char* k0 = ++p;
        while (p < end && *p != '"') ++p;
        if (p >= end) return false;
        std::string key(k0, p - k0);
        ++p;
        while (p < end && (std::isspace((unsigned char)*p) || *p == ':')) ++p;
        if (p >= end) return false;
        std::string val;
        if (*p == '"') {
            const char* v0 = ++p;
            while (p < end && *p != '"') ++p;
            if (p >= end) return false;
            val.assign(v0, p - v0);
            ++p;
        } else {
            const char* v0 = p;
            while (p < end && *p != ',' && *p != '}' && !std::isspace((unsigned char)*p)) ++p;
            val.assign(v0, p - v0);
        }
        (*kv)[key] = val;
    }
    return true;
}
}  // namespace

std::string device_arch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

bool sched_lookup(const std::string& arch, const char* variant, int dt, int64_t N, int64_t* choice, double* ms)
{
    std::lock_guard<std::mutex> lk(s_mu);
    auto it = s_cache.find(Key{arch, variant, dt, N});
    if (it == s_cache.end()) return false;
    *choice = it->second.choice;
    if (ms) *ms = it->second.ms;
    return true;
}

void sched_store(const std::string& arch, const char* variant, int dt, int64_t N, int64_t choice, double ms)
{
    std::lock_guard<std::mutex> lk(s_mu);
    s_cache[Key{arch, variant, dt, N}] = Val{choice, ms};
}

}  // namespace impconv

using namespace impconv;

extern "C" {

impconv_status impconv_schedule_cache_export(char* buf, size_t cap, size_t* len)
{
    if (!len) return fail(IMPCONV_E_ARG, "len is NULL");
    std::string js = "[";
    {
        std::lock_guard<std::mutex> lk(s_mu);
        bool first = true;
        for (const auto& kv : s_cache) {
            char t[384];
            std::snprintf(t, sizeof(t),
                          "%s{\"arch\": \"%s\", \"variant\": \"%s\", \"dtype\": \"%s\", \"N\": %lld, \"choice\": %lld, "
                          "\"ms\": %.6f}",
                          first ? "" : ", ", std::get<0>(kv.first).c_str(), std::get<1>(kv.first).c_str(),
                          std::get<2>(kv.first) ? "c128" : "c64", (long long)std::get<3>(kv.first),
                          (long long)kv.second.choice, kv.second.ms);
            js += t;
            first = false;
        }
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

impconv_status impconv_schedule_cache_import(const char* json)
{
    if (!json) return fail(IMPCONV_E_ARG, "json is NULL");
    const char* p = json;
    const char* end = json + std::strlen(json);
    struct Entry {
        Key k;
        Val v;
    };
    std::vector<Entry> got;
    while (p < end) {
        const char* o = std::strchr(p, '{');
        if (!o) break;
        const char* c = std::strchr(o, '}');
        if (!c) return fail(IMPCONV_E_ARG, "schedule cache: unterminated object");
        std::map<std::string, std::string> kv;
        if (!parse_object(o + 1, c, &kv)) return fail(IMPCONV_E_ARG, "schedule cache: malformed object");
        for (const char* f : {"arch", "variant", "dtype", "N", "choice"})
            if (!kv.count(f)) return fail(IMPCONV_E_ARG, std::string("schedule cache: entry without \"") + f + "\"");
        const std::string& var = kv["variant"];
        if (var != "fused" && var != "fourstep") return fail(IMPCONV_E_ARG, "schedule cache: unknown variant " + var);
        const std::string& d = kv["dtype"];
        if (d != "c64" && d != "c128") return fail(IMPCONV_E_ARG, "schedule cache: unknown dtype " + d);
        char* e1 = nullptr;
        char* e2 = nullptr;
        const long long N = std::strtoll(kv["N"].c_str(), &e1, 10);
        const long long ch = std::strtoll(kv["choice"].c_str(), &e2, 10);
        if (*e1 || *e2 || N < 1 || ch < 1) return fail(IMPCONV_E_ARG, "schedule cache: bad N or choice");
        const double ms = kv.count("ms") ? std::strtod(kv["ms"].c_str(), nullptr) : 0.0;
        got.push_back({Key{kv["arch"], var, d == "c128" ? 1 : 0, N}, Val{ch, ms}});
        p = c + 1;
    }
    // all entries parsed: merge them (a malformed input changes nothing)
    std::lock_guard<std::mutex> lk(s_mu);
    for (const auto& e : got) s_cache[e.k] = e.v;
    return IMPCONV_OK;
}

impconv_status impconv_schedule_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(s_mu);
    s_cache.clear();
    return IMPCONV_OK;
}

}  // extern "C"
