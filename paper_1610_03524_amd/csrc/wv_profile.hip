// wv_profile.hip -- optional per-kernel timing of the builds.
//
// When a build runs with WT_FLAG_PROFILE, every instrumented launch is
// bracketed by two HIP events recorded on the build's stream; the events are
// read (and the totals reset) by wt_profile_read().  Events come from a pool
// that only grows while profiling is used.
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "wv_internal.h"

namespace {

struct Pending {
    std::string name;
    hipEvent_t a, b;
};

struct Totals {
    uint64_t launches = 0;
    double ms = 0;
};

std::mutex g_mu;
std::vector<hipEvent_t> g_pool;
std::vector<Pending> g_pending;
std::map<std::string, Totals> g_totals;

hipEvent_t take_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

int wv_prof_before(hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Pending p;
    p.a = take_event();
    p.b = take_event();
    if (!p.a || !p.b) return -1;
    if (hipEventRecord(p.a, s) != hipSuccess) return -1;
    g_pending.push_back(p);
    return (int)g_pending.size() - 1;
}

void wv_prof_after(int slot, hipStream_t s, const char* name)
{
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending[slot].name = name;
    (void)hipEventRecord(g_pending[slot].b, s);   // a failed record shows as a missing entry
}

extern "C" int wt_profile_read(wt_profile_entry* out, uint32_t cap, uint32_t* count)
{
    if (!count || (cap && !out)) return WT_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    for (Pending& p : g_pending) {
        if (hipEventSynchronize(p.b) != hipSuccess) return WT_EHIP;
        float ms = 0;
        if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) return WT_EHIP;
        Totals& t = g_totals[p.name];
        t.launches++;
        t.ms += ms;
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
    uint32_t k = 0;
    for (auto& kv : g_totals) {
        if (k < cap) {
            std::memset(&out[k], 0, sizeof(out[k]));
            std::strncpy(out[k].name, kv.first.c_str(), sizeof(out[k].name) - 1);
            out[k].launches = kv.second.launches;
            out[k].ms = kv.second.ms;
        }
        k++;
    }
    *count = k;
    g_totals.clear();
    return WT_OK;
}
