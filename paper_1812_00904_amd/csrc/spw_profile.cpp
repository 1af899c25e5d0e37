// Optional per-kernel timing: HIP events recorded on the launch stream around
// every kernel the library launches, folded per kernel name on read.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "spw_internal.h"

namespace spw {
namespace {

struct Rec {
    const char *name;
    hipEvent_t start, stop;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::string g_select;          // time only kernels whose name begins with this (empty: all)
std::vector<Rec> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<int64_t, double>> g_totals;

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

void fold_pending_locked()
{
    for (Rec &r : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            auto &t = g_totals[r.name];
            t.first += 1;
            t.second += (double)ms;
        }
        g_pool.push_back(r.start);
        g_pool.push_back(r.stop);
    }
    g_pending.clear();
}

}  // namespace

bool profile_on() { return g_on.load(std::memory_order_relaxed); }

void profile_begin(void *stream, const char *name, void **token)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_select.empty() && std::strncmp(name, g_select.c_str(), g_select.size()) != 0) {
        *token = nullptr;
        return;
    }
    Rec *r = new Rec{name, take_event(), take_event()};
    if (!r->start || !r->stop) {
        delete r;
        *token = nullptr;
        return;
    }
    (void)hipEventRecord(r->start, (hipStream_t)stream);
    *token = r;
}

void profile_end(void *stream, void *token)
{
    Rec *r = (Rec *)token;
    (void)hipEventRecord(r->stop, (hipStream_t)stream);
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back(*r);
    delete r;
    if (g_pending.size() > 4096) fold_pending_locked();
}

}  // namespace spw

extern "C" {

static spw_status spw_profile_enable_impl(int32_t on)
{
    spw::g_on.store(on != 0);
    return SPW_OK;
}

spw_status spw_profile_enable(int32_t on)
{
    return spw::guarded("spw_profile_enable", [&] { return spw_profile_enable_impl(on); });
}

static spw_status spw_profile_select_impl(const char *prefix)
{
    std::lock_guard<std::mutex> lk(spw::g_mu);
    spw::g_select = prefix ? prefix : "";
    return SPW_OK;
}

spw_status spw_profile_select(const char *prefix)
{
    return spw::guarded("spw_profile_select", [&] { return spw_profile_select_impl(prefix); });
}

static spw_status spw_profile_reset_impl(void)
{
    std::lock_guard<std::mutex> lk(spw::g_mu);
    spw::fold_pending_locked();
    spw::g_totals.clear();
    return SPW_OK;
}

spw_status spw_profile_reset(void)
{
    return spw::guarded("spw_profile_reset", [&] { return spw_profile_reset_impl(); });
}

static spw_status spw_profile_read_impl(spw_profile_entry *entries, int32_t cap, int32_t *count)
{
    if (!count || (cap > 0 && !entries)) {
        spw::set_error("spw_profile_read: NULL count, or NULL entries with cap > 0");
        return SPW_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(spw::g_mu);
    spw::fold_pending_locked();
    int32_t i = 0;
    for (auto &kv : spw::g_totals) {
        if (i < cap) {
            std::memset(entries[i].name, 0, sizeof(entries[i].name));
            std::strncpy(entries[i].name, kv.first.c_str(), sizeof(entries[i].name) - 1);
            entries[i].launches = kv.second.first;
            entries[i].total_ms = kv.second.second;
        }
        ++i;
    }
    *count = i;
    return SPW_OK;
}

spw_status spw_profile_read(spw_profile_entry *entries, int32_t cap, int32_t *count)
{
    return spw::guarded("spw_profile_read", [&] { return spw_profile_read_impl(entries, cap, count); });
}

}  // extern "C"
