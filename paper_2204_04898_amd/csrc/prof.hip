// Stage timing pool behind pm4g_profile_enable / pm4g_profile_read.
#include <mutex>
#include <vector>

#include "../../include/pm4g.h"
#include "prof.hpp"

namespace pm4g {
namespace {

const char* kNames[P_COUNT] = {
    "range_scan",   "radix_hist", "radix_scan", "radix_scatter", "segsort",
    "case_table",   "dfg_main",   "dfg_plan",   "dfg_agg",       "dfg_reduce",
    "variant_hash", "variant_sort", "variant_group", "variant_order", "variant_emit",
    "view_plan",    "view_emit",  "view_place",  "view_agg",      "view_out",
    "view_filter",  "dfg_count",  "view_write", "cases",         "case_filter",
    "df_filter",    "efg",        "sample",        "csv",          "parquet",
    "view_fused"};

struct Rec {
    int id;
    hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_free;

}  // namespace

const char* prof_name(int id) { return (id >= 0 && id < P_COUNT) ? kNames[id] : "unknown"; }

bool prof_on() { return g_on; }

hipEvent_t prof_event() {
    std::lock_guard<std::mutex> l(g_mu);
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void prof_record(int id, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> l(g_mu);
    g_recs.push_back(Rec{id, a, b});
}

}  // namespace pm4g

extern "C" {

int pm4g_profile_enable(int on) {
    const int old = pm4g::g_on ? 1 : 0;
    pm4g::g_on = on != 0;
    return old;
}

int pm4g_profile_read(double* total_ms, int64_t* launches, int n_stages) {
    using namespace pm4g;
    std::vector<Rec> recs;
    {
        std::lock_guard<std::mutex> l(g_mu);
        recs.swap(g_recs);
    }
    for (int i = 0; i < n_stages; ++i) {
        if (total_ms) total_ms[i] = 0.0;
        if (launches) launches[i] = 0;
    }
    int rc = PM4G_OK;
    for (const Rec& r : recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) rc = PM4G_E_DEVICE;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) rc = PM4G_E_DEVICE;
        if (r.id < n_stages) {
            if (total_ms) total_ms[r.id] += ms;
            if (launches) launches[r.id] += 1;
        }
    }
    std::lock_guard<std::mutex> l(g_mu);
    for (const Rec& r : recs) {
        g_free.push_back(r.a);
        g_free.push_back(r.b);
    }
    return rc;
}

const char* pm4g_profile_stage_name(int stage) { return pm4g::prof_name(stage); }

int pm4g_profile_stage_count(void) { return pm4g::P_COUNT; }

}  // extern "C"
