// Opt-in per-stage timing with HIP events on the launching stream.  Off by
// default; when on, each scope records an event pair around its launches and
// pm4g_profile_read() folds the elapsed times per stage.
#pragma once

#include <hip/hip_runtime.h>

namespace pm4g {

enum ProfId {
    P_RANGE = 0,
    P_RADIX_HIST,
    P_RADIX_SCAN,
    P_RADIX_SCATTER,
    P_SEGSORT,
    P_CASE_TABLE,
    P_DFG_MAIN,
    P_DFG_PLAN,
    P_DFG_AGG,
    P_DFG_REDUCE,
    P_VAR_HASH,
    P_VAR_SORT,
    P_VAR_GROUP,
    P_VAR_ORDER,
    P_VAR_EMIT,
    P_VIEW_PLAN,
    P_VIEW_EMIT,
    P_VIEW_PLACE,
    P_VIEW_AGG,
    P_VIEW_OUT,
    P_VIEW_FILTER,
    P_DFG_COUNT,
    P_VIEW_WRITE,
    P_CASES,
    P_CASE_FILTER,
    P_DF_FILTER,
    P_EFG,
    P_SAMPLE,
    P_CSV,
    P_PARQUET,
    P_VIEW_FUSED,
    P_COUNT
};

const char* prof_name(int id);
bool prof_on();
void prof_record(int id, hipEvent_t a, hipEvent_t b);
hipEvent_t prof_event();

struct ProfScope {
    int id;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(int id_, hipStream_t s_) : id(id_), s(s_) {
        if (prof_on()) {
            a = prof_event();
            (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope() {
        if (a) {
            hipEvent_t b = prof_event();
            (void)hipEventRecord(b, s);
            prof_record(id, a, b);
        }
    }
};

}  // namespace pm4g
