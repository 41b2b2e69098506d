// C ABI of libpm4g (declared in include/pm4g.h): argument validation,
// workspace layout, kernel sequencing and error reporting.  Host code only;
// every step of the computation runs in the kernels of the other files.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "../../include/pm4g.h"
#include "internal.hpp"
#include "prof.hpp"

using namespace pm4g;

namespace {

thread_local char g_err[512] = "";
thread_local int g_variant_hash_bits = 0;   // test hook, 0 = full 64-bit hash
thread_local int64_t g_efg_pass_pairs = 0;  // test hook, 0 = the EFG's full LDS pass length
thread_local int g_csv_hash_bits = 0;       // test hook, 0 = full 64-bit value hashes

void set_err(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

#define PM4G_HIP(x)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) {                                                            \
            set_err("%s failed: %s (%s:%d)", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
            return PM4G_E_DEVICE;                                                          \
        }                                                                                  \
    } while (0)

#define PM4G_CHECK(cond, ...)        \
    do {                             \
        if (!(cond)) {               \
            set_err(__VA_ARGS__);    \
            return PM4G_E_INVALID;   \
        }                            \
    } while (0)

constexpr int64_t kMaxEvents = (int64_t(1) << 31) - 1;

__global__ void k_set_status(int32_t* status, int32_t code) { *status = code; }
struct BatchedTune {
    int tile, emit_blocks, agg_blocks, launch;
    int64_t pair_cap, rec_cap, cell_cap;
};

int resolve_tuning(const pm4g_batched_tuning* t, int64_t n, int32_t V, BatchedTune* r) {
    if (t && t->tile_events != 0 && t->tile_events != 2048 && t->tile_events != 4096) {
        set_err("tile_events must be 2048 or 4096 (0: default)");
        return PM4G_E_INVALID;
    }
    if (t && (t->emit_blocks < 0 || t->agg_blocks < 0 || t->emit_blocks > 65535 || t->agg_blocks > 65535 ||
              t->pair_capacity < 0 || t->record_capacity < 0 || t->descriptor_capacity < 0 ||
              t->cell_capacity < 0)) {
        set_err("negative or oversized tuning field");
        return PM4G_E_INVALID;
    }
    if (t && t->launch != 0 && t->launch != 1) {
        set_err("launch must be 0 (one persistent launch) or 1 (one launch per phase)");
        return PM4G_E_INVALID;
    }
    r->launch = t ? t->launch : 0;
    r->tile = (t && t->tile_events) ? t->tile_events : 4096;
    r->emit_blocks = (t && t->emit_blocks) ? t->emit_blocks : 2048;
    r->agg_blocks = (t && t->agg_blocks) ? t->agg_blocks : 512;
    const int64_t tiles = (n + r->tile - 1) / r->tile;
    r->pair_cap = (t && t->pair_capacity) ? t->pair_capacity : 4 * (tiles + V) + 1024;
    r->rec_cap = (t && t->record_capacity) ? t->record_capacity : (n > 4096 ? n : 4096);
    r->cell_cap = (t && t->cell_capacity) ? t->cell_capacity : (r->rec_cap / 2 > 4096 ? r->rec_cap / 2 : 4096);
    if (r->pair_cap > (int64_t)0xFFFFFFF0) {
        set_err("the pair capacity must stay below 2^32");
        return PM4G_E_INVALID;
    }
    return PM4G_OK;
}

size_t batched_ws_bytes(int64_t n, int32_t A, int32_t V, const BatchedTune& t) {
    Bump b(nullptr);
    view_ws_layout(b, n, A, V, t.tile, t.pair_cap, t.rec_cap, t.cell_cap);
    return b.off + 256;
}

}  // namespace

// with_rows: pm4g_prepare's workspace has the row room; the raw-log DFG and
// variants calls do not produce the permutation.
PrepWs pm4g::prep_ws_layout(Bump& bp, int64_t n, bool with_rows) {
    PrepWs w{};
    const size_t m = (size_t)(n > 0 ? n : 1);
    w.info = bp.take<RangeInfo>(1);
    w.rpart = bp.take<RangePart>((size_t)(radix_blocks(n) > kRangeParts ? radix_blocks(n) : kRangeParts));
    w.a.key = bp.take<uint32_t>(m);
    w.a.ts = bp.take<int64_t>(m);
    w.a.act = bp.take<uint32_t>(m);
    w.b.key = bp.take<uint32_t>(m);
    w.b.ts = bp.take<int64_t>(m);
    w.b.act = bp.take<uint32_t>(m);
    w.a.row = with_rows ? bp.take<uint32_t>(m) : nullptr;
    w.b.row = with_rows ? bp.take<uint32_t>(m) : nullptr;
    w.hist = bp.take<uint32_t>(256 * (size_t)(radix_blocks(n) + 1));
    w.hist_raw = bp.take<uint32_t>(256 * (size_t)(radix_blocks(n) + 1));
    w.rowsum = bp.take<uint32_t>(256);
    w.caseblk = bp.take<uint32_t>((size_t)case_blocks(n) + 1);
    w.wincnt = bp.take<uint32_t>((size_t)segsort_blocks(n) + 1);
    return w;
}

namespace {

// Prepared-log arrays carved out of a workspace (raw-log entry points).
pm4g_prepared prepared_in_ws(Bump& bp, int64_t n, int32_t A) {
    pm4g_prepared p{};
    const size_t m = (size_t)(n > 0 ? n : 1);
    p.case_s = bp.take<int32_t>(m);
    p.act_s = bp.take<int32_t>(m);
    p.ts_s = bp.take<int64_t>(m);
    p.case_off = bp.take<int64_t>(m + 1);
    p.case_code = bp.take<int32_t>(m);
    p.n_cases = bp.take<int64_t>(1);
    p.status = bp.take<int32_t>(1);
    p.n_events = n;
    p.n_activities = A;
    return p;
}

int check_log(const pm4g_log* log) {
    PM4G_CHECK(log != nullptr, "log is NULL");
    PM4G_CHECK(log->n_events >= 0 && log->n_events <= kMaxEvents, "n_events %lld outside [0, 2^31)",
               (long long)log->n_events);
    PM4G_CHECK(log->n_activities >= 1 && log->n_activities <= PM4G_MAX_ACTIVITIES,
               "n_activities %d outside [1, %d]", log->n_activities, PM4G_MAX_ACTIVITIES);
    PM4G_CHECK((log->flags & ~(uint32_t)PM4G_PRESORTED) == 0, "unknown flags 0x%x", log->flags);
    PM4G_CHECK(log->n_events == 0 || (log->case_id && log->activity && log->timestamp),
               "a log column is NULL");
    return PM4G_OK;
}

int check_prepared(const pm4g_prepared* p, bool need_case_table) {
    PM4G_CHECK(p != nullptr, "prepared log is NULL");
    PM4G_CHECK(p->n_events >= 0 && p->n_events <= kMaxEvents, "n_events %lld outside [0, 2^31)",
               (long long)p->n_events);
    PM4G_CHECK(p->n_activities >= 1 && p->n_activities <= PM4G_MAX_ACTIVITIES,
               "n_activities %d outside [1, %d]", p->n_activities, PM4G_MAX_ACTIVITIES);
    PM4G_CHECK(p->n_events == 0 || (p->case_s && p->act_s && p->ts_s), "a prepared column is NULL");
    if (need_case_table)
        PM4G_CHECK(p->case_off && p->n_cases && (p->n_events == 0 || p->case_code),
                   "the prepared case table is NULL");
    return PM4G_OK;
}

int bits_of(uint64_t range) {
    int b = 0;
    while (b < 64 && (range >> b) != 0) ++b;
    return b;
}

// Formatting step into `out` (caller's arrays or workspace arrays).  With
// ws_rows the workspace has room for the row order, and out->row (if not
// NULL) receives the original row of each position.
int run_prepare(const pm4g_log* log, const pm4g_prepared* out, bool case_table, Bump& bp,
                hipStream_t s, bool ws_rows = false) {
    const int64_t n = log->n_events;
    const int32_t A = log->n_activities;
    const bool presorted = (log->flags & PM4G_PRESORTED) != 0;
    PrepWs w = prep_ws_layout(bp, n, ws_rows);
    int32_t* const row_s = ws_rows ? out->row : nullptr;
    if (!row_s) w.a.row = w.b.row = nullptr;   // the row order is carried only when asked for
    k_set_status<<<1, 1, 0, s>>>(out->status, 0);
    PM4G_HIP(launch_range_scan(log->case_id, log->activity, log->timestamp, n, A, presorted, false,
                               w.info, w.rpart, presorted ? nullptr : w.hist_raw, s));
    RangeInfo h{};
    PM4G_HIP(hipMemcpyAsync(&h, w.info, sizeof(h), hipMemcpyDeviceToHost, s));
    PM4G_HIP(hipStreamSynchronize(s));
    if (h.status != 0) {
        k_set_status<<<1, 1, 0, s>>>(out->status, h.status);
        PM4G_HIP(hipGetLastError());
        set_err("%s", h.status == PM4G_E_RANGE ? "activity outside [0, n_activities)"
                                               : "rows are not in (case, timestamp, row) order");
        return h.status;
    }
    bool have_wincnt = false;   // the per-case sort counted the cases of each window
    if (presorted) {
        PM4G_HIP(launch_copy_log(log->case_id, log->activity, log->timestamp, n, out->case_s,
                                 out->act_s, out->ts_s, row_s, s));
    } else if (n > 0) {
        const SortBufs raw{(uint32_t*)log->case_id, (int64_t*)log->timestamp, (uint32_t*)log->activity, nullptr};
        const int case_bits = bits_of((uint64_t)(uint32_t)(h.case_max - h.case_min));
        const int act_bits = bits_of((uint64_t)(A - 1));
        // packed keys (activity above the case bits) when both fit in 32 bits
        const int act_shift = (case_bits > 0 && case_bits < 32 && case_bits + act_bits <= 32) ? case_bits : 0;
        int passes = (case_bits + 7) / 8;
        if (passes == 0) passes = 1;   // a single case: one pass still biases the keys
        SortBufs bufs[2] = {w.a, w.b};
        SortBufs in = raw;
        int cur = 0;
        for (int p = 0; p < passes; ++p) {
            PM4G_HIP(launch_radix_pass(in, bufs[cur], n, 0, 8 * p, p == 0, w.info, w.hist, w.rowsum, act_shift,
                                       p == 0 ? w.hist_raw : nullptr, s));
            in = bufs[cur];
            cur ^= 1;
        }
        PM4G_HIP(launch_segsort(in, n, w.info, out->case_s, out->act_s, out->ts_s, act_shift, w.wincnt, row_s, s));
        PM4G_HIP(hipMemcpyAsync(&h, w.info, sizeof(h), hipMemcpyDeviceToHost, s));
        PM4G_HIP(hipStreamSynchronize(s));
        have_wincnt = !h.long_case;
        if (h.long_case) {
            // Full-key fallback: stable passes on the timestamp bits, then the case bits.
            PM4G_HIP(launch_ts_range(log->timestamp, n, w.info, s));
            PM4G_HIP(hipMemcpyAsync(&h, w.info, sizeof(h), hipMemcpyDeviceToHost, s));
            PM4G_HIP(hipStreamSynchronize(s));
            const int ts_bits = bits_of((uint64_t)h.ts_max - (uint64_t)h.ts_min);
            const int ts_passes = (ts_bits + 7) / 8;
            in = raw;
            cur = 0;
            bool first = true;
            for (int p = 0; p < ts_passes; ++p, first = false) {
                PM4G_HIP(launch_radix_pass(in, bufs[cur], n, 1, 8 * p, first, w.info, w.hist, w.rowsum,
                                           act_shift, nullptr, s));
                in = bufs[cur];
                cur ^= 1;
            }
            for (int p = 0; p < passes; ++p, first = false) {
                PM4G_HIP(launch_radix_pass(in, bufs[cur], n, 0, 8 * p, first, w.info, w.hist, w.rowsum,
                                           act_shift, nullptr, s));
                in = bufs[cur];
                cur ^= 1;
            }
            PM4G_HIP(launch_unbias_copy(in, n, w.info, out->case_s, out->act_s, out->ts_s, act_shift, row_s, s));
        }
    }
    if (case_table)
        PM4G_HIP(launch_case_table(out->case_s, n, w.caseblk, out->case_off, out->case_code,
                                   out->n_cases, have_wincnt ? w.wincnt : nullptr, s));
    return PM4G_OK;
}

// Library-owned workspace of pm4g_dfg_prepared_noalloc: one copy per GPU,
// held for the life of the process.  Host code never passes the array's name
// to a kernel (on the host it is a stand-in, not a device address); it uses
// the per-device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[PM4G_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on the current device, looked up once per
// device with that device current.
int scratch_of_current_device(void** ptr) {
    int dev = -1;
    PM4G_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_err("device %d outside [0, %d)", dev, kMaxDevices);
        return PM4G_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        PM4G_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_err("no device address for the scratch array on device %d", dev);
            return PM4G_E_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return PM4G_OK;
}

DfgOutDev dev_out(const pm4g_dfg_out* o) {
    return DfgOutDev{o->count, o->dt_sum, o->dt_min, o->dt_max, o->dt_mean, o->start_count,
                     o->end_count, o->act_count, o->n_cases, o->overflow, o->status};
}

int check_dfg_out(const pm4g_dfg_out* o) {
    PM4G_CHECK(o != nullptr, "dfg output is NULL");
    PM4G_CHECK(o->count && o->dt_sum && o->dt_min && o->dt_max && o->start_count && o->end_count &&
                   o->act_count && o->n_cases && o->overflow && o->status,
               "a dfg output array is NULL (only dt_mean may be NULL)");
    return PM4G_OK;
}

int check_var_out(const pm4g_variants_out* o) {
    PM4G_CHECK(o != nullptr, "variants output is NULL");
    PM4G_CHECK(o->n_variants && o->var_count && o->var_len && o->var_rep && o->var_off && o->var_acts &&
                   o->status,
               "a variants output array is NULL (only case_variant may be NULL)");
    return PM4G_OK;
}

size_t ws_bytes(int op, int64_t n, int32_t A) {
    Bump b(nullptr);
    switch (op) {
        case PM4G_OP_PREPARE:
            prep_ws_layout(b, n, true);
            break;
        case PM4G_OP_DFG_PREPARED:
            dfg_ws_layout(b, n, A);
            break;
        case PM4G_OP_DFG: {
            prepared_in_ws(b, n, A);
            Bump b2(nullptr);
            prep_ws_layout(b2, n, false);
            Bump b3(nullptr);
            dfg_ws_layout(b3, n, A);
            b.off += (b2.off > b3.off ? b2.off : b3.off) + 256;
            break;
        }
        case PM4G_OP_VARIANTS_PREPARED:
            var_ws_layout(b, n);
            break;
        case PM4G_OP_VARIANTS: {
            prepared_in_ws(b, n, A);
            Bump b2(nullptr);
            prep_ws_layout(b2, n, false);
            Bump b3(nullptr);
            var_ws_layout(b3, n);
            b.off += (b2.off > b3.off ? b2.off : b3.off) + 256;
            break;
        }
        default:
            return 0;
    }
    return b.off + 256;
}

}  // namespace

extern "C" {

int pm4g_abi_version(void) { return PM4G_ABI_VERSION; }

const char* pm4g_last_error(void) { return g_err; }

int pm4g_debug_variant_hash_bits(int bits) {
    const int old = g_variant_hash_bits;
    g_variant_hash_bits = (bits < 0 || bits >= 64) ? 0 : bits;
    return old;
}

int pm4g_debug_csv_hash_bits(int bits) {
    const int old = g_csv_hash_bits;
    g_csv_hash_bits = (bits < 0 || bits >= 64) ? 0 : bits;
    return old;
}

int64_t pm4g_debug_efg_pass_pairs(int64_t pairs) {
    const int64_t old = g_efg_pass_pairs;
    g_efg_pass_pairs = pairs > 0 ? pairs : 0;
    return old;
}

const char* pm4g_status_string(int code) {
    switch (code) {
        case PM4G_OK: return "ok";
        case PM4G_E_INVALID: return "invalid argument";
        case PM4G_E_RANGE: return "activity outside [0, n_activities)";
        case PM4G_E_NOT_SORTED: return "rows are not in (case, timestamp, row) order";
        case PM4G_E_CAPACITY: return "output capacity exceeded";
        case PM4G_E_WORKSPACE: return "workspace too small";
        case PM4G_E_DEVICE: return "HIP runtime error";
        case PM4G_E_PARSE: return "parse error";
        case PM4G_E_UNSUPPORTED: return "Parquet feature outside the covered subset";
        default: return "unknown status";
    }
}

size_t pm4g_workspace_bytes(int op, int64_t n_events, int32_t n_activities, int32_t n_views) {
    if (n_events < 0 || n_events > kMaxEvents) return 0;
    if (n_activities < 1 || n_activities > PM4G_MAX_ACTIVITIES) return 0;
    if (op == PM4G_OP_DFG_BATCHED) return pm4g_batched_workspace_bytes(n_events, n_activities, n_views, nullptr);
    return ws_bytes(op, n_events, n_activities);
}

size_t pm4g_batched_workspace_bytes(int64_t n_events, int32_t n_activities, int32_t n_views,
                                    const pm4g_batched_tuning* tuning) {
    if (n_events < 0 || n_events > kMaxEvents || n_views < 0) return 0;
    if (n_activities < 1 || n_activities > PM4G_BATCHED_MAX_ACTIVITIES) return 0;
    if ((int64_t)n_views * view_buckets(n_activities) > (int64_t)0xFFFFFFFF) return 0;
    BatchedTune t;
    if (resolve_tuning(tuning, n_events, n_views, &t) != PM4G_OK) return 0;
    return batched_ws_bytes(n_events, n_activities, n_views, t);
}

size_t pm4g_filter_workspace_bytes(int64_t n_events) {
    if (n_events < 0 || n_events > kMaxEvents) return 0;
    Bump b(nullptr);
    filter_ws_layout(b, n_events);
    return b.off + 256;
}

int pm4g_filter_view(const pm4g_prepared* log, const pm4g_view* view, const uint64_t* act_mask,
                     const pm4g_prepared* out, void* ws, size_t ws_size, void* stream) {
    if (int rc = check_prepared(log, true)) return rc;
    PM4G_CHECK(view && act_mask, "view or act_mask is NULL");
    PM4G_CHECK(out && out->case_off && out->n_cases && out->status &&
                   (log->n_events == 0 || (out->case_s && out->act_s && out->ts_s && out->case_code)),
               "a filtered-log output array is NULL");
    PM4G_CHECK(out->n_events >= 0 && out->n_activities == log->n_activities,
               "the filtered log needs a capacity >= 0 and the same n_activities");
    const size_t need = pm4g_filter_workspace_bytes(log->n_events);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    Bump bp(ws);
    FilterWs w = filter_ws_layout(bp, log->n_events);
    PM4G_HIP(launch_filter_view(log, view, act_mask, out, w, (hipStream_t)stream));
    return PM4G_OK;
}

int pm4g_filter_df_events(const pm4g_prepared* log, const uint64_t* pair_mask, int32_t side, int32_t keep,
                          const pm4g_prepared* out, void* ws, size_t ws_size, void* stream) {
    if (int rc = check_prepared(log, true)) return rc;
    PM4G_CHECK(pair_mask != nullptr, "pair_mask is NULL");
    PM4G_CHECK(side == 0 || side == 1, "side must be 0 (previous event) or 1 (next event)");
    PM4G_CHECK(keep == 0 || keep == 1, "keep must be 0 or 1");
    PM4G_CHECK(out && out->case_off && out->n_cases && out->status &&
                   (log->n_events == 0 || (out->case_s && out->act_s && out->ts_s && out->case_code)),
               "a filtered-log output array is NULL");
    PM4G_CHECK(out->n_events >= 0 && out->n_activities == log->n_activities,
               "the filtered log needs a capacity >= 0 and the same n_activities");
    const size_t need = pm4g_filter_workspace_bytes(log->n_events);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    Bump bp(ws);
    FilterWs w = filter_ws_layout(bp, log->n_events);
    PM4G_HIP(launch_filter_df_events(log, pair_mask, side, keep, out, w, (hipStream_t)stream));
    return PM4G_OK;
}

size_t pm4g_efg_workspace_bytes(int64_t n_events, int32_t n_activities) {
    if (n_events < 0 || n_events > kMaxEvents || n_activities < 1 || n_activities > PM4G_EFG_MAX_ACTIVITIES)
        return 0;
    Bump b(nullptr);
    efg_ws_layout(b, n_events, n_activities);
    return b.off + 256;
}

int pm4g_efg(const pm4g_prepared* log, const pm4g_efg_out* out, void* ws, size_t ws_size, void* stream) {
    if (int rc = check_prepared(log, true)) return rc;
    PM4G_CHECK(log->n_activities <= PM4G_EFG_MAX_ACTIVITIES, "n_activities %d above %d for the EFG",
               log->n_activities, PM4G_EFG_MAX_ACTIVITIES);
    PM4G_CHECK(out && out->count && out->sum_lo && out->sum_hi && out->sq_lo && out->sq_hi && out->n_pairs &&
                   out->status,
               "an EFG output array is NULL (only mean and std may be NULL)");
    const size_t need = pm4g_efg_workspace_bytes(log->n_events, log->n_activities);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    Bump bp(ws);
    EfgWs w = efg_ws_layout(bp, log->n_events, log->n_activities);
    const EfgOutDev o{out->count, out->sum_lo, out->sum_hi, out->sq_lo, out->sq_hi,
                      out->mean, out->std, out->n_pairs, out->status};
    PM4G_HIP(launch_efg(log, w, o, g_efg_pass_pairs, (hipStream_t)stream));
    return PM4G_OK;
}

size_t pm4g_sample_workspace_bytes(int64_t n_events) {
    if (n_events < 0 || n_events > kMaxEvents) return 0;
    Bump a(nullptr);
    a.take<SelState>(1);
    filter_ws_layout(a, n_events);
    Bump b(nullptr);
    b.take<SelState>(1);
    case_filter_ws_layout(b, n_events);
    return (a.off > b.off ? a.off : b.off) + 256;
}

int pm4g_sample(const pm4g_prepared* log, int64_t k, uint64_t seed, int32_t by_events, const pm4g_prepared* out,
                void* ws, size_t ws_size, void* stream) {
    if (int rc = check_prepared(log, true)) return rc;
    PM4G_CHECK(k >= 0, "k < 0");
    PM4G_CHECK(by_events == 0 || by_events == 1, "by_events must be 0 or 1");
    PM4G_CHECK(out && out->case_off && out->n_cases && out->status &&
                   (log->n_events == 0 || (out->case_s && out->act_s && out->ts_s && out->case_code)),
               "a sampled-log output array is NULL");
    PM4G_CHECK(out->n_events >= 0 && out->n_activities == log->n_activities,
               "the sampled log needs a capacity >= 0 and the same n_activities");
    const size_t need = pm4g_sample_workspace_bytes(log->n_events);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    ProfScope ps(P_SAMPLE, s);
    Bump bp(ws);
    SelState* sel = bp.take<SelState>(1);
    PM4G_HIP(launch_sample_select(log, k, seed, by_events != 0, sel, s));
    if (by_events) {
        FilterWs w = filter_ws_layout(bp, log->n_events);
        PM4G_HIP(launch_sample_events(log, seed, sel, out, w, s));
    } else {
        CaseFilterWs w = case_filter_ws_layout(bp, log->n_events);
        PM4G_HIP(launch_sample_cases(log, seed, sel, out, w, s));
    }
    return PM4G_OK;
}

size_t pm4g_ingest_csv_workspace_bytes(int64_t n_bytes, int64_t capacity) {
    if (n_bytes < 0 || capacity < 0 || capacity > kMaxEvents) return 0;
    Bump b(nullptr);
    csv_ws_layout(b, n_bytes, capacity);
    return b.off + 256;
}

int pm4g_ingest_csv(const uint8_t* text, int64_t n_bytes, const pm4g_csv_schema* sc, const pm4g_csv_out* out,
                    void* ws, size_t ws_size, void* stream) {
    PM4G_CHECK(n_bytes >= 0 && (n_bytes == 0 || text), "text is NULL or n_bytes < 0");
    PM4G_CHECK(sc != nullptr && out != nullptr, "schema or out is NULL");
    PM4G_CHECK(sc->case_col >= 0 && sc->act_col >= 0 && sc->ts_col >= 0, "a column index is negative");
    PM4G_CHECK(sc->ts_iso == 0 || sc->ts_iso == 1, "ts_iso must be 0 or 1");
    PM4G_CHECK(sc->ts_scale >= 0 && sc->ts_scale <= 9, "ts_scale outside [0, 9]");
    PM4G_CHECK(sc->sep != '"' && sc->sep != '\n' && sc->sep != '\r', "the separator cannot be a quote or a line end");
    PM4G_CHECK(out->capacity >= 0 && out->capacity <= kMaxEvents, "capacity outside [0, 2^31)");
    PM4G_CHECK(out->n_rows && out->n_cases && out->n_acts && out->status && out->bad_row &&
                   (out->capacity == 0 || (out->case_code && out->act_code && out->ts && out->case_dict_off &&
                                           out->case_dict_len && out->act_dict_off && out->act_dict_len)),
               "a CSV output array is NULL");
    const size_t need = pm4g_ingest_csv_workspace_bytes(n_bytes, out->capacity);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    ProfScope ps(P_CSV, s);
    Bump bp(ws);
    CsvWs w = csv_ws_layout(bp, n_bytes, out->capacity);
    PM4G_HIP(launch_csv_lines(text, n_bytes, sc->has_header, out->capacity, w, s));
    // values are matched by 64-bit hash, then checked byte by byte; the code
    // kernels do nothing after a parse or capacity error or a collision (two
    // values, one hash), and a collision repeats the call with the next seed
    int64_t sc_host[16];
    for (uint64_t attempt = 0;; ++attempt) {
        PM4G_HIP(launch_csv_parse(text, n_bytes, *sc, 0x5851F42D4C957F2Dull * (attempt + 1),
                                  attempt == 0 ? g_csv_hash_bits : 0, out->capacity, w, *out, s));
        PM4G_HIP(launch_csv_codes(w, out->capacity, *out, s));
        PM4G_HIP(launch_csv_finish(w, *out, s));
        PM4G_HIP(hipMemcpyAsync(sc_host, w.scal, sizeof(sc_host), hipMemcpyDeviceToHost, s));
        PM4G_HIP(hipStreamSynchronize(s));
        if (sc_host[6] || sc_host[3] != INT64_MAX || !sc_host[4]) break;
        PM4G_CHECK(attempt < 8, "value hashes kept colliding");
    }
    if (sc_host[6]) {
        set_err("more than %lld data rows", (long long)out->capacity);
        return PM4G_E_CAPACITY;
    }
    if (sc_host[3] != INT64_MAX) {
        set_err("CSV parse error at data row %lld", (long long)sc_host[3]);
        return PM4G_E_PARSE;
    }
    return PM4G_OK;
}

// The footer of a Parquet file in device memory, copied to the host.
static int parquet_footer(const uint8_t* file, int64_t n_bytes, hipStream_t s, std::vector<uint8_t>* meta) {
    PM4G_CHECK(n_bytes >= 0 && (n_bytes == 0 || file), "file is NULL or n_bytes < 0");
    if (n_bytes < 12) {
        set_err("%lld bytes: not a Parquet file", (long long)n_bytes);
        return PM4G_E_PARSE;
    }
    uint8_t tail[8], head[4];
    PM4G_HIP(hipMemcpyAsync(tail, file + n_bytes - 8, 8, hipMemcpyDeviceToHost, s));
    PM4G_HIP(hipMemcpyAsync(head, file, 4, hipMemcpyDeviceToHost, s));
    PM4G_HIP(hipStreamSynchronize(s));
    const int64_t len = (int64_t)((uint32_t)tail[0] | (uint32_t)tail[1] << 8 | (uint32_t)tail[2] << 16 |
                                  (uint32_t)tail[3] << 24);
    if (memcmp(tail + 4, "PAR1", 4) != 0 || memcmp(head, "PAR1", 4) != 0 || len > n_bytes - 12) {
        set_err("not a Parquet file (magic or footer length)");
        return PM4G_E_PARSE;
    }
    meta->resize((size_t)(len > 0 ? len : 1));
    if (len > 0) {
        PM4G_HIP(hipMemcpyAsync(meta->data(), file + n_bytes - 8 - len, (size_t)len, hipMemcpyDeviceToHost, s));
        PM4G_HIP(hipStreamSynchronize(s));
    }
    meta->resize((size_t)len);
    return PM4G_OK;
}

int pm4g_parquet_rows(const uint8_t* file, int64_t n_bytes, int64_t* rows, void* stream) {
    PM4G_CHECK(rows != nullptr, "rows is NULL");
    std::vector<uint8_t> meta;
    if (int rc = parquet_footer(file, n_bytes, (hipStream_t)stream, &meta)) return rc;
    std::vector<PqChunk> chunks;
    const int32_t cols[3] = {0, 0, 0};
    char msg[256];
    const int rc = pq_parse_footer(meta.data(), (int64_t)meta.size(), n_bytes, cols, &chunks, rows, msg, sizeof(msg));
    if (rc == PM4G_E_UNSUPPORTED || rc == PM4G_OK) return PM4G_OK;   // the row count is read either way
    set_err("%s", msg);
    return rc;
}

size_t pm4g_ingest_parquet_workspace_bytes(int64_t n_bytes, int64_t capacity) {
    if (n_bytes < 0 || capacity < 0 || capacity > kMaxEvents) return 0;
    Bump b(nullptr);
    pq_ws_layout(b, capacity);
    return b.off + 256;
}

int pm4g_ingest_parquet(const uint8_t* file, int64_t n_bytes, const pm4g_parquet_schema* sc, const pm4g_csv_out* out,
                        void* ws, size_t ws_size, void* stream) {
    PM4G_CHECK(sc != nullptr && out != nullptr, "schema or out is NULL");
    PM4G_CHECK(sc->case_col >= 0 && sc->act_col >= 0 && sc->ts_col >= 0, "a column index is negative");
    PM4G_CHECK(out->capacity >= 0 && out->capacity <= kMaxEvents, "capacity outside [0, 2^31)");
    PM4G_CHECK(out->n_rows && out->n_cases && out->n_acts && out->status && out->bad_row &&
                   (out->capacity == 0 || (out->case_code && out->act_code && out->ts && out->case_dict_off &&
                                           out->case_dict_len && out->act_dict_off && out->act_dict_len)),
               "an ingestion output array is NULL");
    const size_t need = pm4g_ingest_parquet_workspace_bytes(n_bytes, out->capacity);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    ProfScope ps(P_PARQUET, s);
    std::vector<uint8_t> meta;
    if (int rc = parquet_footer(file, n_bytes, s, &meta)) return rc;
    std::vector<PqChunk> chunks;
    const int32_t cols[3] = {sc->case_col, sc->act_col, sc->ts_col};
    int64_t rows = 0;
    char msg[256];
    int rc = pq_parse_footer(meta.data(), (int64_t)meta.size(), n_bytes, cols, &chunks, &rows, msg, sizeof(msg));
    if (rc == PM4G_OK && (int64_t)chunks.size() > kPqMaxChunks) {
        snprintf(msg, sizeof(msg), "more than %lld row groups", (long long)(kPqMaxChunks / 3));
        rc = PM4G_E_UNSUPPORTED;
    }
    if (rc == PM4G_OK && rows > out->capacity) {
        snprintf(msg, sizeof(msg), "%lld rows, capacity %lld", (long long)rows, (long long)out->capacity);
        rc = PM4G_E_CAPACITY;
    }
    if (rc != PM4G_OK) {
        set_err("%s", msg);
        if (rc == PM4G_E_UNSUPPORTED || rc == PM4G_E_CAPACITY || rc == PM4G_E_PARSE) {
            k_set_status<<<1, 1, 0, s>>>(out->status, rc);
            PM4G_HIP(hipGetLastError());
            PM4G_HIP(hipMemsetAsync(out->n_rows, 0, sizeof(int64_t), s));
            PM4G_HIP(hipStreamSynchronize(s));
        }
        return rc;
    }
    Bump bp(ws);
    PqWs w = pq_ws_layout(bp, out->capacity);
    w.max_rows = out->capacity > 0 ? out->capacity : 1;
    // page-table ranges: a data page of at least 32 values on average fits
    // (a chunk whose pages do not fit has them found by walking again)
    int64_t pt_used = 0;
    for (PqChunk& c : chunks) {
        const int64_t want = c.num_values / 32 + 4;
        const int64_t cap = want < w.pt_size - pt_used ? want : w.pt_size - pt_used;
        c.pt_off = pt_used;
        c.pt_cap = (int32_t)(cap < INT32_MAX ? cap : INT32_MAX);
        pt_used += c.pt_cap;
    }
    if (!chunks.empty())
        PM4G_HIP(hipMemcpyAsync(w.chunks, chunks.data(), chunks.size() * sizeof(PqChunk), hipMemcpyHostToDevice, s));
    PM4G_HIP(launch_pq_decode(file, w, (int64_t)chunks.size(), rows, out->ts, s));
    // values matched by hash and compared as they enter the tables; the code
    // kernels do nothing after a decode error or a null
    PM4G_HIP(launch_pq_match(file, w, rows, 0x2545F4914F6CDD1Dull, g_csv_hash_bits, s));
    PM4G_HIP(launch_pq_codes(w, rows, *out, s));
    PM4G_HIP(launch_pq_finish(w, *out, s));
    int64_t sc_host[16];
    PM4G_HIP(hipMemcpyAsync(sc_host, w.scal, sizeof(sc_host), hipMemcpyDeviceToHost, s));
    PM4G_HIP(hipStreamSynchronize(s));
    if (sc_host[0] != 0) {
        set_err("%s", sc_host[0] == PM4G_E_UNSUPPORTED ? "a page encoding outside the covered subset"
                                                       : "malformed Parquet page");
        return (int)sc_host[0];
    }
    if (sc_host[1] != INT64_MAX) {
        set_err("null value at row %lld", (long long)sc_host[1]);
        return PM4G_E_PARSE;
    }
    return PM4G_OK;
}

int pm4g_cases(const pm4g_prepared* log, int64_t* n_events_out, int64_t* throughput_out, void* stream) {
    if (int rc = check_prepared(log, true)) return rc;
    PM4G_HIP(launch_cases_df(log, n_events_out, throughput_out, (hipStream_t)stream));
    return PM4G_OK;
}

size_t pm4g_filter_cases_workspace_bytes(int64_t n_events) {
    if (n_events < 0 || n_events > kMaxEvents) return 0;
    Bump b(nullptr);
    case_filter_ws_layout(b, n_events);
    return b.off + 256;
}

int pm4g_filter_cases(const pm4g_prepared* log, const pm4g_case_filter* filter, const pm4g_prepared* out,
                      void* ws, size_t ws_size, void* stream) {
    if (int rc = check_prepared(log, true)) return rc;
    PM4G_CHECK(filter != nullptr, "filter is NULL");
    PM4G_CHECK(filter->path_keep == 0 || filter->path_keep == 1, "path_keep must be 0 or 1");
    PM4G_CHECK(filter->variant_keep == 0 || filter->variant_keep == 1, "variant_keep must be 0 or 1");
    PM4G_CHECK(!filter->variant_mask || (filter->case_variant && filter->n_variant_bits >= 0),
               "variant_mask needs case_variant and n_variant_bits >= 0");
    PM4G_CHECK(out && out->case_off && out->n_cases && out->status &&
                   (log->n_events == 0 || (out->case_s && out->act_s && out->ts_s && out->case_code)),
               "a filtered-log output array is NULL");
    PM4G_CHECK(out->n_events >= 0 && out->n_activities == log->n_activities,
               "the filtered log needs a capacity >= 0 and the same n_activities");
    const size_t need = pm4g_filter_cases_workspace_bytes(log->n_events);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    Bump bp(ws);
    CaseFilterWs w = case_filter_ws_layout(bp, log->n_events);
    PM4G_HIP(launch_filter_cases(log, filter, out, w, (hipStream_t)stream));
    return PM4G_OK;
}

int pm4g_dfg_batched(const pm4g_prepared* log, const pm4g_view* views, const uint64_t* act_masks,
                     int32_t n_views, const pm4g_batched_out* out, const pm4g_batched_tuning* tuning,
                     void* ws, size_t ws_size, void* stream) {
    if (int rc = check_prepared(log, true)) return rc;
    PM4G_CHECK(log->n_activities <= PM4G_BATCHED_MAX_ACTIVITIES, "n_activities %d above %d for batched views",
               log->n_activities, PM4G_BATCHED_MAX_ACTIVITIES);
    PM4G_CHECK(n_views >= 0, "n_views < 0");
    PM4G_CHECK((int64_t)n_views * view_buckets(log->n_activities) <= (int64_t)0xFFFFFFFF,
               "%d views of %d activities: more (view, cell bucket) pairs than 2^32 - 1; split the views",
               n_views, log->n_activities);
    PM4G_CHECK(n_views == 0 || (views && act_masks), "views or act_masks is NULL");
    PM4G_CHECK(out && out->edge_off && out->start_count && out->end_count && out->act_count && out->n_events &&
                   out->n_cases && out->required && out->status && out->cap_edges >= 0 &&
                   (out->cap_edges == 0 ||
                    (out->src && out->dst && out->count && out->dt_sum && out->dt_min && out->dt_max)),
               "a batched output array is NULL (only dt_mean may be NULL)");
    BatchedTune t;
    if (int rc = resolve_tuning(tuning, log->n_events, n_views, &t)) return rc;
    const size_t need = batched_ws_bytes(log->n_events, log->n_activities, n_views, t);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    Bump bp(ws);
    ViewWs w = view_ws_layout(bp, log->n_events, log->n_activities, n_views, t.tile, t.pair_cap, t.rec_cap,
                              t.cell_cap);
    const BatchedOutDev o{out->edge_off, out->src, out->dst, out->count, out->dt_sum, out->dt_min,
                          out->dt_max, out->dt_mean, out->start_count, out->end_count, out->act_count,
                          out->n_events, out->n_cases, out->cap_edges, out->required, out->status};
    if (t.launch == 0) {
        PM4G_HIP(launch_views_fused(log, views, act_masks, n_views, w, o, s));
    } else {
        PM4G_HIP(launch_views_plan(log, views, n_views, w, o, s));
        PM4G_HIP(launch_views_count(log, views, act_masks, w, t.emit_blocks, s));
        PM4G_HIP(launch_views_reduce(log, views, act_masks, n_views, w, o, t.emit_blocks, t.agg_blocks, s));
    }
    return PM4G_OK;
}

int pm4g_prepare(const pm4g_log* log, const pm4g_prepared* out, void* ws, size_t ws_size,
                 void* stream) {
    if (int rc = check_log(log)) return rc;
    PM4G_CHECK(out && out->case_off && out->n_cases && out->status &&
                   (log->n_events == 0 || (out->case_s && out->act_s && out->ts_s && out->case_code)),
               "a prepared output array is NULL");
    PM4G_CHECK(out->n_events == log->n_events && out->n_activities == log->n_activities,
               "prepared n_events/n_activities differ from the log's");
    const size_t need = ws_bytes(PM4G_OP_PREPARE, log->n_events, log->n_activities);
    if (ws_size < need || (need && !ws)) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    Bump bp(ws);
    return run_prepare(log, out, true, bp, (hipStream_t)stream, true);
}

int pm4g_dfg_prepared(const pm4g_prepared* log, const pm4g_dfg_out* out, void* ws, size_t ws_size,
                      void* stream) {
    if (int rc = check_prepared(log, false)) return rc;
    if (int rc = check_dfg_out(out)) return rc;
    const size_t need = ws_bytes(PM4G_OP_DFG_PREPARED, log->n_events, log->n_activities);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    Bump bp(ws);
    DfgWs w = dfg_ws_layout(bp, log->n_events, log->n_activities);
    PM4G_HIP(launch_dfg(log->case_s, log->act_s, log->ts_s, log->n_events, log->n_activities,
                        log->status, w, dev_out(out), (hipStream_t)stream));
    return PM4G_OK;
}

int pm4g_dfg_prepared_noalloc(const pm4g_prepared* log, const pm4g_dfg_out* out, void* stream) {
    if (int rc = check_prepared(log, false)) return rc;
    if (int rc = check_dfg_out(out)) return rc;
    const size_t need = ws_bytes(PM4G_OP_DFG_PREPARED, log->n_events, log->n_activities);
    if (need > PM4G_NOALLOC_SCRATCH_BYTES) {
        set_err("%lld events of %d activities need %zu bytes of workspace; the library's scratch holds %zu",
                (long long)log->n_events, log->n_activities, need, (size_t)PM4G_NOALLOC_SCRATCH_BYTES);
        return PM4G_E_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    void* ptr = nullptr;
    if (int rc = scratch_of_current_device(&ptr)) return rc;
    if (s) {
        int cur = -1;
        hipDevice_t sdev = -1;
        PM4G_HIP(hipGetDevice(&cur));
        PM4G_HIP(hipStreamGetDevice(s, &sdev));
        PM4G_CHECK(sdev == cur, "the stream belongs to device %d, the current device is %d", (int)sdev, cur);
    }
    Bump bp(ptr);
    DfgWs w = dfg_ws_layout(bp, log->n_events, log->n_activities);
    PM4G_HIP(launch_dfg(log->case_s, log->act_s, log->ts_s, log->n_events, log->n_activities,
                        log->status, w, dev_out(out), s));
    return PM4G_OK;
}

int pm4g_dfg(const pm4g_log* log, const pm4g_dfg_out* out, void* ws, size_t ws_size, void* stream) {
    if (int rc = check_log(log)) return rc;
    if (int rc = check_dfg_out(out)) return rc;
    const size_t need = ws_bytes(PM4G_OP_DFG, log->n_events, log->n_activities);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    Bump bp(ws);
    pm4g_prepared p = prepared_in_ws(bp, log->n_events, log->n_activities);
    const size_t rest = bp.off;
    {
        Bump b2(static_cast<char*>(ws) + ((rest + 255) & ~size_t(255)));
        int rc = run_prepare(log, &p, false, b2, s);
        if (rc != PM4G_OK) {
            if (rc != PM4G_E_DEVICE) {
                k_set_status<<<1, 1, 0, s>>>(out->status, rc);
                PM4G_HIP(hipGetLastError());
            }
            return rc;
        }
    }
    Bump b3(static_cast<char*>(ws) + ((rest + 255) & ~size_t(255)));
    DfgWs w = dfg_ws_layout(b3, log->n_events, log->n_activities);
    PM4G_HIP(launch_dfg(p.case_s, p.act_s, p.ts_s, p.n_events, p.n_activities, p.status, w,
                        dev_out(out), s));
    return PM4G_OK;
}

int pm4g_variants_prepared(const pm4g_prepared* log, const pm4g_variants_out* out, void* ws,
                           size_t ws_size, void* stream) {
    if (int rc = check_prepared(log, true)) return rc;
    if (int rc = check_var_out(out)) return rc;
    const size_t need = ws_bytes(PM4G_OP_VARIANTS_PREPARED, log->n_events, log->n_activities);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    Bump bp(ws);
    VarWs w = var_ws_layout(bp, log->n_events);
    const VarOutDev o{out->n_variants, out->var_count, out->var_len, out->var_rep,
                      out->var_off,    out->var_acts,  out->case_variant, out->status};
    PM4G_HIP(launch_variants(log->act_s, log->case_off, log->case_code, log->n_cases, log->status,
                             log->n_events, w, o, (uint32_t)g_variant_hash_bits,
                             (hipStream_t)stream));
    return PM4G_OK;
}

int pm4g_variants(const pm4g_log* log, const pm4g_variants_out* out, void* ws, size_t ws_size,
                  void* stream) {
    if (int rc = check_log(log)) return rc;
    if (int rc = check_var_out(out)) return rc;
    const size_t need = ws_bytes(PM4G_OP_VARIANTS, log->n_events, log->n_activities);
    if (ws_size < need || !ws) {
        set_err("workspace of %zu bytes, %zu needed", ws_size, need);
        return PM4G_E_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    Bump bp(ws);
    pm4g_prepared p = prepared_in_ws(bp, log->n_events, log->n_activities);
    const size_t rest = bp.off;
    {
        Bump b2(static_cast<char*>(ws) + ((rest + 255) & ~size_t(255)));
        int rc = run_prepare(log, &p, true, b2, s);
        if (rc != PM4G_OK) {
            if (rc != PM4G_E_DEVICE) {
                k_set_status<<<1, 1, 0, s>>>(out->status, rc);
                PM4G_HIP(hipGetLastError());
            }
            return rc;
        }
    }
    Bump b3(static_cast<char*>(ws) + ((rest + 255) & ~size_t(255)));
    VarWs w = var_ws_layout(b3, log->n_events);
    const VarOutDev o{out->n_variants, out->var_count, out->var_len, out->var_rep,
                      out->var_off,    out->var_acts,  out->case_variant, out->status};
    PM4G_HIP(launch_variants(p.act_s, p.case_off, p.case_code, p.n_cases, p.status, p.n_events, w, o,
                             (uint32_t)g_variant_hash_bits, s));
    return PM4G_OK;
}

}  // extern "C"
