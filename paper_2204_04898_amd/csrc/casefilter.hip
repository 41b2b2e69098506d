// Cases dataframe and case-level filters of a prepared log (Sec. 3: the cases
// dataframe holds, per case, its number of events and its throughput time;
// case-level filtering on them; the DFG module's paths filtering, which keeps
// or drops the cases that contain given directly-follows pairs; timestamp
// filters on whole cases; start/end activity and variant filters).
//
//   k_cases_df      per case: events = case_off[c+1] - case_off[c], throughput
//                   = ts of its last event - ts of its first (mod 2^64)
//   k_cf_contains   only with an activity or path set: a wave walks the events
//                   of 64 consecutive cases coalesced; an event whose activity
//                   (or whose pair with the previous event of its case) is in
//                   the set marks its case in LDS
//   k_cf_decide     per case: all predicates -> kept; kept events, kept flag
//                   (range, time-window, start/end activity and variant
//                   predicates read the case's first and last event and its
//                   variant id)
//   scans           output position of each kept case's events and of its row
//                   in the output case table
//   k_cf_emit       kept cases' events copied in order (a wave per 64 cases,
//                   coalesced writes), case table rows
//   k_cf_finish     case count, case_off[K], status
// Counts stay on the device; nothing synchronises.  Bytes: per case 16 read +
// 24 written (tables), 16 per kept event read + 16 written; the containment
// pass reads 4-8 B per event.
#include "common.hpp"
#include "devsort.hpp"
#include "internal.hpp"
#include "prof.hpp"
#include "../../include/pm4g.h"

namespace pm4g {

// Segment of event position p among 64 consecutive segments, as seg_at, with
// 32-bit starts: event positions stay below 2^31 (the log's size limit), so
// each search step exchanges one dword instead of two.  INT32_MAX marks an
// absent lane; every lane of the wave must execute it.
__device__ __forceinline__ int seg_at32(int32_t vstart, int64_t p) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int cand = lo + step;
        if ((int64_t)__shfl(vstart, cand) <= p) lo = cand;
    }
    return lo;
}

CaseFilterWs case_filter_ws_layout(Bump& b, int64_t n) {
    CaseFilterWs w{};
    const size_t m = (size_t)(n > 0 ? n : 1);
    w.flags = b.take<uint32_t>(m);
    w.cnt = b.take<uint32_t>(m);
    w.kept = b.take<uint32_t>(m);
    w.eoff = b.take<int64_t>(m);
    w.koff = b.take<uint32_t>(m);
    w.part32 = b.take<uint32_t>(dev::kScanGrid);
    w.part64 = b.take<int64_t>(dev::kScanGrid);
    w.scal = b.take<int64_t>(8);
    w.uscal = b.take<uint32_t>(8);
    return w;
}

namespace {

constexpr int kCB = 256;
constexpr int kCGrid = 2048;

__global__ __launch_bounds__(kCB) void k_cases_df(const int64_t* __restrict__ case_off,
                                                  const int64_t* __restrict__ ts_s, const int64_t* n_cases,
                                                  int64_t* __restrict__ n_events, int64_t* __restrict__ thr) {
    const int64_t C = *n_cases;
    for (int64_t c = (int64_t)blockIdx.x * kCB + threadIdx.x; c < C; c += (int64_t)gridDim.x * kCB) {
        const int64_t a = case_off[c], b = case_off[c + 1];
        if (n_events) n_events[c] = b - a;
        if (thr) thr[c] = (int64_t)((uint64_t)ts_s[b - 1] - (uint64_t)ts_s[a]);
    }
}

__device__ __forceinline__ bool bit_of(const uint64_t* m, int64_t b) { return (m[b >> 6] >> (b & 63)) & 1ull; }

// flags[c]: bit 0 = the case has an activity of act_mask, bit 1 = it has a
// directly-follows pair of path_mask.
__global__ __launch_bounds__(kCB) void k_cf_contains(const int32_t* __restrict__ act_s,
                                                     const int64_t* __restrict__ case_off, const int64_t* n_cases,
                                                     int32_t A, const uint64_t* __restrict__ act_mask,
                                                     const uint64_t* __restrict__ path_mask,
                                                     uint32_t* __restrict__ flags) {
    __shared__ uint32_t lflag[kCB / kWave][kWave];
    const int64_t C = *n_cases;
    const int wl = threadIdx.x / kWave;
    const int64_t wv = ((int64_t)blockIdx.x * kCB + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * kCB / kWave;
    for (int64_t c0 = wv * kWave; c0 < C; c0 += nw * kWave) {
        const int64_t c = c0 + lane();
        const bool has = c < C;
        const int64_t st = has ? case_off[c] : INT64_MAX;
        const int64_t en = has ? case_off[c + 1] : 0;
        lflag[wl][lane()] = 0;
        const int last = (C - 1 - c0) < (kWave - 1) ? (int)(C - 1 - c0) : (kWave - 1);
        const int64_t base = __shfl(st, 0);
        const int64_t end = __shfl(en, last);
        const int32_t st32 = has ? (int32_t)st : INT32_MAX;
        for (int64_t p0 = base; p0 < end; p0 += kWave) {   // wave-uniform trip count
            const int64_t p = p0 + lane();
            const int m = seg_at32(st32, p);
            const int64_t s_m = __shfl(st32, m);
            if (p < end) {
                const int32_t a = act_s[p];
                uint32_t bits = 0;
                if (act_mask && bit_of(act_mask, a)) bits |= 1u;
                if (path_mask && p > s_m && bit_of(path_mask, (int64_t)act_s[p - 1] * A + a)) bits |= 2u;
                if (bits) atomicOr(&lflag[wl][m], bits);
            }
        }
        if (has) flags[c] = lflag[wl][lane()];
    }
}

__global__ __launch_bounds__(kCB) void k_cf_decide(const int32_t* __restrict__ act_s,
                                                   const int64_t* __restrict__ case_off,
                                                   const int64_t* __restrict__ ts_s, const int64_t* n_cases,
                                                   pm4g_case_filter f, CaseFilterWs w) {
    const int64_t C = *n_cases;
    const bool use_act = f.act_mask != nullptr, use_path = f.path_mask != nullptr;
    for (int64_t c = (int64_t)blockIdx.x * kCB + threadIdx.x; c < C; c += (int64_t)gridDim.x * kCB) {
        const int64_t a = case_off[c], b = case_off[c + 1];
        const int64_t ev = b - a;
        const int64_t t0 = ts_s[a], t1 = ts_s[b - 1];
        const int64_t thr = (int64_t)((uint64_t)t1 - (uint64_t)t0);
        bool keep = ev >= f.min_events && ev <= f.max_events && thr >= f.min_throughput &&
                    thr <= f.max_throughput && t0 >= f.contain_lo && t1 <= f.contain_hi && t0 <= f.meet_hi &&
                    t1 >= f.meet_lo;
        if (use_act || use_path) {
            const uint32_t fl = w.flags[c];
            if (use_act) keep = keep && (fl & 1u);
            if (use_path) keep = keep && (((fl >> 1) & 1u) == (f.path_keep ? 1u : 0u));
        }
        if (f.start_mask) keep = keep && bit_of(f.start_mask, act_s[a]);
        if (f.end_mask) keep = keep && bit_of(f.end_mask, act_s[b - 1]);
        if (f.variant_mask) {
            const int64_t v = f.case_variant[c];
            const bool in = v >= 0 && v < f.n_variant_bits && bit_of(f.variant_mask, v);
            keep = keep && (in == (f.variant_keep != 0));
        }
        w.cnt[c] = keep ? (uint32_t)ev : 0u;
        w.kept[c] = keep ? 1u : 0u;
    }
}

// scal[1] = kept events (scan total), uscal[0] = kept cases; scal[2] = 1 when
// the output cannot hold them (nothing is written then).
__global__ void k_cf_check(CaseFilterWs w, int64_t cap) { w.scal[2] = w.scal[1] > cap ? 1 : 0; }

__global__ __launch_bounds__(kCB) void k_cf_emit(const int32_t* __restrict__ case_s,
                                                 const int32_t* __restrict__ act_s,
                                                 const int64_t* __restrict__ ts_s,
                                                 const int64_t* __restrict__ case_off,
                                                 const int32_t* __restrict__ case_code, const int64_t* n_cases,
                                                 CaseFilterWs w, int32_t* __restrict__ o_case,
                                                 int32_t* __restrict__ o_act, int64_t* __restrict__ o_ts,
                                                 int64_t* __restrict__ o_off, int32_t* __restrict__ o_code) {
    if (w.scal[2]) return;   // over capacity (block-uniform)
    const int64_t C = *n_cases;
    const int64_t wv = ((int64_t)blockIdx.x * kCB + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * kCB / kWave;
    for (int64_t c0 = wv * kWave; c0 < C; c0 += nw * kWave) {
        const int64_t c = c0 + lane();
        const bool has = c < C;
        int64_t src = 0, dst = INT64_MAX, len = 0;
        if (has) {
            src = case_off[c];
            dst = w.eoff[c];
            len = w.cnt[c];
            if (w.kept[c]) {
                const uint32_t k = w.koff[c];
                o_off[k] = dst;
                o_code[k] = case_code[c];
            }
        }
        const int last = (C - 1 - c0) < (kWave - 1) ? (int)(C - 1 - c0) : (kWave - 1);
        const int64_t base = __shfl(dst, 0);
        const int64_t end = __shfl(dst + len, last);
        // positions fit 32 bits: output starts and the source-minus-output shift
        // are exchanged as dwords
        const int32_t dst32 = has ? (int32_t)dst : INT32_MAX;
        const int32_t shift = (int32_t)(src - (has ? dst : 0));
        // dropped cases are empty segments: the last segment starting at or before
        // p is the kept case that holds p
        for (int64_t p0 = base; p0 < end; p0 += kWave) {   // wave-uniform trip count
            const int64_t p = p0 + lane();
            const int m = seg_at32(dst32, p);
            const int32_t sh = __shfl(shift, m);
            if (p < end) {
                const int64_t i = p + sh;
                o_case[p] = case_s[i];
                o_act[p] = act_s[i];
                o_ts[p] = ts_s[i];
            }
        }
    }
}

__global__ void k_cf_finish(CaseFilterWs w, int64_t* o_off, int64_t* o_n_cases, int32_t* o_status,
                            const int32_t* status_in) {
    const bool over = w.scal[2] != 0;
    const int64_t K = over ? 0 : (int64_t)w.uscal[0];
    o_off[K] = over ? 0 : w.scal[1];
    *o_n_cases = K;
    *o_status = (status_in && *status_in) ? *status_in : (over ? PM4G_E_CAPACITY : 0);
}

}  // namespace

hipError_t launch_cases_df(const pm4g_prepared* p, int64_t* n_events, int64_t* thr, hipStream_t s) {
    ProfScope ps(P_CASES, s);
    const int64_t n = p->n_events;
    const int64_t g = (n + kCB - 1) / kCB;
    k_cases_df<<<(unsigned)(g < kCGrid ? (g < 1 ? 1 : g) : kCGrid), kCB, 0, s>>>(p->case_off, p->ts_s, p->n_cases,
                                                                                n_events, thr);
    return hipGetLastError();
}

namespace {

// Sampling by cases: a case is kept iff its id's SplitMix64 key is at most the
// selected threshold.
__global__ __launch_bounds__(kCB) void k_cf_sample(const int64_t* __restrict__ case_off,
                                                   const int32_t* __restrict__ case_code, const int64_t* n_cases,
                                                   uint64_t seed, const SelState* sel, CaseFilterWs w) {
    const int64_t C = *n_cases;
    const uint64_t T = sel->T;
    const bool none = sel->none != 0, all = sel->all != 0;
    for (int64_t c = (int64_t)blockIdx.x * kCB + threadIdx.x; c < C; c += (int64_t)gridDim.x * kCB) {
        const bool keep = !none && (all || splitmix64(seed, (uint64_t)(uint32_t)case_code[c]) <= T);
        w.cnt[c] = keep ? (uint32_t)(case_off[c + 1] - case_off[c]) : 0u;
        w.kept[c] = keep ? 1u : 0u;
    }
}

// The kept cases (w.cnt, w.kept) copied into out.
void materialise_cases(const pm4g_prepared* p, const pm4g_prepared* out, CaseFilterWs w, hipStream_t s) {
    dev::excl_scan<int64_t>(w.cnt, p->n_cases, w.eoff, w.part64, &w.scal[1], s);
    dev::excl_scan<uint32_t>(w.kept, p->n_cases, w.koff, w.part32, &w.uscal[0], s);
    k_cf_check<<<1, 1, 0, s>>>(w, out->n_events);
    k_cf_emit<<<kCGrid, kCB, 0, s>>>(p->case_s, p->act_s, p->ts_s, p->case_off, p->case_code, p->n_cases, w,
                                     out->case_s, out->act_s, out->ts_s, out->case_off, out->case_code);
    k_cf_finish<<<1, 1, 0, s>>>(w, out->case_off, out->n_cases, out->status, p->status);
}

}  // namespace

hipError_t launch_filter_cases(const pm4g_prepared* p, const pm4g_case_filter* f, const pm4g_prepared* out,
                               CaseFilterWs w, hipStream_t s) {
    ProfScope ps(P_CASE_FILTER, s);
    const pm4g_case_filter fv = *f;
    if (fv.act_mask || fv.path_mask)
        k_cf_contains<<<kCGrid, kCB, 0, s>>>(p->act_s, p->case_off, p->n_cases, p->n_activities, fv.act_mask,
                                             fv.path_mask, w.flags);
    k_cf_decide<<<kCGrid, kCB, 0, s>>>(p->act_s, p->case_off, p->ts_s, p->n_cases, fv, w);
    materialise_cases(p, out, w, s);
    return hipGetLastError();
}

hipError_t launch_sample_cases(const pm4g_prepared* p, uint64_t seed, const SelState* sel,
                               const pm4g_prepared* out, CaseFilterWs w, hipStream_t s) {
    k_cf_sample<<<kCGrid, kCB, 0, s>>>(p->case_off, p->case_code, p->n_cases, seed, sel, w);
    materialise_cases(p, out, w, s);
    return hipGetLastError();
}

}  // namespace pm4g
