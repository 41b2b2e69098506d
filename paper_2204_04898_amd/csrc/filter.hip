// Event-level filters of a prepared log, each materialised as a prepared log
// of its own whose events keep the (case, timestamp, row) order:
//   - one drill-down view (Sec. 3: timestamp filter on events and attribute
//     filter), over the view's slice [p0, p1) of whole cases;
//   - the directly-follows level filter (Sec. 3: an event kept or dropped on
//     the pair it forms with the previous, or next, event of its case), over
//     the whole log;
//   - a sample of events (Sec. 3 sampling module): the positions whose
//     SplitMix64 key is at most the selected threshold.
// Stream compaction with the predicate as a template parameter:
//   k_filter_slice / k_filter_whole   p0, p1 on the device
//   k_filter_count   per-tile kept counts (persistent grid over the slice)
//   scan             tile offsets, kept total
//   k_filter_cap     (whole-log filter) kept total against the capacity
//   k_filter_emit    kept events written in order
//   case table       of the kept events; case_off[C] = kept total
// Bytes per event: the view reads 12 (act, ts), the pair filter 8 (case, act;
// the partner's sit in the same lines) in each of the count and emit passes;
// 16 read + 16 written per kept event.
#include "common.hpp"
#include "devsort.hpp"
#include "internal.hpp"
#include "prof.hpp"
#include "../../include/pm4g.h"

namespace pm4g {

FilterWs filter_ws_layout(Bump& b, int64_t n) {
    FilterWs w{};
    const int64_t tiles = (n + kFilterTile - 1) / kFilterTile;
    w.scal = b.take<int64_t>(8);
    w.tile_cnt = b.take<uint32_t>((size_t)tiles + 1);
    w.tile_off = b.take<int64_t>((size_t)tiles + 1);
    w.part64 = b.take<int64_t>(dev::kScanGrid);
    w.caseblk = b.take<uint32_t>((size_t)case_blocks(n) + 1);
    return w;
}

namespace {

constexpr int kFB = 256;
constexpr int kFI = kFilterTile / kFB;   // 16 events per thread

__device__ int64_t lb_i32(const int32_t* a, int64_t n, int32_t x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// scal: [0] p0, [1] p1, [2] tiles of the slice, [3] kept total, [5] kept cases,
// [6] case-table blocks, [7] slice size when it exceeded the output capacity
__global__ void k_filter_slice(const pm4g_view* view, const int64_t* case_off, const int32_t* case_code,
                               const int64_t* n_cases, int64_t cap, FilterWs w) {
    const pm4g_view v = *view;
    const int64_t C = *n_cases;
    int64_t p0 = 0, p1 = 0;
    if (v.case_lo < v.case_hi && v.t_lo <= v.t_hi) {
        p0 = case_off[lb_i32(case_code, C, v.case_lo)];
        p1 = case_off[lb_i32(case_code, C, v.case_hi)];
    }
    w.scal[7] = 0;
    if (p1 - p0 > cap) {   // the output cannot hold the slice: keep nothing, report
        w.scal[7] = p1 - p0;
        p1 = p0;
    }
    w.scal[0] = p0;
    w.scal[1] = p1;
    w.scal[2] = (p1 - p0 + kFilterTile - 1) / kFilterTile;
}

// Event predicates of the compaction.  ready() runs once per kernel (it may
// read device memory); the result answers for a position i of the log that is
// in the slice when `in` is set (out-of-slice positions answer false).  The
// 64 lanes of a wave call it together on consecutive positions.
struct ViewPred {
    const pm4g_view* view;
    const uint64_t* mask;
    const int32_t* act_s;
    const int64_t* ts_s;
    struct Ready {
        pm4g_view v;
        const uint64_t* mask;
        const int32_t* act_s;
        const int64_t* ts_s;
        __device__ __forceinline__ bool operator()(int64_t i, bool in) const {
            if (!in) return false;
            const int32_t a = act_s[i];
            const int64_t t = ts_s[i];
            return t >= v.t_lo && t <= v.t_hi && ((mask[a >> 6] >> (a & 63)) & 1ull);
        }
    };
    __device__ __forceinline__ Ready ready() const { return Ready{*view, mask, act_s, ts_s}; }
};

// Directly-follows level: the pair an event forms with the previous (side 0)
// or next (side 1) event of its case, looked up in a bit set over src*A+dst.
// Its slice is the whole log (positions 0..n-1), so the partner of an event,
// when it exists, sits in the neighbouring lane, except at the wave's edge,
// whose lane loads it.
struct PairPred {
    const int32_t* case_s;
    const int32_t* act_s;
    const uint64_t* pairs;
    int64_t n;
    int32_t A;
    int32_t side;
    int32_t keep;
    __device__ __forceinline__ PairPred ready() const { return *this; }
    __device__ __forceinline__ bool operator()(int64_t i, bool in) const {
        const int32_t c = in ? case_s[i] : 0;
        const int32_t a = in ? act_s[i] : 0;
        const int64_t j = side ? i + 1 : i - 1;   // partner position
        int32_t cj = side ? __shfl_down(c, 1) : __shfl_up(c, 1);
        int32_t aj = side ? __shfl_down(a, 1) : __shfl_up(a, 1);
        const bool has = in && j >= 0 && j < n;
        const bool edge = side ? lane() == kWave - 1 : lane() == 0;
        if (edge && has) {
            cj = case_s[j];
            aj = act_s[j];
        }
        bool match = false;
        if (has && cj == c) {
            const int64_t src = side ? a : aj;
            const int64_t dst = side ? aj : a;
            const int64_t cell = src * A + dst;
            match = (pairs[cell >> 6] >> (cell & 63)) & 1ull;
        }
        return in && (keep ? match : !match);
    }
};

// Sampling by events: a position is kept iff its SplitMix64 key is at most
// the selected threshold.
struct SamplePred {
    uint64_t seed;
    const SelState* sel;
    struct Ready {
        uint64_t seed, T;
        int32_t none, all;
        __device__ __forceinline__ bool operator()(int64_t i, bool in) const {
            return in && !none && (all || splitmix64(seed, (uint64_t)i) <= T);
        }
    };
    __device__ __forceinline__ Ready ready() const { return Ready{seed, sel->T, sel->none, sel->all}; }
};

template <class Pred>
__global__ __launch_bounds__(kFB) void k_filter_count(Pred pred, FilterWs w) {
    __shared__ uint32_t tmp[kFB / kWave + 1];
    const auto keep = pred.ready();
    const int64_t p0 = w.scal[0], p1 = w.scal[1], nt = w.scal[2];
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        uint32_t c = 0;
        for (int q = 0; q < kFI; ++q) {
            const int64_t i = p0 + t * kFilterTile + q * kFB + threadIdx.x;
            if (keep(i, i < p1)) ++c;
        }
        uint32_t total;
        block_excl_sum<kFB>(c, tmp, &total);
        if (threadIdx.x == 0) w.tile_cnt[t] = total;
    }
}

// Order-preserving compaction of one tile of kPer * kB positions, striped:
// stripe q covers positions [q*kB, (q+1)*kB) of the tile, thread x holds
// position q*kB + x of each stripe (coalesced loads and stores).  A kept
// position's rank is the kept count of the earlier stripes, then of the
// earlier waves of its stripe, then of the lower lanes of its wave.
// flag(q) says whether this thread's position of stripe q is kept;
// emit(q, rank) writes it.  wcnt is kPer x (kB/64) words of LDS.  Every
// thread of the block must call it; it synchronises the block twice.
template <int kB, int kPer, class Flag, class Emit>
__device__ __forceinline__ void striped_compact(int64_t r0, uint32_t (*wcnt)[kB / kWave], Flag flag, Emit emit) {
    const int wid = threadIdx.x / kWave;
    uint64_t m[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        m[q] = __ballot(flag(q));
        if (lane() == 0) wcnt[q][wid] = (uint32_t)__popcll(m[q]);
    }
    __syncthreads();
    int64_t r = r0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int k = 0; k < kB / kWave; ++k) {
            const uint32_t c = wcnt[q][k];
            before += k < wid ? c : 0u;
            all += c;
        }
        if ((m[q] >> lane()) & 1ull) emit(q, r + before + __popcll(m[q] & lanes_below()));
        r += all;
    }
    __syncthreads();   // wcnt is rewritten by the next call
}

template <class Pred>
__global__ __launch_bounds__(kFB) void k_filter_emit(const int32_t* __restrict__ case_s,
                                                     const int32_t* __restrict__ act_s,
                                                     const int64_t* __restrict__ ts_s, Pred pred, FilterWs w,
                                                     int32_t* __restrict__ o_case, int32_t* __restrict__ o_act,
                                                     int64_t* __restrict__ o_ts) {
    __shared__ uint32_t wcnt[kFI][kFB / kWave];
    const auto keep = pred.ready();
    const int64_t p0 = w.scal[0], p1 = w.scal[1], nt = w.scal[2];
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const int64_t base = p0 + t * kFilterTile + threadIdx.x;
        striped_compact<kFB, kFI>(
            w.tile_off[t], wcnt,
            [&](int q) {
                const int64_t i = base + (int64_t)q * kFB;
                return keep(i, i < p1);
            },
            [&](int q, int64_t o) {
                const int64_t i = base + (int64_t)q * kFB;
                o_case[o] = case_s[i];
                o_act[o] = act_s[i];
                o_ts[o] = ts_s[i];
            });
    }
}

// whole log as the slice
__global__ void k_filter_whole(int64_t n, FilterWs w) {
    w.scal[0] = 0;
    w.scal[1] = n;
    w.scal[2] = (n + kFilterTile - 1) / kFilterTile;
    w.scal[7] = 0;
}

// after the count: a kept total above the output's capacity empties the
// result (no tile is emitted) and is reported through scal[7]
__global__ void k_filter_cap(int64_t cap, FilterWs w) {
    if (w.scal[3] > cap) {
        w.scal[7] = w.scal[3];
        w.scal[2] = 0;
        w.scal[3] = 0;
    }
}

__global__ void k_filter_nblocks(FilterWs w) { w.scal[6] = (w.scal[3] + kCaseTile - 1) / kCaseTile; }

// case table of the kept events (their count is on the device)
__global__ __launch_bounds__(256) void k_filter_case_count(const int32_t* __restrict__ c, FilterWs w,
                                                           uint32_t* blockcnt, int64_t nbmax) {
    __shared__ uint32_t tmp[256 / kWave + 1];
    const int64_t n = w.scal[3];
    const int64_t nb = (n + kCaseTile - 1) / kCaseTile;
    for (int64_t b = blockIdx.x; b < nb && b < nbmax; b += gridDim.x) {
        uint32_t cnt = 0;
        for (int k = 0; k < kCaseTile / 256; ++k) {
            const int64_t i = b * kCaseTile + k * 256 + threadIdx.x;
            if (i < n && (i == 0 || c[i] != c[i - 1])) ++cnt;
        }
        uint32_t total;
        block_excl_sum<256>(cnt, tmp, &total);
        if (threadIdx.x == 0) blockcnt[b] = total;
    }
}

__global__ __launch_bounds__(256) void k_filter_case_emit(const int32_t* __restrict__ c, FilterWs w,
                                                          const int64_t* blockoff, int64_t* __restrict__ case_off,
                                                          int32_t* __restrict__ case_code, int64_t* n_cases) {
    constexpr int kCI = kCaseTile / 256;
    __shared__ uint32_t wcnt[kCI][256 / kWave];
    const int64_t n = w.scal[3];
    const int64_t nb = (n + kCaseTile - 1) / kCaseTile;
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int64_t base = b * kCaseTile + threadIdx.x;
        striped_compact<256, kCI>(
            blockoff[b], wcnt,
            [&](int q) {
                const int64_t i = base + (int64_t)q * 256;
                return i < n && (i == 0 || c[i] != c[i - 1]);
            },
            [&](int q, int64_t o) {
                const int64_t i = base + (int64_t)q * 256;
                case_off[o] = i;
                case_code[o] = c[i];
            });
    }
}

__global__ void k_filter_case_done(FilterWs w, const int64_t* ncase_total, int64_t* case_off, int64_t* n_cases,
                                   int32_t* status, const int32_t* status_in) {
    const int64_t C = *ncase_total;
    case_off[C] = w.scal[3];
    *n_cases = C;
    *status = (status_in && *status_in) ? *status_in : (w.scal[7] ? PM4G_E_CAPACITY : 0);
}

// Kept events of the slice in scal[0..2] -> out (events, then their case table).
template <class Pred>
void filter_compact(const pm4g_prepared* p, Pred pred, const pm4g_prepared* out, FilterWs w, bool cap_after_count,
                    unsigned grid, hipStream_t s) {
    const int64_t n = p->n_events;
    k_filter_count<<<grid, kFB, 0, s>>>(pred, w);
    // tile offsets: tile_cnt has scal[2] valid entries; total -> scal[3]
    dev::excl_scan<int64_t>(w.tile_cnt, &w.scal[2], w.tile_off, w.part64, &w.scal[3], s);
    if (cap_after_count) k_filter_cap<<<1, 1, 0, s>>>(out->n_events, w);
    k_filter_emit<<<grid, kFB, 0, s>>>(p->case_s, p->act_s, p->ts_s, pred, w, out->case_s, out->act_s, out->ts_s);
    const int64_t nbc = case_blocks(n);
    const unsigned g2 = (unsigned)(nbc < 2048 ? (nbc < 1 ? 1 : nbc) : 2048);
    k_filter_case_count<<<g2, 256, 0, s>>>(out->case_s, w, w.caseblk, nbc + 1);
    // per-block case offsets into tile_off (free again after the emit); total cases -> scal[5]
    k_filter_nblocks<<<1, 1, 0, s>>>(w);
    dev::excl_scan<int64_t>(w.caseblk, &w.scal[6], w.tile_off, w.part64, &w.scal[5], s);
    k_filter_case_emit<<<g2, 256, 0, s>>>(out->case_s, w, w.tile_off, out->case_off, out->case_code, out->n_cases);
    k_filter_case_done<<<1, 1, 0, s>>>(w, &w.scal[5], out->case_off, out->n_cases, out->status, p->status);
}

unsigned filter_grid(int64_t n) {
    const int64_t ntiles = (n + kFilterTile - 1) / kFilterTile;
    return (unsigned)(ntiles < 2048 ? (ntiles < 1 ? 1 : ntiles) : 2048);
}

}  // namespace

hipError_t launch_filter_view(const pm4g_prepared* p, const pm4g_view* view, const uint64_t* mask,
                              const pm4g_prepared* out, FilterWs w, hipStream_t s) {
    ProfScope ps(P_VIEW_FILTER, s);
    k_filter_slice<<<1, 1, 0, s>>>(view, p->case_off, p->case_code, p->n_cases, out->n_events, w);
    filter_compact(p, ViewPred{view, mask, p->act_s, p->ts_s}, out, w, false, filter_grid(p->n_events), s);
    return hipGetLastError();
}

hipError_t launch_sample_events(const pm4g_prepared* p, uint64_t seed, const SelState* sel,
                                const pm4g_prepared* out, FilterWs w, hipStream_t s) {
    k_filter_whole<<<1, 1, 0, s>>>(p->n_events, w);
    filter_compact(p, SamplePred{seed, sel}, out, w, true, filter_grid(p->n_events), s);
    return hipGetLastError();
}

hipError_t launch_filter_df_events(const pm4g_prepared* p, const uint64_t* pairs, int32_t side, int32_t keep,
                                   const pm4g_prepared* out, FilterWs w, hipStream_t s) {
    ProfScope ps(P_DF_FILTER, s);
    k_filter_whole<<<1, 1, 0, s>>>(p->n_events, w);
    filter_compact(p, PairPred{p->case_s, p->act_s, pairs, p->n_events, p->n_activities, side, keep}, out, w,
                   true, filter_grid(p->n_events), s);
    return hipGetLastError();
}

}  // namespace pm4g
