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
// the columns the predicate did not read (and 16 written) per kept event.
// Each pass issues all loads of a stretch of positions before it uses any
// (clamped positions, no branch around a load), then the bit-set words, then
// decides.
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
// read device memory).  A predicate names the columns it reads (kC, kA, kT:
// case, activity, timestamp; kPartner: the case and activity of the event's
// neighbour) and whether it looks a bit up in a bit set (kBits).  The kernels
// load the columns first, for all their positions at once, into Rows; then
// prep(row, i, in) gives the bit set's word to read (and keeps the bit in the
// row), the words of all positions are read at once, and decide(row, word, i,
// in) answers for position i of the log, which is in the slice when `in` is
// set (out-of-slice positions answer false).  The 64 lanes of a wave call
// prep together on consecutive positions.
struct Row {
    int32_t c, a;
    int64_t t;
    int32_t cj, aj;   // the neighbour's case and activity (kPartner)
    int32_t bit;      // bit within the looked-up word, -1: none
};

// Every step of one predicate over kN positions of a thread (base + q*kFB):
// prep, the bit-set words (all issued together), decide.
template <int kN, class Pred, class Ready>
__device__ __forceinline__ void decide_all(const Ready& keep, Row (&x)[kN], int64_t base, int64_t p1,
                                           bool (&flag)[kN]) {
    int64_t ix[kN];
#pragma unroll
    for (int q = 0; q < kN; ++q) {
        const int64_t i = base + (int64_t)q * kFB;
        ix[q] = keep.prep(x[q], i, i < p1);
    }
    uint64_t wd[kN];
#pragma unroll
    for (int q = 0; q < kN; ++q) wd[q] = Pred::kBits ? keep.bits()[ix[q]] : 0ull;
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < kN; ++q) {
        const int64_t i = base + (int64_t)q * kFB;
        flag[q] = keep.decide(x[q], wd[q], i, i < p1);
    }
}

struct ViewPred {
    static constexpr bool kC = false, kA = true, kT = true, kPartner = false, kBits = true;
    const pm4g_view* view;
    const uint64_t* mask;
    struct Ready {
        pm4g_view v;
        const uint64_t* mask;
        __device__ __forceinline__ int64_t partner(int64_t) const { return 0; }
        __device__ __forceinline__ const uint64_t* bits() const { return mask; }
        __device__ __forceinline__ int64_t prep(Row& x, int64_t, bool in) const {
            x.bit = x.a & 63;
            return in ? (x.a >> 6) : 0;
        }
        __device__ __forceinline__ bool decide(const Row& x, uint64_t word, int64_t, bool in) const {
            return in && x.t >= v.t_lo && x.t <= v.t_hi && ((word >> x.bit) & 1ull);
        }
    };
    __device__ __forceinline__ Ready ready() const { return Ready{*view, mask}; }
};

// Directly-follows level: the pair an event forms with the previous (side 0)
// or next (side 1) event of its case, looked up in a bit set over src*A+dst.
// Its slice is the whole log (positions 0..n-1), so the partner of an event,
// when it exists, sits in the neighbouring lane, except at the wave's edge,
// whose lane takes the partner's loaded values (every lane loads them, at a
// clamped position, so that no load waits behind a branch).
struct PairPred {
    static constexpr bool kC = true, kA = true, kT = false, kPartner = true, kBits = true;
    const uint64_t* pairs;
    int64_t n;
    int32_t A;
    int32_t side;
    int32_t keep;
    __device__ __forceinline__ PairPred ready() const { return *this; }
    __device__ __forceinline__ int64_t partner(int64_t i) const {
        const int64_t j = side ? i + 1 : i - 1;
        return j < 0 ? 0 : (j >= n ? n - 1 : j);
    }
    __device__ __forceinline__ const uint64_t* bits() const { return pairs; }
    __device__ __forceinline__ int64_t prep(Row& x, int64_t i, bool in) const {
        const int32_t c = in ? x.c : 0;
        const int32_t a = in ? x.a : 0;
        const int64_t j = side ? i + 1 : i - 1;   // partner position
        int32_t cj = side ? __shfl_down(c, 1) : __shfl_up(c, 1);
        int32_t aj = side ? __shfl_down(a, 1) : __shfl_up(a, 1);
        const bool has = in && j >= 0 && j < n;
        const bool edge = side ? lane() == kWave - 1 : lane() == 0;
        if (edge && has) {
            cj = x.cj;
            aj = x.aj;
        }
        x.bit = -1;
        if (!(has && cj == c)) return 0;
        const int64_t src = side ? a : aj;
        const int64_t dst = side ? aj : a;
        const int64_t cell = src * A + dst;
        x.bit = (int32_t)(cell & 63);
        return cell >> 6;
    }
    __device__ __forceinline__ bool decide(const Row& x, uint64_t word, int64_t, bool in) const {
        const bool match = x.bit >= 0 && ((word >> x.bit) & 1ull);
        return in && (keep ? match : !match);
    }
};

// Sampling by events: a position is kept iff its SplitMix64 key is at most
// the selected threshold.
struct SamplePred {
    static constexpr bool kC = false, kA = false, kT = false, kPartner = false, kBits = false;
    uint64_t seed;
    const SelState* sel;
    struct Ready {
        uint64_t seed, T;
        int32_t none, all;
        __device__ __forceinline__ int64_t partner(int64_t) const { return 0; }
        __device__ __forceinline__ const uint64_t* bits() const { return nullptr; }
        __device__ __forceinline__ int64_t prep(Row&, int64_t, bool) const { return 0; }
        __device__ __forceinline__ bool decide(const Row&, uint64_t, int64_t i, bool in) const {
            return in && !none && (all || splitmix64(seed, (uint64_t)i) <= T);
        }
    };
    __device__ __forceinline__ Ready ready() const { return Ready{seed, sel->T, sel->none, sel->all}; }
};

// The columns a predicate (or the copy, ALL) needs at position i, or at the
// in-bounds position `safe` when i is past the slice: plain loads with no
// branch around them.
template <class Pred, bool ALL, class Ready>
__device__ __forceinline__ Row load_row(const Ready& keep, const int32_t* __restrict__ case_s,
                                        const int32_t* __restrict__ act_s, const int64_t* __restrict__ ts_s,
                                        int64_t i, bool in, int64_t safe) {
    Row x{0, 0, 0, 0, 0, -1};
    const int64_t ic = in ? i : safe;
    if (ALL || Pred::kC) x.c = case_s[ic];
    if (ALL || Pred::kA) x.a = act_s[ic];
    if (ALL || Pred::kT) x.t = ts_s[ic];
    if (Pred::kPartner) {
        const int64_t jc = keep.partner(ic);
        x.cj = case_s[jc];
        x.aj = act_s[jc];
    }
    return x;
}

template <class Pred>
__global__ __launch_bounds__(kFB) void k_filter_count(Pred pred, const int32_t* __restrict__ case_s,
                                                      const int32_t* __restrict__ act_s,
                                                      const int64_t* __restrict__ ts_s, FilterWs w) {
    __shared__ uint32_t tmp[kFB / kWave + 1];
    const auto keep = pred.ready();
    const int64_t p0 = w.scal[0], p1 = w.scal[1], nt = w.scal[2];
    const int64_t safe = p1 > p0 ? p1 - 1 : 0;
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        Row x[kFI];
#pragma unroll
        for (int q = 0; q < kFI; ++q) {
            const int64_t i = p0 + t * kFilterTile + q * kFB + threadIdx.x;
            x[q] = load_row<Pred, false>(keep, case_s, act_s, ts_s, i, i < p1, safe);
        }
        __builtin_amdgcn_sched_barrier(0);
        bool f[kFI];
        decide_all<kFI, Pred>(keep, x, p0 + t * kFilterTile + threadIdx.x, p1, f);
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < kFI; ++q) c += f[q] ? 1u : 0u;
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
// Returns r0 plus the tile's kept count.
template <int kB, int kPer, class Flag, class Emit>
__device__ __forceinline__ int64_t striped_compact(int64_t r0, uint32_t (*wcnt)[kB / kWave], Flag flag, Emit emit) {
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
    return r;
}

template <class Pred>
__global__ __launch_bounds__(kFB) void k_filter_emit(const int32_t* __restrict__ case_s,
                                                     const int32_t* __restrict__ act_s,
                                                     const int64_t* __restrict__ ts_s, Pred pred, FilterWs w,
                                                     int32_t* __restrict__ o_case, int32_t* __restrict__ o_act,
                                                     int64_t* __restrict__ o_ts) {
    constexpr int kHalf = kFI / 2;   // stripes per half tile: all loads of a half are issued together
    __shared__ uint32_t wcnt[kHalf][kFB / kWave];
    const auto keep = pred.ready();
    const int64_t p0 = w.scal[0], p1 = w.scal[1], nt = w.scal[2];
    const int64_t safe = p1 > p0 ? p1 - 1 : 0;
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        int64_t r = w.tile_off[t];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t base = p0 + t * kFilterTile + (int64_t)h * kHalf * kFB + threadIdx.x;
            // 1. the predicate's columns, all positions of the half at once
            Row x[kHalf];
#pragma unroll
            for (int q = 0; q < kHalf; ++q) {
                const int64_t i = base + (int64_t)q * kFB;
                x[q] = load_row<Pred, false>(keep, case_s, act_s, ts_s, i, i < p1, safe);
            }
            __builtin_amdgcn_sched_barrier(0);
            // 2. kept flags and output places
            bool f[kHalf];
            decide_all<kHalf, Pred>(keep, x, base, p1, f);
            int64_t o[kHalf];
#pragma unroll
            for (int q = 0; q < kHalf; ++q) o[q] = -1;
            r = striped_compact<kFB, kHalf>(
                r, wcnt, [&](int q) { return f[q]; }, [&](int q, int64_t at) { o[q] = at; });
            // 3. the other columns of the kept events, then the stores
#pragma unroll
            for (int q = 0; q < kHalf; ++q) {
                const int64_t i = base + (int64_t)q * kFB;
                if (o[q] >= 0) {
                    if (!Pred::kC) x[q].c = case_s[i];
                    if (!Pred::kA) x[q].a = act_s[i];
                    if (!Pred::kT) x[q].t = ts_s[i];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < kHalf; ++q) {
                if (o[q] >= 0) {
                    o_case[o[q]] = x[q].c;
                    o_act[o[q]] = x[q].a;
                    o_ts[o[q]] = x[q].t;
                }
            }
        }
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
        // loads at clamped positions (n >= 1 here), all issued before any is used
        constexpr int kCI = kCaseTile / 256;
        int32_t cv[kCI], pv[kCI];
#pragma unroll
        for (int k = 0; k < kCI; ++k) {
            const int64_t i = b * kCaseTile + k * 256 + threadIdx.x;
            const int64_t ic = i < n ? i : n - 1;
            cv[k] = c[ic];
            pv[k] = c[ic > 0 ? ic - 1 : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
        uint32_t cnt = 0;
#pragma unroll
        for (int k = 0; k < kCI; ++k) {
            const int64_t i = b * kCaseTile + k * 256 + threadIdx.x;
            if (i < n && (i == 0 || cv[k] != pv[k])) ++cnt;
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
        // loads at clamped positions (n >= 1 here), all issued before any is used
        int32_t cv[kCI], pv[kCI];
#pragma unroll
        for (int q = 0; q < kCI; ++q) {
            const int64_t i = base + (int64_t)q * 256;
            const int64_t ic = i < n ? i : n - 1;
            cv[q] = c[ic];
            pv[q] = c[ic > 0 ? ic - 1 : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
        striped_compact<256, kCI>(
            blockoff[b], wcnt,
            [&](int q) {
                const int64_t i = base + (int64_t)q * 256;
                return i < n && (i == 0 || cv[q] != pv[q]);
            },
            [&](int q, int64_t o) {
                const int64_t i = base + (int64_t)q * 256;
                case_off[o] = i;
                case_code[o] = cv[q];
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
    k_filter_count<<<grid, kFB, 0, s>>>(pred, p->case_s, p->act_s, p->ts_s, w);
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
    filter_compact(p, ViewPred{view, mask}, out, w, false, filter_grid(p->n_events), s);
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
    filter_compact(p, PairPred{pairs, p->n_events, p->n_activities, side, keep}, out, w,
                   true, filter_grid(p->n_events), s);
    return hipGetLastError();
}

}  // namespace pm4g
