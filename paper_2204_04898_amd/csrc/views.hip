// Batched drill-down views over a prepared log (Sec. 1 drill-down: each view
// is a filtered part of the log; Sec. 3: event-level timestamp filter,
// attribute filter on the activity, and the DFG re-discovered on what is kept).
//
// A view v keeps event i iff case_lo <= c_i < case_hi, t_lo <= t_i <= t_hi and
// bit a_i of its activity mask is set.  Its DFG pairs each kept event with the
// previous kept event of the same case.  Every kept event is either the first
// kept event of its case (a start) or the destination of exactly one pair, and
// either the last one (an end) or the source of exactly one pair, so
//   act_count(y) = start(y) + sum_x count(x, y),  end(x) = act_count(x) - sum_y count(x, y).
//
// Pipeline (sizes stay on the device and so do the capacity checks: the call
// never waits for the device; when a capacity is short, the kernels after the
// check return at once and the status word and the required sizes say so):
//   k_view_slice     case range -> event slice [p0, p1) (binary search in the
//                    case table); a slice always holds whole cases
//   k_view_tile_scan per-tile counts of overlapping views, offsets
//   k_view_fill      per-tile lists of overlapping views
//   k_view_count /   tile-major: a block stages one tile of the log in LDS;
//   k_view_write     each wave takes one overlapping view and walks the tile:
//                    the view's predicate lists the kept positions (ballots),
//                    and the kept events, 64 at a time, find the previous kept
//                    event in the neighbouring lane, carried across groups and
//                    (by a backward search) across tiles.  A pair gives a
//                    record (cell = x*A+y, gap); a start gives (A*A + y, 0).
//                    The walk runs twice:
//                    count per cell bucket (cell >> 12) and take each run's
//                    place in its (view, bucket) segment with one atomic (kept
//                    per (tile, view, bucket)), then write the runs
//   scans            (view, bucket) counters -> segment places; non-empty
//                    pairs -> the segment list
//   k_view_agg       one block per (view, bucket) segment: 4096-cell LDS table;
//                    non-empty pair cells -> temporary sparse records, start
//                    cells -> start counts
//   scans, copy      per-view lists ordered by (src, dst), offsets, FP64 mean
//   k_view_acts      per view: activity and end counts from the start counts
//                    and the row / column sums
#include <math.h>

#include <atomic>
#include <random>

#include "common.hpp"
#include "devsort.hpp"
#include "internal.hpp"
#include "prof.hpp"
#include "../../include/pm4g.h"

namespace pm4g {

namespace {

constexpr int kVB = 512;                  // threads per emit block (8 waves)
constexpr int kVW = kVB / kWave;
constexpr int kMaxBuckets = 264;          // >= ceil(1024 * 1025 / 4096) = 257
constexpr int kMaskWords = PM4G_BATCHED_MAX_ACTIVITIES / 64;
constexpr int kAB2 = 1024;                // threads per aggregation block
constexpr int kFT = 1024;                 // threads per block of the persistent launch
constexpr uint64_t kRecGapLimit = 1ull << 52;   // gaps below it share a u64 with the cell

// A phase's view of the grid: block bid of nblk.  A phase launched as a
// kernel of its own takes blockIdx / gridDim; the single persistent launch
// runs every phase on its own grid, with grid barriers in between.
struct Grid {
    int64_t bid, nblk;
};
__device__ __forceinline__ Grid hw_grid() { return Grid{(int64_t)blockIdx.x, (int64_t)gridDim.x}; }


// Value of lane l (l the same in every lane: read into a scalar register, no
// LDS round trip as a shuffle would take).
__device__ __forceinline__ int32_t lane_i32(int32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ int64_t lane_i64(int64_t v, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

}  // namespace

int64_t view_buckets(int32_t A) {
    return ((int64_t)A * (A + 1) + kCellsPerTable - 1) / kCellsPerTable;
}

ViewWs view_ws_layout(Bump& b, int64_t n, int32_t A, int32_t V, int32_t tile, int64_t pair_cap,
                      int64_t rec_cap, int64_t cell_cap) {
    ViewWs w{};
    const size_t cc = (size_t)(cell_cap > 0 ? cell_cap : 1);
    w.cell_cap = cell_cap;
    const int64_t tiles = (n + tile - 1) / tile;
    const size_t vm = (size_t)(V > 0 ? V : 1);
    const size_t rc = (size_t)(rec_cap > 0 ? rec_cap : 1);
    w.tile = tile;
    w.n_tiles = tiles;
    w.n_buckets = (int32_t)view_buckets(A);
    w.pair_cap = pair_cap;
    w.rec_cap = rec_cap;
    w.p0 = b.take<int64_t>(vm);
    w.p1 = b.take<int64_t>(vm);
    w.tcount = b.take<uint32_t>((size_t)tiles + 2);
    w.toff = b.take<uint32_t>((size_t)tiles + 2);
    w.tcursor = b.take<uint32_t>((size_t)tiles + 2);
    w.list = b.take<uint32_t>((size_t)(pair_cap > 0 ? pair_cap : 1));
    w.scal = b.take<int64_t>(16);
    w.part32 = b.take<uint32_t>(dev::kScanGrid);
    w.part64 = b.take<int64_t>(dev::kScanGrid);
    w.part64b = b.take<int64_t>(dev::kScanGrid);
    w.bar = b.take<uint64_t>(kViewMaxBlocks + 1);
    w.rec_cell = b.take<uint16_t>(rc);
    w.rec_gap = b.take<uint64_t>(rc);
    w.pair_carry = b.take<uint4>((size_t)(pair_cap > 0 ? pair_cap : 1));
    w.pair_rel = b.take<uint32_t>((size_t)(pair_cap > 0 ? pair_cap : 1) * (size_t)w.n_buckets);
    w.n_vb = (int64_t)(V > 0 ? V : 0) * w.n_buckets;
    const size_t nvb = (size_t)(w.n_vb > 0 ? w.n_vb : 1);
    w.vb_cnt = b.take<uint32_t>(nvb);
    w.vb_base = b.take<int64_t>(nvb);
    w.vb_flag = b.take<uint32_t>(nvb);
    w.vb_seg = b.take<uint32_t>(nvb);
    w.seg_key = b.take<uint32_t>(nvb);
    w.seg_rec = b.take<int64_t>(nvb + 1);
    w.seg_cells = b.take<uint32_t>(nvb);
    w.seg_tmp = b.take<int64_t>(nvb);
    w.seg_out = b.take<int64_t>(nvb);
    w.view_cells = b.take<uint32_t>(vm);
    w.t_cell = b.take<uint32_t>(cc);
    w.t_count = b.take<uint32_t>(cc);
    w.t_sum = b.take<uint64_t>(cc);
    w.t_min = b.take<int64_t>(cc);
    w.t_max = b.take<int64_t>(cc);
    return w;
}

namespace {

// scal: [2] #segments (u32 total written at [8] as u32 by the scan, copied
// here), [3] temporary cell cursor, [4] total output cells, [6] #views, [7]
// #pairs, [9] records (scan total), [10] nonzero when some case lasts 2^52
// time units or more (records then keep the cell in a separate array), [11]
// (view, bucket) pairs, [12] the gate after the count walk: 0, or the status
// that stops the call
//
// Record places.  The count walk adds each (tile, view) pair's records per
// bucket to the (view, bucket) counter with one atomic, whose old value is the
// run's place inside that (view, bucket) segment (kept per pair and bucket);
// an exclusive scan of the counters in (view, bucket) order gives the
// segments' places, so every segment's records form one contiguous range in
// (view, bucket) order.
//
// Records.  A record's gap is at most its case's duration, so when every case
// of the log lasts less than 2^52 units a record is one u64 in rec_gap:
// cell within its bucket (12 bits) << 52 | gap.  Otherwise the cell goes to
// rec_cell and the full gap to rec_gap.

__device__ __forceinline__ void ph_init(Grid gd, ViewWs w, int32_t V, int32_t A, const int32_t* status_in,
                                        BatchedOutDev out) {
    const int64_t stride = (int64_t)gd.nblk * blockDim.x;
    const int64_t i0 = (int64_t)gd.bid * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < w.n_tiles + 2; i += stride) {
        w.tcount[i] = 0;
        w.tcursor[i] = 0;
    }
    for (int64_t i = i0; i < V; i += stride) w.view_cells[i] = 0;
    for (int64_t i = i0; i < w.n_vb; i += stride) w.vb_cnt[i] = 0;
    for (int64_t i = i0; i < (int64_t)V * A; i += stride) out.start_count[i] = 0;
    if (i0 < 16) w.scal[i0] = i0 == 11 ? w.n_vb : 0;
    if (i0 == 0) {
        *out.status = (status_in && *status_in) ? *status_in : 0;
        out.required[0] = 0;
        out.required[1] = 0;
        out.required[2] = 0;
        out.required[3] = 0;
        out.required[4] = 0;
    }
}

__global__ void k_view_init(ViewWs w, int32_t V, int32_t A, const int32_t* status_in, BatchedOutDev out) {
    ph_init(hw_grid(), w, V, A, status_in, out);
}

// Sets scal[10] when a case of the log lasts 2^52 time units or more (its
// last timestamp minus its first; the prepared log is sorted by (case, ts)).
__device__ __forceinline__ void ph_span(Grid gd, const int64_t* __restrict__ case_off,
                                        const int64_t* __restrict__ ts_s, const int64_t* n_cases, ViewWs w) {
    const int64_t C = *n_cases;
    bool wide = false;
    for (int64_t c = (int64_t)gd.bid * blockDim.x + threadIdx.x; c < C;
         c += (int64_t)gd.nblk * blockDim.x) {
        const uint64_t d = (uint64_t)ts_s[case_off[c + 1] - 1] - (uint64_t)ts_s[case_off[c]];
        wide |= d >= kRecGapLimit;
    }
    if (__ballot(wide) != 0 && lane() == 0) atomicOr(reinterpret_cast<unsigned long long*>(&w.scal[10]), 1ull);
}

__global__ void k_view_span(const int64_t* __restrict__ case_off, const int64_t* __restrict__ ts_s,
                            const int64_t* n_cases, ViewWs w) {
    ph_span(hw_grid(), case_off, ts_s, n_cases, w);
}

__device__ int64_t lower_bound_i32(const int32_t* a, int64_t n, int32_t x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Event slice of every view (whole cases) and the per-tile overlap differences.
__device__ __forceinline__ void ph_slice(Grid gd, const pm4g_view* views, int32_t V, const int64_t* case_off,
                                         const int32_t* case_code, const int64_t* n_cases, ViewWs w) {
    const int64_t C = *n_cases;
    for (int64_t v = (int64_t)gd.bid * blockDim.x + threadIdx.x; v < V;
         v += (int64_t)gd.nblk * blockDim.x) {
        const pm4g_view vw = views[v];
        int64_t p0 = 0, p1 = 0;
        if (vw.case_lo < vw.case_hi && vw.t_lo <= vw.t_hi) {
            p0 = case_off[lower_bound_i32(case_code, C, vw.case_lo)];
            p1 = case_off[lower_bound_i32(case_code, C, vw.case_hi)];
        }
        w.p0[v] = p0;
        w.p1[v] = p1;
        if (p1 > p0) {
            atomicAdd(&w.tcount[p0 / w.tile], 1u);
            atomicAdd(&w.tcount[(p1 - 1) / w.tile + 1], 0xFFFFFFFFu);   // -1
        }
    }
}

__global__ void k_view_slice(const pm4g_view* views, int32_t V, const int64_t* case_off,
                             const int32_t* case_code, const int64_t* n_cases, ViewWs w) {
    ph_slice(hw_grid(), views, V, case_off, case_code, n_cases, w);
}

// tcount holds differences; one block turns them into counts and offsets.
__device__ __forceinline__ void ph_tile_scan(Grid gd, ViewWs w) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
    if (gd.bid != 0) return;   // one block (of 1024 threads)
    uint32_t run_cnt = 0, run_off = 0;
    const int64_t nt = w.n_tiles;
    for (int64_t t0 = 0; t0 < nt; t0 += 1024) {
        const int64_t t = t0 + threadIdx.x;
        const uint32_t d = t < nt ? w.tcount[t] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_sum<1024>(d, tmp, &total);
        const uint32_t cnt = run_cnt + ex + d;
        uint32_t total2;
        const uint32_t ex2 = block_excl_sum<1024>(t < nt ? cnt : 0u, tmp, &total2);
        if (t < nt) {
            w.tcount[t] = cnt;
            w.toff[t] = run_off + ex2;
        }
        run_cnt += total;
        run_off += total2;
    }
    if (threadIdx.x == 0) {
        w.toff[nt] = run_off;
        w.scal[7] = run_off;
    }
}

__global__ __launch_bounds__(1024) void k_view_tile_scan(ViewWs w) { ph_tile_scan(hw_grid(), w); }

// One wave per view, its lanes over the view's tiles (a view can span
// thousands of tiles; one thread per view made that a serial atomic chain).
__device__ __forceinline__ void ph_fill(Grid gd, int32_t V, ViewWs w) {
    const int64_t wv = ((int64_t)gd.bid * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gd.nblk * blockDim.x / kWave;
    for (int64_t v = wv; v < V; v += nw) {
        const int64_t p0 = w.p0[v], p1 = w.p1[v];
        if (p1 <= p0) continue;
        const int64_t t1 = (p1 - 1) / w.tile;
        for (int64_t t = p0 / w.tile + lane(); t <= t1; t += kWave) {
            const int64_t at = (int64_t)w.toff[t] + atomicAdd(&w.tcursor[t], 1u);
            if (at < w.pair_cap) w.list[at] = (uint32_t)v;
        }
    }
}

__global__ void k_view_fill(int32_t V, ViewWs w) { ph_fill(hw_grid(), V, w); }

__device__ __forceinline__ bool kept(int32_t a, int64_t t, int64_t tlo, int64_t thi, const uint64_t* mask) {
    return t >= tlo && t <= thi && ((mask[a >> 6] >> (a & 63)) & 1ull);
}

struct WalkState {
    bool have_cur;   // the position before the window is in the slice
    int32_t cur;     // ... and its case
    bool cr_valid;   // a kept event of case `cur` precedes the window
    int32_t cr_a;
    int64_t cr_t;
};

// Initial state for a walk that starts at e0 inside slice [p0, p1): the case at
// e0 - 1 and, if it continues at e0, its last kept event before e0.
__device__ WalkState walk_init(const int32_t* case_s, const int32_t* act_s, const int64_t* ts_s,
                               int64_t e0, int64_t p0, int64_t tlo, int64_t thi, const uint64_t* mask) {
    WalkState st{false, 0, false, 0, 0};
    if (e0 <= p0) return st;   // slices start at a case start
    st.have_cur = true;
    st.cur = case_s[e0 - 1];
    if (case_s[e0] != st.cur) return st;
    for (int64_t hi = e0; hi > p0; hi -= kWave) {
        const int64_t i = hi - 1 - lane();
        bool same = false, k = false;
        int32_t a = 0;
        int64_t t = 0;
        if (i >= p0) {
            same = case_s[i] == st.cur;
            if (same) {
                a = act_s[i];
                t = ts_s[i];
                k = kept(a, t, tlo, thi, mask);
            }
        }
        const uint64_t kb = __ballot(k);
        const int l = kb ? (__ffsll((long long)kb) - 1) : 0;   // lowest lane = latest position
        const int32_t al = __shfl(a, l);
        const int64_t tl = __shfl(t, l);
        if (kb) {
            st.cr_valid = true;
            st.cr_a = al;
            st.cr_t = tl;
            return st;
        }
        if (__ballot(i >= p0 && !same) != 0) return st;   // reached the case start
    }
    return st;
}

// One walk over [e0, e1) of the staged tile (T0 = first position of the tile),
// in rounds of kSub events.  Pass 1 tests the view's predicate on the round's
// events and appends the kept positions to the wave's list; pass 2 takes the
// listed kept events 64 at a time (a partial group waits for the next round,
// except in the last one): lane l's previous kept event of the slice is lane
// l - 1's (a DPP shift; lane 0 takes the carry, the last kept event before
// the group), and the event starts its case's kept events iff that previous
// one lies in another case or does not exist (cases are contiguous).  Every
// kept event yields one record: WRITE=false counts per bucket in cursor[],
// WRITE=true takes record places from cursor[] (each bucket's cursor starts
// at its run) and writes the records.
constexpr int kSub = 512;             // events per round (8 windows of 64)
constexpr int kList = kSub + kWave;   // a round's kept positions plus the previous round's rest
constexpr int kListAlloc = kList + kWave;   // and a slot per lane for the events not kept

// Pass 1 over [r0, r1) (FULL: r1 = r0 + kSub): all loads issued before any
// use; returns the list length.  mask32: the view's activity mask as 32-bit
// words (bit a of the mask is bit a & 31 of word a >> 5).
template <bool FULL>
__device__ __forceinline__ int list_kept(const int16_t* __restrict__ s_act, const int64_t* __restrict__ s_ts,
                                         int r0, int r1, int64_t tlo, int64_t thi,
                                         const uint32_t* __restrict__ mask32, uint16_t* __restrict__ list, int n) {
    constexpr int kU = kSub / kWave;
    int32_t av[kU];
    int64_t tv[kU];
    uint32_t mv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int i = r0 + u * kWave + lane();
        const int ii = FULL ? i : (i < r1 ? i : r1 - 1);   // past the round: its last event, not kept
        av[u] = s_act[ii];
        tv[u] = s_ts[ii];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) mv[u] = mask32[av[u] >> 5];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        // one ballot per comparison (each folds to the comparison's lane
        // mask); every lane stores, the kept ones at their list place, the
        // others at their own slot past the list (no branch)
        const int i = r0 + u * kWave + lane();
        const bool ki = FULL || i < r1;
        const bool ka = __builtin_amdgcn_ubfe(mv[u], (uint32_t)av[u], 1u) != 0;   // bit a & 31
        const bool k1 = tv[u] >= tlo;
        const bool k2 = tv[u] <= thi;
        uint64_t K = __builtin_amdgcn_ballot_w64(ka) & __builtin_amdgcn_ballot_w64(k1) &
                     __builtin_amdgcn_ballot_w64(k2);
        if (!FULL) K &= __builtin_amdgcn_ballot_w64(ki);
        const uint32_t at = __builtin_amdgcn_mbcnt_hi((uint32_t)(K >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)K, 0u));
        list[(ki & ka & k1 & k2) ? (uint32_t)n + at : (uint32_t)(kList + lane())] = (uint16_t)i;
        n += __popcll(K);
    }
    return n;
}

struct KeptEv {
    int32_t c, a;
    int64_t t;
};

__device__ __forceinline__ KeptEv kept_event(const int32_t* __restrict__ s_case, const int16_t* __restrict__ s_act,
                                             const int64_t* __restrict__ s_ts, const uint16_t* __restrict__ list,
                                             int j, int n) {
    KeptEv e{0, 0, 0};
    if (j < n) {
        const int q = list[j];
        e.c = s_case[q];
        e.a = s_act[q];
        e.t = s_ts[q];
    }
    return e;
}

template <bool WRITE>
__device__ __forceinline__ void walk(const int32_t* __restrict__ s_case, const int16_t* __restrict__ s_act,
                                     const int64_t* __restrict__ s_ts, int64_t T0, int64_t e0, int64_t e1,
                                     WalkState st, int32_t A, int64_t tlo, int64_t thi,
                                     const uint64_t* __restrict__ mask, uint16_t* __restrict__ list,
                                     uint32_t* __restrict__ cursor, uint16_t* __restrict__ rec_cell,
                                     uint64_t* __restrict__ rec_gap, bool wide) {
    const int32_t AA = A * A;
    const uint32_t* mask32 = reinterpret_cast<const uint32_t*>(mask);
    // carry: the last kept event of the slice before the current group
    bool pv = st.cr_valid;
    int32_t pc = st.cur, pa = st.cr_a;
    int64_t pt = st.cr_t;
    int n = 0;   // listed kept positions (wave-uniform)
    const int b1 = (int)(e1 - T0);
    for (int r0 = (int)(e0 - T0); r0 < b1; r0 += kSub) {
        const int r1 = r0 + kSub < b1 ? r0 + kSub : b1;
        if (r1 - r0 == kSub) n = list_kept<true>(s_act, s_ts, r0, r1, tlo, thi, mask32, list, n);
        else n = list_kept<false>(s_act, s_ts, r0, r1, tlo, thi, mask32, list, n);
        __builtin_amdgcn_wave_barrier();
        const bool last = r1 >= b1;
        int c0 = 0;
        for (; c0 + kWave <= n || (last && c0 < n); c0 += kWave) {
            const bool in = c0 + lane() < n;
            const KeptEv e = kept_event(s_case, s_act, s_ts, list, c0 + lane(), n);
            // lane l - 1's event: a DPP wave shift right by one, whose lane 0
            // (no source lane) keeps the first operand, the carry
            const int32_t cq = __builtin_amdgcn_update_dpp(pc, e.c, 0x138, 0xF, 0xF, false);
            const int32_t aq = __builtin_amdgcn_update_dpp(pa, e.a, 0x138, 0xF, 0xF, false);
            const uint32_t tql = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)pt, (int)(uint32_t)e.t,
                                                                       0x138, 0xF, 0xF, false);
            const uint32_t tqh = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)((uint64_t)pt >> 32),
                                                                       (int)(uint32_t)((uint64_t)e.t >> 32),
                                                                       0x138, 0xF, 0xF, false);
            const uint64_t tq = ((uint64_t)tqh << 32) | tql;
            const bool starts = (lane() == 0 && !pv) || e.c != cq;
            if (in) {
                const int32_t cell = starts ? AA + e.a : aq * A + e.a;
                const uint64_t gap = starts ? 0ull : (uint64_t)e.t - tq;
                const uint32_t slot = atomicAdd(&cursor[(uint32_t)cell >> 12], 1u);
                if (WRITE) {   // slot: the record's place (the cursor starts at its run)
                    const uint64_t qc = (uint64_t)(cell & (kCellsPerTable - 1));
                    if (wide) {
                        rec_cell[slot] = (uint16_t)qc;
                        rec_gap[slot] = gap;
                    } else {
                        rec_gap[slot] = (qc << 52) | gap;
                    }
                }
            }
            const int ll = (n - c0 < kWave ? n - c0 : kWave) - 1;
            pv = true;
            pc = lane_i32(e.c, ll);
            pa = lane_i32(e.a, ll);
            pt = lane_i64(e.t, ll);
        }
        // the rest (fewer than 64) moves to the front of the list
        if (c0 > 0 && c0 < n) {
            const int rest = n - c0;
            uint16_t x = 0;
            if (lane() < rest) x = list[c0 + lane()];
            __builtin_amdgcn_wave_barrier();
            if (lane() < rest) list[lane()] = x;
        }
        n = c0 < n ? n - c0 : 0;
        __builtin_amdgcn_wave_barrier();
    }
}

// LDS of a walk block (NW waves over a TILE-event tile).
template <int TILE, int NW>
struct WalkSmem {
    int32_t s_case[TILE];
    int16_t s_act[TILE];
    int64_t s_ts[TILE];
    uint64_t s_mask[NW][kMaskWords];
    uint32_t s_cur[NW][kMaxBuckets];
    uint16_t s_list[NW][kListAlloc];
    uint32_t s_next;
};

// Tile order of the walks: chunks of kXcdChunk consecutive tiles are dealt
// round-robin to the 8 XCDs (block b runs on XCD b % 8) and an XCD's blocks
// stride over its chunks' tiles, so neighbouring tiles, whose runs of records
// sit side by side in the record segments, are written through the same L2,
// while the chunks keep the XCDs' loads even along the log.  The block's i-th
// tile, or -1 past the end (the order is increasing in i).
constexpr int64_t kXcdChunk = 64;
__device__ __forceinline__ int64_t walk_tile(Grid gd, int64_t i, int64_t n_tiles) {
    const int64_t G = gd.nblk, b = gd.bid;
    int64_t t;
    if (G % 8 != 0) {
        t = b + i * G;
    } else {
        const int64_t x = b % 8, s = b / 8 + i * (G / 8);
        t = ((s / kXcdChunk) * 8 + x) * kXcdChunk + s % kXcdChunk;
    }
    return t < n_tiles ? t : -1;
}

// The tile's (view) pairs are taken in turn by the block's waves: the first
// kVW by wave index, the others from an LDS counter as waves finish theirs.
__device__ __forceinline__ uint32_t next_pair(uint32_t* s_next) {
    uint32_t j = 0;
    if (lane() == 0) j = atomicAdd(s_next, 1u);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)j);
}

// Count walk.  After a view's walk, each non-empty bucket's run takes its
// place in the (view, bucket) segment with one atomic on the segment's
// counter; the walk's initial carry and whether the pair keeps an event are
// kept for the write walk (pair_carry: ts, case, act | valid << 30 | kept << 31).
template <int TILE, int NW>
__device__ __forceinline__ void ph_count(Grid gd, const int32_t* __restrict__ case_s,
                                        const int32_t* __restrict__ act_s,
                                        const int64_t* __restrict__ ts_s, int64_t n, int32_t A,
                                        const pm4g_view* __restrict__ views,
                                        const uint64_t* __restrict__ masks, ViewWs w,
                                        WalkSmem<TILE, NW>& S) {
    int32_t* s_case = S.s_case;
    int16_t* s_act = S.s_act;
    int64_t* s_ts = S.s_ts;
    constexpr int kVB = NW * kWave;

    const int wv = threadIdx.x / kWave;
    const int NB = w.n_buckets;
    const int MW = (A + 63) / 64;
    uint64_t* mask = S.s_mask[wv];
    uint32_t* cur = S.s_cur[wv];
    if (w.scal[7] > w.pair_cap) return;   // the tile lists are incomplete: the gate stops the call
    for (int64_t it = 0, tile; (tile = walk_tile(gd, it, w.n_tiles)) >= 0; ++it) {
        if (w.tcount[tile] == 0) continue;   // no view overlaps the tile (block-uniform)
        const int64_t T0 = tile * TILE;
        const int64_t T1 = (T0 + TILE) < n ? (T0 + TILE) : n;
        for (int64_t i = T0 + threadIdx.x; i < T1; i += kVB) {
            s_case[i - T0] = case_s[i];
            s_act[i - T0] = (int16_t)act_s[i];
            s_ts[i - T0] = ts_s[i];
        }
        if (threadIdx.x == 0) S.s_next = NW;
        __syncthreads();
        const uint32_t cnt = w.tcount[tile];
        const int64_t off = w.toff[tile];
        for (uint32_t j = wv; j < cnt; j = next_pair(&S.s_next)) {
            const uint32_t v = w.list[off + j];
            const pm4g_view vw = views[v];
            const int64_t p0 = w.p0[v], p1 = w.p1[v];
            for (int q = lane(); q < MW; q += kWave) mask[q] = masks[(size_t)v * MW + q];
            const int64_t e0 = T0 > p0 ? T0 : p0;
            const int64_t e1 = T1 < p1 ? T1 : p1;
            const WalkState st = walk_init(case_s, act_s, ts_s, e0, p0, vw.t_lo, vw.t_hi, mask);
            for (int q = lane(); q < NB; q += kWave) cur[q] = 0;
            walk<false>(s_case, s_act, s_ts, T0, e0, e1, st, A, vw.t_lo, vw.t_hi, mask, S.s_list[wv], cur,
                        w.rec_cell, w.rec_gap, false);
            uint32_t* rel = w.pair_rel + (size_t)(off + j) * (size_t)NB;
            uint64_t any = 0;
            for (int q0 = 0; q0 < NB; q0 += kWave) {
                const int q = q0 + lane();
                const uint32_t c = q < NB ? cur[q] : 0u;
                any |= __ballot(c != 0);
                if (c != 0) rel[q] = atomicAdd(&w.vb_cnt[(size_t)v * NB + q], c);
            }
            if (lane() == 0) {
                const uint32_t aw = (uint32_t)(st.cr_valid ? st.cr_a : 0) | (st.cr_valid ? 1u << 30 : 0u) |
                                    (any != 0 ? 1u << 31 : 0u);
                w.pair_carry[off + j] = make_uint4((uint32_t)(uint64_t)st.cr_t, (uint32_t)((uint64_t)st.cr_t >> 32),
                                                   (uint32_t)st.cur, aw);
            }
        }
        __syncthreads();
    }
}

template <int TILE>
__global__ __launch_bounds__(kVB) void k_view_count(const int32_t* __restrict__ case_s,
                                        const int32_t* __restrict__ act_s,
                                        const int64_t* __restrict__ ts_s, int64_t n, int32_t A,
                                        const pm4g_view* __restrict__ views,
                                        const uint64_t* __restrict__ masks, ViewWs w) {
    __shared__ WalkSmem<TILE, kVW> S;
    ph_count<TILE, kVW>(hw_grid(), case_s, act_s, ts_s, n, A, views, masks, w, S);
}

// Write walk: each (tile, view) pair's buckets start at their runs' places in
// the segment-contiguous record layout; the walk starts from the carry the
// count walk found.
template <int TILE, int NW>
__device__ __forceinline__ void ph_write(Grid gd, const int32_t* __restrict__ case_s,
                                        const int32_t* __restrict__ act_s,
                                        const int64_t* __restrict__ ts_s, int64_t n, int32_t A,
                                        const pm4g_view* __restrict__ views,
                                        const uint64_t* __restrict__ masks, ViewWs w,
                                        WalkSmem<TILE, NW>& S) {
    int32_t* s_case = S.s_case;
    int16_t* s_act = S.s_act;
    int64_t* s_ts = S.s_ts;
    constexpr int kVB = NW * kWave;
    constexpr int kQ = (kMaxBuckets + kWave - 1) / kWave;   // buckets per lane

    const int wv = threadIdx.x / kWave;
    const int NB = w.n_buckets;
    const int MW = (A + 63) / 64;
    const bool wide = w.scal[10] != 0;
    uint64_t* mask = S.s_mask[wv];
    uint32_t* cur = S.s_cur[wv];
    if (w.scal[12] != 0) return;   // a capacity is short: no record is written
    for (int64_t it = 0, tile; (tile = walk_tile(gd, it, w.n_tiles)) >= 0; ++it) {
        if (w.tcount[tile] == 0) continue;   // no view overlaps the tile (block-uniform)
        const int64_t T0 = tile * TILE;
        const int64_t T1 = (T0 + TILE) < n ? (T0 + TILE) : n;
        for (int64_t i = T0 + threadIdx.x; i < T1; i += kVB) {
            s_case[i - T0] = case_s[i];
            s_act[i - T0] = (int16_t)act_s[i];
            s_ts[i - T0] = ts_s[i];
        }
        if (threadIdx.x == 0) S.s_next = NW;
        __syncthreads();
        const uint32_t cnt = w.tcount[tile];
        const int64_t off = w.toff[tile];
        for (uint32_t j = wv; j < cnt; j = next_pair(&S.s_next)) {
            const uint4 cy = w.pair_carry[off + j];
            if (!(cy.w >> 31)) continue;   // no kept event
            const uint32_t v = w.list[off + j];
            // the runs' first records (buckets without a run get no record),
            // loaded before anything waits
            const uint32_t* rel = w.pair_rel + (size_t)(off + j) * (size_t)NB;
            const int64_t* vbb = w.vb_base + (size_t)v * NB;
            uint32_t qv[kQ];
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
                const int q = u * kWave + lane();
                qv[u] = q < NB ? (uint32_t)vbb[q] + rel[q] : 0u;
            }
            const pm4g_view vw = views[v];
            const int64_t p0 = w.p0[v], p1 = w.p1[v];
            for (int q = lane(); q < MW; q += kWave) mask[q] = masks[(size_t)v * MW + q];
#pragma unroll
            for (int u = 0; u < kQ; ++u) {
                const int q = u * kWave + lane();
                if (q < NB) cur[q] = qv[u];
            }
            const int64_t e0 = T0 > p0 ? T0 : p0;
            const int64_t e1 = T1 < p1 ? T1 : p1;
            WalkState st;
            st.have_cur = true;
            st.cur = (int32_t)cy.z;
            st.cr_valid = (cy.w >> 30) & 1u;
            st.cr_a = (int32_t)(cy.w & 0x3FFFFFFFu);
            st.cr_t = (int64_t)(((uint64_t)cy.y << 32) | cy.x);
            walk<true>(s_case, s_act, s_ts, T0, e0, e1, st, A, vw.t_lo, vw.t_hi, mask, S.s_list[wv], cur,
                       w.rec_cell, w.rec_gap, wide);
        }
        __syncthreads();
    }
}

template <int TILE>
__global__ __launch_bounds__(kVB) void k_view_write(const int32_t* __restrict__ case_s,
                                        const int32_t* __restrict__ act_s,
                                        const int64_t* __restrict__ ts_s, int64_t n, int32_t A,
                                        const pm4g_view* __restrict__ views,
                                        const uint64_t* __restrict__ masks, ViewWs w) {
    __shared__ WalkSmem<TILE, kVW> S;
    ph_write<TILE, kVW>(hw_grid(), case_s, act_s, ts_s, n, A, views, masks, w, S);
}

// The gate after the count walk and the segment scans: every capacity the
// later kernels write into is known now; if one is short (or the records
// exceed 32-bit places) the call stops here, reported by k_view_finish.
__device__ __forceinline__ void ph_gate(Grid gd, ViewWs w) {
    if (threadIdx.x == 0 && gd.bid == 0) {
        int64_t g = 0;
        if (w.scal[7] > w.pair_cap || w.scal[9] > w.rec_cap) g = PM4G_E_CAPACITY;
        if (w.scal[7] <= w.pair_cap && w.scal[9] > (int64_t)0xFFFFFFFF) g = PM4G_E_INVALID;
        w.scal[12] = g;
    }
}

__global__ void k_view_gate(ViewWs w) { ph_gate(hw_grid(), w); }

__device__ __forceinline__ void ph_vb_flags(Grid gd, ViewWs w, int32_t V) {
    for (int64_t i = (int64_t)gd.bid * blockDim.x + threadIdx.x; i < w.n_vb;
         i += (int64_t)gd.nblk * blockDim.x)
        w.vb_flag[i] = w.vb_cnt[i] != 0 ? 1u : 0u;
    if (gd.bid == 0 && threadIdx.x == 0) w.scal[6] = V;
}

__global__ void k_view_vb_flags(ViewWs w, int32_t V) { ph_vb_flags(hw_grid(), w, V); }

// Segments: the non-empty (view, bucket) pairs in increasing order, each with
// its first record; the records' total closes the list.
__device__ __forceinline__ void ph_segs(Grid gd, ViewWs w) {
    for (int64_t i = (int64_t)gd.bid * blockDim.x + threadIdx.x; i < w.n_vb;
         i += (int64_t)gd.nblk * blockDim.x) {
        if (!w.vb_flag[i]) continue;
        const uint32_t g = w.vb_seg[i];
        w.seg_key[g] = (uint32_t)i;
        w.seg_rec[g] = w.vb_base[i];
    }
    if (gd.bid == 0 && threadIdx.x == 0) {
        const int64_t S = (int64_t)((uint32_t*)&w.scal[8])[0];
        w.seg_rec[S] = w.scal[9];
        w.scal[2] = S;
    }
}

__global__ void k_view_segs(ViewWs w) { ph_segs(hw_grid(), w); }

// LDS of an aggregation block: one 4096-cell table.
struct AggSmem {
    uint32_t scount[kCellsPerTable];
    uint64_t ssum[kCellsPerTable];
    alignas(16) int64_t smm[2 * kCellsPerTable];   // min, max of each cell side by side
    uint32_t tmp[kAB2 / kWave + 1];
    int64_t s_base;
};

// LDS of an activity-count block.
template <int BLOCK>
struct ActsSmem {
    uint32_t rows[PM4G_BATCHED_MAX_ACTIVITIES];
    uint32_t cols[PM4G_BATCHED_MAX_ACTIVITIES];
    int64_t s_src[kMaxBuckets];
    uint32_t s_m[kMaxBuckets];
    int64_t red[2][BLOCK / kWave];
};

// smm: each cell's min and max side by side, read with one 16-byte load (a
// stale pair only makes an atomic run that was not needed: min only falls
// and max only rises).
__device__ __forceinline__ void view_agg_rec(uint32_t* scount, uint64_t* ssum, int64_t* smm,
                                             uint32_t cell, uint64_t gap) {
    const int64_t gg = (int64_t)gap;
    atomicAdd(&scount[cell], 1u);
    atomicAdd(reinterpret_cast<unsigned long long*>(&ssum[cell]), (unsigned long long)gap);
    const longlong2 mm = *reinterpret_cast<const longlong2*>(&smm[2 * cell]);
    if (gg < mm.x) __hip_atomic_fetch_min(&smm[2 * cell], gg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (gg > mm.y) __hip_atomic_fetch_max(&smm[2 * cell + 1], gg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Records [r, r1) of a segment, this thread's share (stride kAB2), into the
// LDS table; WIDE: the cell sits in rec_cell, else in the top 12 bits.
template <bool WIDE>
__device__ __forceinline__ void agg_records(const ViewWs& w, int64_t r, int64_t r1, uint32_t* scount,
                                            uint64_t* ssum, int64_t* smm) {
    constexpr int kU = 4;   // records in flight per thread
    for (; r + (kU - 1) * kAB2 < r1; r += kU * kAB2) {
        uint64_t x[kU];
        uint32_t cell[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            x[u] = w.rec_gap[r + u * kAB2];
            if (WIDE) cell[u] = w.rec_cell[r + u * kAB2];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            view_agg_rec(scount, ssum, smm, WIDE ? cell[u] : (uint32_t)(x[u] >> 52),
                         WIDE ? x[u] : (x[u] & (kRecGapLimit - 1)));
    }
    for (; r < r1; r += kAB2) {
        const uint64_t x = w.rec_gap[r];
        view_agg_rec(scount, ssum, smm, WIDE ? (uint32_t)w.rec_cell[r] : (uint32_t)(x >> 52),
                     WIDE ? x : (x & (kRecGapLimit - 1)));
    }
}

// One block per (view, bucket) segment: its records are one contiguous range,
// streamed into a 4096-cell LDS table; after compaction only the touched
// cells are reset, so the table is cleared once per block.
__device__ __forceinline__ void ph_agg(Grid gd, int32_t A, ViewWs w, BatchedOutDev out, AggSmem& L) {
    uint32_t* scount = L.scount;
    uint64_t* ssum = L.ssum;
    int64_t* smm = L.smm;
    uint32_t* tmp = L.tmp;
    int64_t& s_base = L.s_base;
    if (w.scal[12] != 0) return;
    const int64_t S = w.scal[2];
    const int64_t AA = (int64_t)A * A;
    const int NB = w.n_buckets;
    const bool wide = w.scal[10] != 0;
    for (int c = threadIdx.x; c < kCellsPerTable; c += kAB2) {
        scount[c] = 0;
        ssum[c] = 0;
        smm[2 * c] = INT64_MAX;
        smm[2 * c + 1] = INT64_MIN;
    }
    __syncthreads();
    for (int64_t g = gd.bid; g < S; g += gd.nblk) {
        const uint32_t key = w.seg_key[g];
        const uint32_t v = key / (uint32_t)NB;
        const uint32_t bk = key % (uint32_t)NB;
        const int64_t r1 = w.seg_rec[g + 1];
        if (wide) agg_records<true>(w, w.seg_rec[g] + threadIdx.x, r1, scount, ssum, smm);
        else agg_records<false>(w, w.seg_rec[g] + threadIdx.x, r1, scount, ssum, smm);
        __syncthreads();
        // compaction in cell order; start cells go straight to the start counts
        constexpr int kPer = kCellsPerTable / kAB2;   // 4 cells per thread, blocked
        uint32_t flags = 0, touched = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int c = threadIdx.x * kPer + q;
            const int64_t cell = (int64_t)bk * kCellsPerTable + c;
            if (scount[c] == 0) continue;
            touched |= 1u << q;
            if (cell < AA) flags |= 1u << q;
            else if (cell < AA + A) out.start_count[(size_t)v * A + (cell - AA)] = scount[c];
        }
        uint32_t total;
        uint32_t rr = block_excl_sum<kAB2>((uint32_t)__popc(flags), tmp, &total);
        if (threadIdx.x == 0) {
            s_base = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(&w.scal[3]),
                                        (unsigned long long)total);
            w.seg_cells[g] = total;
            w.seg_tmp[g] = s_base;
            atomicAdd(&w.view_cells[v], total);
        }
        __syncthreads();
        const int64_t base = s_base;
        if (base + (int64_t)total > w.cell_cap) flags = 0;   // over capacity: counted, not written
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            if (!(touched & (1u << q))) continue;
            const int c = threadIdx.x * kPer + q;
            if (flags & (1u << q)) {
                const int64_t at = base + rr;
                w.t_cell[at] = (uint32_t)((int64_t)bk * kCellsPerTable + c);
                w.t_count[at] = scount[c];
                w.t_sum[at] = ssum[c];
                w.t_min[at] = smm[2 * c];
                w.t_max[at] = smm[2 * c + 1];
                ++rr;
            }
            scount[c] = 0;   // reset for the next segment
            ssum[c] = 0;
            smm[2 * c] = INT64_MAX;
            smm[2 * c + 1] = INT64_MIN;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kAB2) void k_view_agg(int32_t A, ViewWs w, BatchedOutDev out) {
    __shared__ AggSmem S;
    ph_agg(hw_grid(), A, w, out, S);
}

__device__ __forceinline__ void ph_copy(Grid gd, int32_t A, ViewWs w, BatchedOutDev out) {
    const int64_t S = w.scal[2];
    const bool fits = w.scal[12] == 0 && w.scal[4] <= out.cap_edges && w.scal[3] <= w.cell_cap;
    if (!fits) return;
    const int wv = (gd.bid * blockDim.x + threadIdx.x) / kWave;
    const int nw = gd.nblk * blockDim.x / kWave;
    for (int64_t g = wv; g < S; g += nw) {
        const int64_t src = w.seg_tmp[g], dst = w.seg_out[g];
        const uint32_t m = w.seg_cells[g];
        constexpr int kU = 4;   // all loads of kU steps issued before the stores
        for (uint32_t r0 = 0; r0 < m; r0 += kU * kWave) {
            uint32_t cell[kU], cnt[kU];
            uint64_t sum[kU];
            int64_t mn[kU], mx[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t r = r0 + u * kWave + lane();
                if (r < m) {
                    cell[u] = w.t_cell[src + r];
                    cnt[u] = w.t_count[src + r];
                    sum[u] = w.t_sum[src + r];
                    mn[u] = w.t_min[src + r];
                    mx[u] = w.t_max[src + r];
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t r = r0 + u * kWave + lane();
                if (r < m) {
                    out.src[dst + r] = (int32_t)(cell[u] / (uint32_t)A);
                    out.dst[dst + r] = (int32_t)(cell[u] % (uint32_t)A);
                    out.count[dst + r] = cnt[u];
                    out.dt_sum[dst + r] = (int64_t)sum[u];
                    out.dt_min[dst + r] = mn[u];
                    out.dt_max[dst + r] = mx[u];
                    if (out.dt_mean) out.dt_mean[dst + r] = (double)(int64_t)sum[u] / (double)(int64_t)cnt[u];
                }
            }
        }
    }
}



// Per view: its segments form a run of the sorted segment list; fold their
// cells into row and column sums; derive activity and end counts.
template <int BLOCK>
__device__ __forceinline__ void ph_acts(Grid gd, int32_t V, int32_t A, ViewWs w, BatchedOutDev out,
                                        ActsSmem<BLOCK>& L) {
    uint32_t* rows = L.rows;   // at most the view's kept events (< 2^31)
    uint32_t* cols = L.cols;
    int64_t* s_src = L.s_src;
    uint32_t* s_m = L.s_m;
    const int64_t S = w.scal[2];
    const uint32_t NB = (uint32_t)w.n_buckets;
    if (w.scal[12] != 0 || w.scal[3] > w.cell_cap) return;   // temporary cells were not all written
    for (int64_t v = gd.bid; v < V; v += gd.nblk) {
        for (int a = threadIdx.x; a < A; a += BLOCK) rows[a] = cols[a] = 0;
        __syncthreads();
        // first segment of this view: lower bound of key v*NB over segment keys
        int64_t lo = 0, hi = S;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (w.seg_key[mid] < (uint32_t)v * NB) lo = mid + 1;
            else hi = mid;
        }
        // the view's segments (at most NB): their places and cell counts to LDS
        int ns = 0;
        for (int k0 = 0; k0 < (int)NB; k0 += BLOCK) {
            const int k = k0 + threadIdx.x;
            const bool mine = k < (int)NB && lo + k < S && w.seg_key[lo + k] / NB == (uint32_t)v;
            if (mine) {
                s_src[k] = w.seg_tmp[lo + k];
                s_m[k] = w.seg_cells[lo + k];
            }
            ns += __syncthreads_count(mine);
        }
        __syncthreads();
        for (int g = 0; g < ns; ++g) {
            const int64_t src = s_src[g];
            const uint32_t m = s_m[g];
            constexpr int kU = 2;
            for (uint32_t r0 = 0; r0 < m; r0 += kU * BLOCK) {
                uint32_t cell[kU], c[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const uint32_t r = r0 + u * BLOCK + threadIdx.x;
                    cell[u] = 0;
                    c[u] = 0;
                    if (r < m) {
                        cell[u] = w.t_cell[src + r];
                        c[u] = w.t_count[src + r];
                    }
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    if (c[u]) {
                        atomicAdd(&rows[cell[u] / (uint32_t)A], c[u]);
                        atomicAdd(&cols[cell[u] % (uint32_t)A], c[u]);
                    }
                }
            }
        }
        __syncthreads();
        int64_t ne = 0, nc = 0;
        for (int a = threadIdx.x; a < A; a += BLOCK) {
            const size_t at = (size_t)v * A + a;
            const int64_t st = out.start_count[at];
            const int64_t act = st + (int64_t)cols[a];
            out.act_count[at] = act;
            out.end_count[at] = act - (int64_t)rows[a];
            ne += act;
            nc += st;
        }
        ne = wave_sum(ne);
        nc = wave_sum(nc);
        if (lane() == 0) {
            L.red[0][threadIdx.x / kWave] = ne;
            L.red[1][threadIdx.x / kWave] = nc;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t a = 0, b = 0;
            for (int k = 0; k < BLOCK / kWave; ++k) {
                a += L.red[0][k];
                b += L.red[1][k];
            }
            out.n_events[v] = a;
            out.n_cases[v] = b;
        }
        __syncthreads();
    }
}

// The copy and the activity counts read the same temporary cells and write
// disjoint outputs: one launch, its first kOutCopyBlocks blocks copying and the
// others counting, so that the two latency-bound phases overlap.
constexpr int64_t kOutCopyBlocks = 2048;

__global__ __launch_bounds__(256) void k_view_out(int32_t V, int32_t A, ViewWs w, BatchedOutDev out) {
    __shared__ ActsSmem<256> S;
    if ((int64_t)blockIdx.x < kOutCopyBlocks)
        ph_copy(Grid{(int64_t)blockIdx.x, kOutCopyBlocks}, A, w, out);
    else
        ph_acts<256>(Grid{(int64_t)blockIdx.x - kOutCopyBlocks, (int64_t)gridDim.x - kOutCopyBlocks}, V, A, w,
                     out, S);
}

__device__ __forceinline__ void ph_finish(Grid gd, int32_t V, ViewWs w, BatchedOutDev out) {
    if (threadIdx.x == 0 && gd.bid == 0) {
        const int64_t gate = w.scal[12];
        const bool pairs_short = w.scal[7] > w.pair_cap;   // then the count walk did not run
        out.edge_off[V] = gate ? 0 : w.scal[4];
        out.required[0] = gate ? 0 : w.scal[4];             // unknown until the records are placed
        out.required[1] = pairs_short ? 0 : w.scal[9];
        out.required[2] = w.scal[7] * (int64_t)w.n_buckets;   // run places: pairs x buckets
        out.required[3] = w.scal[7];
        out.required[4] = gate ? 0 : w.scal[3];
        if (gate) set_status(out.status, (int32_t)gate);
        else if (w.scal[4] > out.cap_edges || w.scal[3] > w.cell_cap) set_status(out.status, PM4G_E_CAPACITY);
    }
}

__global__ void k_view_finish(int32_t V, ViewWs w, BatchedOutDev out) { ph_finish(hw_grid(), V, w, out); }


// ---- the single persistent launch ----

// Exclusive scans over the persistent grid: per-block sums of contiguous
// chunks, one block scans the sums (nblk <= 1024 = the block size), each block
// applies its prefix.
template <typename T>
__device__ __forceinline__ void gscan_reduce(Grid gd, const uint32_t* in, int64_t n, T* partial) {
    __shared__ T red[kFT / kWave];
    const int64_t chunk = (n + gd.nblk - 1) / gd.nblk;
    const int64_t b0 = gd.bid * chunk;
    const int64_t b1 = (b0 + chunk) < n ? (b0 + chunk) : n;
    T sum = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kFT) sum += in[i];
    sum = wave_sum(sum);
    if (lane() == 0) red[threadIdx.x / kWave] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int k = 0; k < kFT / kWave; ++k) t += red[k];
        partial[gd.bid] = t;
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void gscan_top(Grid gd, T* partial, T* total) {
    __shared__ T tmp[kFT / kWave + 1];
    if (gd.bid != 0) return;
    const T v = (int64_t)threadIdx.x < gd.nblk ? partial[threadIdx.x] : (T)0;
    T tot;
    const T ex = block_excl_sum<kFT>(v, tmp, &tot);
    if ((int64_t)threadIdx.x < gd.nblk) partial[threadIdx.x] = ex;
    if (threadIdx.x == 0 && total) *total = tot;
}

template <typename T>
__device__ __forceinline__ void gscan_apply(Grid gd, const uint32_t* in, int64_t n, const T* partial, T* out) {
    __shared__ T tmp[kFT / kWave + 1];
    const int64_t chunk = (n + gd.nblk - 1) / gd.nblk;
    const int64_t b0 = gd.bid * chunk;
    const int64_t b1 = (b0 + chunk) < n ? (b0 + chunk) : n;
    T run = partial[gd.bid];
    for (int64_t c0 = b0; c0 < b1; c0 += kFT) {   // block-uniform
        const int64_t i = c0 + threadIdx.x;
        const T v = i < b1 ? (T)in[i] : (T)0;
        T tot;
        const T ex = block_excl_sum<kFT>(v, tmp, &tot);
        if (i < b1) out[i] = run + ex;
        run += tot;
    }
}

// Grid barrier of the persistent launch (every block resident: a cooperative
// launch).  Block b announces its arrival at barrier k by writing the tag
// (call epoch << 6 | k) into bar[b]; block 0 waits until every block has
// announced it and publishes the tag in bar[kViewMaxBlocks]; the others wait
// for that.  Tags are unique per call, so words left in the workspace by
// earlier calls never match.  The release fence before the arrival and the
// acquire fence after the wait make each phase's writes visible to the next
// phase on every XCD.  A wait is bounded: past kBarrierPolls polls (seconds,
// far beyond any phase) the call's status becomes PM4G_E_DEVICE and the
// block goes on, so a broken schedule ends the call instead of hanging it.
constexpr int64_t kBarrierPolls = int64_t(1) << 22;

__device__ void grid_barrier(Grid gd, uint64_t* bar, uint64_t tag, int32_t* status) {
    __syncthreads();
    if (threadIdx.x < kWave) {
        __threadfence();
        if (lane() == 0) __hip_atomic_store(&bar[gd.bid], tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool late = false;
        if (gd.bid == 0) {
            for (int64_t b0 = 0; b0 < gd.nblk; b0 += kWave) {
                const int64_t b = b0 + lane();
                int64_t polls = 0;
                for (;;) {
                    const bool here = b >= gd.nblk ||
                                      __hip_atomic_load(&bar[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == tag;
                    if (__ballot(!here) == 0) break;
                    if (++polls > kBarrierPolls) {
                        late = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __threadfence();
            if (lane() == 0) __hip_atomic_store(&bar[kViewMaxBlocks], tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (lane() == 0) {
            int64_t polls = 0;
            while (__hip_atomic_load(&bar[kViewMaxBlocks], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != tag) {
                if (++polls > kBarrierPolls) {
                    late = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (late && lane() == 0) set_status(status, PM4G_E_DEVICE);
        __threadfence();
    }
    __syncthreads();
}

struct FusedArgs {
    const int32_t* case_s;
    const int32_t* act_s;
    const int64_t* ts_s;
    const int64_t* case_off;
    const int32_t* case_code;
    const int64_t* n_cases;
    const int32_t* status_in;
    const pm4g_view* views;
    const uint64_t* masks;
    int64_t n;
    int32_t A, V;
    uint64_t epoch;
    ViewWs w;
    BatchedOutDev out;
};

template <int TILE>
union FusedSmem {
    WalkSmem<TILE, kFT / kWave> walk;
    AggSmem agg;
    ActsSmem<kFT> acts;
};

// The whole batched call in one launch: the phases of the per-phase kernels,
// in the same order, separated by grid barriers.
// The kernel's arguments are read through a pointer that each phase takes
// anew from an empty register move the compiler cannot see through, so a
// phase loads the fields it uses instead of the whole set staying live (in
// scalar registers, then spilled) across the launch.
typedef const FusedArgs __attribute__((address_space(4))) KernArgs;   // the kernel-argument segment
__device__ __forceinline__ FusedArgs fresh(KernArgs* p) {
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(p));
    return *p;
#else
    (void)p;   // the host pass compiles device code it never runs
    return FusedArgs{};
#endif
}

template <int TILE>
__global__ __launch_bounds__(kFT) void k_view_fused(FusedArgs args) {
    __shared__ FusedSmem<TILE> sm;
    const Grid gd = hw_grid();
    KernArgs* ap = (KernArgs*)__builtin_amdgcn_kernarg_segment_ptr();
    uint64_t k = args.epoch << 6;
    int32_t* st = args.out.status;
    uint64_t* bar = args.w.bar;
#define PA (fresh(ap))
    ph_init(gd, PA.w, PA.V, PA.A, PA.status_in, PA.out);
    grid_barrier(gd, bar, ++k, st);
    ph_span(gd, PA.case_off, PA.ts_s, PA.n_cases, PA.w);
    ph_slice(gd, PA.views, PA.V, PA.case_off, PA.case_code, PA.n_cases, PA.w);
    grid_barrier(gd, bar, ++k, st);
    ph_tile_scan(gd, PA.w);
    grid_barrier(gd, bar, ++k, st);
    ph_fill(gd, PA.V, PA.w);
    grid_barrier(gd, bar, ++k, st);
    {
        const FusedArgs a = PA;
        ph_count<TILE, kFT / kWave>(gd, a.case_s, a.act_s, a.ts_s, a.n, a.A, a.views, a.masks, a.w, sm.walk);
    }
    grid_barrier(gd, bar, ++k, st);
    ph_vb_flags(gd, PA.w, PA.V);
    grid_barrier(gd, bar, ++k, st);
    {
        const ViewWs w = PA.w;
        const int64_t nvb = w.scal[11];
        gscan_reduce<int64_t>(gd, w.vb_cnt, nvb, w.part64);
        gscan_reduce<uint32_t>(gd, w.vb_flag, nvb, w.part32);
    }
    grid_barrier(gd, bar, ++k, st);
    {
        const ViewWs w = PA.w;
        gscan_top<int64_t>(gd, w.part64, &w.scal[9]);
        gscan_top<uint32_t>(gd, w.part32, reinterpret_cast<uint32_t*>(&w.scal[8]));
    }
    grid_barrier(gd, bar, ++k, st);
    {
        const ViewWs w = PA.w;
        const int64_t nvb = w.scal[11];
        gscan_apply<int64_t>(gd, w.vb_cnt, nvb, w.part64, w.vb_base);
        gscan_apply<uint32_t>(gd, w.vb_flag, nvb, w.part32, w.vb_seg);
    }
    grid_barrier(gd, bar, ++k, st);
    ph_gate(gd, PA.w);
    ph_segs(gd, PA.w);
    grid_barrier(gd, bar, ++k, st);
    {
        const FusedArgs a = PA;
        ph_write<TILE, kFT / kWave>(gd, a.case_s, a.act_s, a.ts_s, a.n, a.A, a.views, a.masks, a.w, sm.walk);
    }
    grid_barrier(gd, bar, ++k, st);
    ph_agg(gd, PA.A, PA.w, PA.out, sm.agg);
    grid_barrier(gd, bar, ++k, st);
    {
        const FusedArgs a = PA;
        const int64_t S = a.w.scal[2];
        gscan_reduce<int64_t>(gd, a.w.seg_cells, S, a.w.part64);
        gscan_reduce<int64_t>(gd, a.w.view_cells, a.V, a.w.part64b);
    }
    grid_barrier(gd, bar, ++k, st);
    {
        const FusedArgs a = PA;
        gscan_top<int64_t>(gd, a.w.part64, &a.w.scal[4]);
        gscan_top<int64_t>(gd, a.w.part64b, nullptr);
    }
    grid_barrier(gd, bar, ++k, st);
    {
        const FusedArgs a = PA;
        const int64_t S = a.w.scal[2];
        gscan_apply<int64_t>(gd, a.w.seg_cells, S, a.w.part64, a.w.seg_out);
        gscan_apply<int64_t>(gd, a.w.view_cells, a.V, a.w.part64b, a.out.edge_off);
    }
    grid_barrier(gd, bar, ++k, st);
    {   // the copy on half of the blocks, the activity counts on the other half
        const int64_t half = gd.nblk / 2 > 0 ? gd.nblk / 2 : 1;
        if (gd.bid < half || gd.nblk < 2) ph_copy(Grid{gd.bid, half}, PA.A, PA.w, PA.out);
        if (gd.bid >= half || gd.nblk < 2)
            ph_acts<kFT>(gd.nblk < 2 ? gd : Grid{gd.bid - half, gd.nblk - half}, PA.V, PA.A, PA.w, PA.out, sm.acts);
    }
    grid_barrier(gd, bar, ++k, st);
    ph_finish(gd, PA.V, PA.w, PA.out);
#undef PA
}

}  // namespace

// Grid of the persistent launch on the current device: every block resident
// (blocks per CU from the occupancy query, times the CUs), at most
// kViewMaxBlocks.
static int fused_grid(int tile) {
    static int cache[64][2] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int& g = cache[dev][tile == 2048 ? 0 : 1];
    if (g == 0) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        const void* fn = tile == 2048 ? (const void*)k_view_fused<2048> : (const void*)k_view_fused<4096>;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kFT, 0) != hipSuccess) return 0;
        const int64_t t = (int64_t)cus * per;
        g = (int)(t < kViewMaxBlocks ? t : kViewMaxBlocks);
    }
    return g;
}

hipError_t launch_views_fused(const pm4g_prepared* p, const pm4g_view* views, const uint64_t* masks, int32_t V,
                              ViewWs w, BatchedOutDev out, hipStream_t s) {
    ProfScope ps(P_VIEW_FUSED, s);
    // call epochs: distinct per call (and, from a random start, from any word
    // an earlier owner of the workspace left behind)
    static std::atomic<uint64_t> epoch{std::random_device{}() * 0x9E3779B97F4A7C15ull};
    const int grid = fused_grid(w.tile);
    if (grid <= 0) return hipErrorInvalidConfiguration;
    FusedArgs a{p->case_s, p->act_s, p->ts_s, p->case_off, p->case_code, p->n_cases, p->status, views, masks,
                p->n_events, p->n_activities, V, epoch.fetch_add(1) & ((uint64_t(1) << 57) - 1), w, out};
    void* args[] = {&a};
    const void* fn = w.tile == 2048 ? (const void*)k_view_fused<2048> : (const void*)k_view_fused<4096>;
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(kFT), args, 0, s);
}

hipError_t launch_views_plan(const pm4g_prepared* p, const pm4g_view* views, int32_t V, ViewWs w,
                             BatchedOutDev out, hipStream_t s) {
    ProfScope ps(P_VIEW_PLAN, s);
    const int32_t A = p->n_activities;
    k_view_init<<<1024, 256, 0, s>>>(w, V, A, p->status, out);
    k_view_span<<<1024, 256, 0, s>>>(p->case_off, p->ts_s, p->n_cases, w);
    if (V > 0) k_view_slice<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(views, V, p->case_off, p->case_code,
                                                                          p->n_cases, w);
    k_view_tile_scan<<<1, 1024, 0, s>>>(w);
    if (V > 0) k_view_fill<<<(unsigned)((V + 3) / 4), 256, 0, s>>>(V, w);
    return hipGetLastError();
}

hipError_t launch_views_count(const pm4g_prepared* p, const pm4g_view* views, const uint64_t* masks,
                              ViewWs w, int grid, hipStream_t s) {
    ProfScope ps(P_VIEW_EMIT, s);
    const int64_t n = p->n_events;
    if (w.n_tiles > 0) {
        const unsigned g = (unsigned)(w.n_tiles < grid ? w.n_tiles : grid);
        if (w.tile == 2048)
            k_view_count<2048><<<g, kVB, 0, s>>>(p->case_s, p->act_s, p->ts_s, n, p->n_activities, views, masks, w);
        else
            k_view_count<4096><<<g, kVB, 0, s>>>(p->case_s, p->act_s, p->ts_s, n, p->n_activities, views, masks, w);
    }
    return hipGetLastError();
}

hipError_t launch_views_write(const pm4g_prepared* p, const pm4g_view* views, const uint64_t* masks,
                              ViewWs w, int grid, hipStream_t s) {
    ProfScope ps(P_VIEW_WRITE, s);
    const int64_t n = p->n_events;
    if (w.n_tiles > 0) {
        const unsigned g = (unsigned)(w.n_tiles < grid ? w.n_tiles : grid);
        if (w.tile == 2048)
            k_view_write<2048><<<g, kVB, 0, s>>>(p->case_s, p->act_s, p->ts_s, n, p->n_activities, views, masks, w);
        else
            k_view_write<4096><<<g, kVB, 0, s>>>(p->case_s, p->act_s, p->ts_s, n, p->n_activities, views, masks, w);
    }
    return hipGetLastError();
}

// Places the (view, bucket) segments, writes the records (write walk),
// aggregates per segment.
hipError_t launch_views_reduce(const pm4g_prepared* p, const pm4g_view* views, const uint64_t* masks, int32_t V,
                               ViewWs w, BatchedOutDev out, int emit_grid, int agg_grid, hipStream_t s) {
    const int32_t A = p->n_activities;
    {
        ProfScope ps(P_VIEW_PLACE, s);
        k_view_vb_flags<<<1024, 256, 0, s>>>(w, V);
        dev::excl_scan<int64_t>(w.vb_cnt, &w.scal[11], w.vb_base, w.part64, &w.scal[9], s);
        dev::excl_scan<uint32_t>(w.vb_flag, &w.scal[11], w.vb_seg, w.part32, (uint32_t*)&w.scal[8], s);
        k_view_gate<<<1, 64, 0, s>>>(w);
        k_view_segs<<<1024, 256, 0, s>>>(w);
    }
    {
        const hipError_t e = launch_views_write(p, views, masks, w, emit_grid, s);
        if (e != hipSuccess) return e;
    }
    {
        ProfScope ps(P_VIEW_AGG, s);
        k_view_agg<<<(unsigned)agg_grid, kAB2, 0, s>>>(A, w, out);
    }
    {
        ProfScope ps(P_VIEW_OUT, s);
        dev::excl_scan<int64_t>(w.seg_cells, &w.scal[2], w.seg_out, w.part64, &w.scal[4], s);
        dev::excl_scan<int64_t>(w.view_cells, &w.scal[6], out.edge_off, w.part64, (int64_t*)nullptr, s);
        k_view_out<<<(unsigned)(kOutCopyBlocks + 2048), 256, 0, s>>>(V, A, w, out);
        k_view_finish<<<1, 1, 0, s>>>(V, w, out);
    }
    return hipGetLastError();
}

}  // namespace pm4g
