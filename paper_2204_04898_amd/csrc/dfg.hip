// Directly-follows graph aggregation over a prepared log (Sec. 3, the
// aggregations over consecutive event pairs: frequency and performance DFG;
// start and end activities; how often each activity occurs).  For position i
// of the ordered log, the event
// directly follows i-1 iff both have the same case; the pair contributes to
// cell act_s[i-1]*A + act_s[i] with gap ts_s[i] - ts_s[i-1] (mod 2^64).
//
// Two aggregation paths, both free of per-event global atomics (global
// atomics run at ~25 G/s on MI355X, LDS atomics at ~700 G/s):
//   A*A <= 4096  k_dfg_lds: 256 persistent blocks, one privatised LDS table
//                each (count u32, sum u64, min, max: 112 KB), partial tables
//                written out and reduced per cell.
//   A*A >  4096  cells are cut into buckets of 4096 (cell >> 12) and the
//                edges are partitioned bucket-major, so that each bucket's
//                edges are one contiguous stream:
//                k_dfg_count    per (bucket, chunk of the log) edge counts,
//                               and the start / end counts (an activity's
//                               count is folded from those and the pair
//                               counts by k_dfg_acts);
//                scan           first edge index of every (bucket, chunk);
//                k_dfg_scatter  edges (u16 cell within the bucket, u64 gap)
//                               written to their place via LDS cursors;
//                k_dfg_plan     buckets cut into slots of about E/512 edges
//                               (Zipf-heavy buckets get more slots);
//                k_dfg_agg      one block per slot streams its edges into a
//                               4096-cell LDS table, writes a partial table.
// k_dfg_reduce folds the partial tables, writes the dense outputs and the
// FP64 mean; k_dfg_acts / k_dfg_final fold the activity counts, n_cases and the
// overflow flag.
// Bytes per event: 16 read (+ 8 read, 10 write and 10 read per edge on the
// bucketed path).
#include <math.h>

#include "common.hpp"
#include "devsort.hpp"
#include "internal.hpp"
#include "prof.hpp"
#include "../../include/pm4g.h"

namespace pm4g {

constexpr int kLB = 1024;   // threads of k_dfg_lds
constexpr int kAB = 1024;   // threads of k_dfg_agg

static int64_t n_buckets(int32_t A) {
    return ((int64_t)A * A + kCellsPerTable - 1) / kCellsPerTable;
}
// chunk of the log per (bucket, chunk) counter: about 64 buckets per 4096 events
static int64_t dfg_chunk(int64_t nbk) { return (int64_t)kDfgTile * (nbk <= 64 ? 1 : (nbk + 63) / 64); }
static int64_t dfg_chunks(int64_t n, int64_t nbk) {
    const int64_t c = dfg_chunk(nbk);
    return (n + c - 1) / c;
}

DfgWs dfg_ws_layout(Bump& b, int64_t n, int32_t A) {
    DfgWs w{};
    if (A <= kDfgLdsMaxA) {
        const int64_t slots = kDfgLdsBlocks;
        w.n_slots_max = (int32_t)slots;
        w.n_act_blocks = kDfgLdsBlocks;
        w.pcount = b.take<uint32_t>(slots * kCellsPerTable);
        w.psum = b.take<uint64_t>(slots * kCellsPerTable);
        w.pmin = b.take<int64_t>(slots * kCellsPerTable);
        w.pmax = b.take<int64_t>(slots * kCellsPerTable);
    } else {
        const int64_t nbk = n_buckets(A);
        const int64_t nch = dfg_chunks(n, nbk);
        const int64_t slots = nbk + kDfgAggTarget;
        w.n_slots_max = (int32_t)slots;
        const int64_t g = nch < kDfgPartBlocks ? (nch < 1 ? 1 : nch) : kDfgPartBlocks;
        w.n_act_blocks = (int32_t)g;
        const size_t m = (size_t)(n > 0 ? n : 1);
        w.pcount = b.take<uint32_t>(slots * kCellsPerTable);
        w.psum = b.take<uint64_t>(slots * kCellsPerTable);
        w.pmin = b.take<int64_t>(slots * kCellsPerTable);
        w.pmax = b.take<int64_t>(slots * kCellsPerTable);
        w.ecell = b.take<uint16_t>(m);
        w.egap = b.take<uint64_t>(m);
        w.ecnt = b.take<uint32_t>((size_t)(nbk * nch) + 1);
        w.escan = b.take<uint32_t>((size_t)(nbk * nch) + 1);
        w.bbase = b.take<uint32_t>(nbk);
        w.btotal = b.take<uint32_t>(nbk);
        w.bfirst = b.take<uint32_t>(nbk);
        w.bslots = b.take<uint32_t>(nbk);
        w.plan = b.take<int4>(slots);
        w.nplan = b.take<uint32_t>(1);
        w.part32 = b.take<uint32_t>(dev::kScanGrid);
        w.scal = b.take<int64_t>(2);
        w.utotal = b.take<uint32_t>(1);
    }
    w.pfreq = b.take<uint32_t>((size_t)w.n_act_blocks * A);
    w.pstart = b.take<uint32_t>((size_t)w.n_act_blocks * A);
    w.pend = b.take<uint32_t>((size_t)w.n_act_blocks * A);
    w.pspan = b.take<uint64_t>(w.n_act_blocks);
    return w;
}

// ---------------------------------------------------------------------------
// A*A <= 4096: privatised LDS tables

__global__ __launch_bounds__(kLB) void k_dfg_lds(const int32_t* __restrict__ case_s,
                                                 const int32_t* __restrict__ act_s,
                                                 const int64_t* __restrict__ ts_s, int64_t n,
                                                 int32_t A, DfgWs ws, int32_t* status) {
    __shared__ uint32_t scount[kCellsPerTable];
    __shared__ uint64_t ssum[kCellsPerTable];
    __shared__ int64_t smin[kCellsPerTable];
    __shared__ int64_t smax[kCellsPerTable];
    __shared__ uint32_t sfreq[kDfgLdsMaxA], sstart[kDfgLdsMaxA], send[kDfgLdsMaxA];
    __shared__ uint64_t sspan[kLB / kWave];

    const int cells = A * A;
    for (int c = threadIdx.x; c < cells; c += kLB) {
        scount[c] = 0;
        ssum[c] = 0;
        smin[c] = INT64_MAX;
        smax[c] = INT64_MIN;
    }
    if (threadIdx.x < A) sfreq[threadIdx.x] = sstart[threadIdx.x] = send[threadIdx.x] = 0;
    __syncthreads();

    uint64_t span = 0;
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * kLB;
    for (int64_t i = (int64_t)blockIdx.x * kLB + threadIdx.x; i < n; i += stride) {
        const int32_t c = case_s[i];
        const int32_t a = act_s[i];
        if ((uint32_t)a >= (uint32_t)A) {
            bad = true;
            continue;
        }
        const bool first = (i == 0) || case_s[i - 1] != c;
        const bool last = (i == n - 1) || case_s[i + 1] != c;
        atomicAdd(&sfreq[a], 1u);
        if (first) atomicAdd(&sstart[a], 1u);
        if (last) atomicAdd(&send[a], 1u);
        if (!first) {
            const int32_t p = act_s[i - 1];
            if ((uint32_t)p >= (uint32_t)A) continue;
            const int cell = p * A + a;
            const uint64_t gap = (uint64_t)ts_s[i] - (uint64_t)ts_s[i - 1];
            const int64_t g = (int64_t)gap;
            atomicAdd(&scount[cell], 1u);
            atomicAdd(reinterpret_cast<unsigned long long*>(&ssum[cell]), (unsigned long long)gap);
            if (g < __hip_atomic_load(&smin[cell], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                __hip_atomic_fetch_min(&smin[cell], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (g > __hip_atomic_load(&smax[cell], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                __hip_atomic_fetch_max(&smax[cell], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            span = sat_add63(span, cap63(gap));
        }
    }
    if (__ballot(bad) != 0 && lane() == 0) set_status(status, PM4G_E_RANGE);
    // saturating block sum of the span
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) span = sat_add63(span, __shfl_xor(span, o));
    if (lane() == 0) sspan[threadIdx.x / kWave] = span;
    __syncthreads();

    const size_t slot = (size_t)blockIdx.x * kCellsPerTable;
    for (int c = threadIdx.x; c < cells; c += kLB) {
        ws.pcount[slot + c] = scount[c];
        ws.psum[slot + c] = ssum[c];
        ws.pmin[slot + c] = smin[c];
        ws.pmax[slot + c] = smax[c];
    }
    const size_t ab = (size_t)blockIdx.x * A;
    if (threadIdx.x < A) {
        ws.pfreq[ab + threadIdx.x] = sfreq[threadIdx.x];
        ws.pstart[ab + threadIdx.x] = sstart[threadIdx.x];
        ws.pend[ab + threadIdx.x] = send[threadIdx.x];
    }
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int k = 0; k < kLB / kWave; ++k) s = sat_add63(s, sspan[k]);
        ws.pspan[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// A*A > 4096: bucket-major edges

constexpr int kCB = 512;                  // threads of k_dfg_count / k_dfg_scatter


// Four consecutive events [e0, e0 + 4) of the prepared log in registers,
// with the event before e0 (and the case after e0 + 3): 16-byte loads when
// the quad lies inside [.., lim) and the columns are 16-byte aligned, element
// loads otherwise; neighbours come from the adjacent lanes (the lanes hold
// consecutive quads), the wave's edge lanes load them.  Every lane of the
// wave must execute it.  Lanes past `lim` get case ~prev so nothing pairs.
struct Quad {
    int32_t c[4], a[4];
    int64_t t[4];
    int32_t cp, ap;   // event e0 - 1 (cp = ~c[0] when e0 == 0)
    int64_t tp;
    int32_t cn;       // case of event e0 + 4 (~c[3] past the log)
};

template <bool WANT_TS, bool WANT_NEXT>
__device__ __forceinline__ Quad load_quad(const int32_t* __restrict__ case_s, const int32_t* __restrict__ act_s,
                                          const int64_t* __restrict__ ts_s, int64_t e0, int64_t lim, int64_t n,
                                          bool aligned) {
    Quad q;
    if (aligned && e0 + 3 < lim) {
        const int4 c4 = *reinterpret_cast<const int4*>(case_s + e0);
        const int4 a4 = *reinterpret_cast<const int4*>(act_s + e0);
        q.c[0] = c4.x; q.c[1] = c4.y; q.c[2] = c4.z; q.c[3] = c4.w;
        q.a[0] = a4.x; q.a[1] = a4.y; q.a[2] = a4.z; q.a[3] = a4.w;
        if (WANT_TS) {
            const longlong2 t01 = *reinterpret_cast<const longlong2*>(ts_s + e0);
            const longlong2 t23 = *reinterpret_cast<const longlong2*>(ts_s + e0 + 2);
            q.t[0] = t01.x; q.t[1] = t01.y; q.t[2] = t23.x; q.t[3] = t23.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = e0 + j;
            const bool in = i < lim;
            q.c[j] = in ? case_s[i] : (j ? ~q.c[j - 1] : 0);
            q.a[j] = in ? act_s[i] : 0;
            if (WANT_TS) q.t[j] = in ? ts_s[i] : 0;
        }
    }
    q.cp = __shfl_up(q.c[3], 1);
    q.ap = __shfl_up(q.a[3], 1);
    if (WANT_TS) q.tp = __shfl_up(q.t[3], 1);
    if (lane() == 0) {
        if (e0 > 0 && e0 - 1 < n) {
            q.cp = case_s[e0 - 1];
            q.ap = act_s[e0 - 1];
            if (WANT_TS) q.tp = ts_s[e0 - 1];
        } else {
            q.cp = ~q.c[0];
        }
    }
    if (WANT_NEXT) {
        q.cn = __shfl_down(q.c[0], 1);
        if (lane() == kWave - 1) q.cn = e0 + 4 < n ? case_s[e0 + 4] : ~q.c[3];
    }
    return q;
}

// Per chunk: edge counts per bucket; per block: start and end counts.
// Dynamic LDS: (2 * A + nbk) u32.
__global__ __launch_bounds__(kCB) void k_dfg_count(const int32_t* __restrict__ case_s,
                                                   const int32_t* __restrict__ act_s, int64_t n,
                                                   int32_t A, int64_t nbk, int64_t nch, int64_t chunk,
                                                   DfgWs ws, int32_t* status) {
    extern __shared__ uint32_t dsm[];
    uint32_t* sstart = dsm;
    uint32_t* send = dsm + A;
    uint32_t* bcnt = dsm + 2 * A;
    for (int a = threadIdx.x; a < 2 * A; a += kCB) dsm[a] = 0;
    const bool aligned = ((reinterpret_cast<uintptr_t>(case_s) | reinterpret_cast<uintptr_t>(act_s)) & 15) == 0;
    bool bad = false;
    for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        for (int64_t k = threadIdx.x; k < nbk; k += kCB) bcnt[k] = 0;
        __syncthreads();
        const int64_t i1 = (ch + 1) * chunk < n ? (ch + 1) * chunk : n;
        for (int64_t t0 = ch * chunk; t0 < i1; t0 += kDfgTile) {
#pragma unroll
            for (int h = 0; h < kDfgTile / (4 * kCB); ++h) {
                const int64_t e0 = t0 + 4 * (h * kCB + (int64_t)threadIdx.x);
                if (t0 + 4 * h * kCB >= i1) break;   // block-uniform
                const Quad qd = load_quad<false, true>(case_s, act_s, nullptr, e0, i1, n, aligned);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (e0 + j >= i1) break;
                    const int32_t c = qd.c[j], a = qd.a[j];
                    if ((uint32_t)a >= (uint32_t)A) {
                        bad = true;
                        continue;
                    }
                    const int32_t cp = j ? qd.c[j - 1] : qd.cp;
                    const int32_t ap = j ? qd.a[j - 1] : qd.ap;
                    const int32_t cn = j < 3 ? qd.c[j + 1] : qd.cn;
                    const bool first = cp != c;
                    if (first) atomicAdd(&sstart[a], 1u);
                    if (e0 + j + 1 >= n || cn != c) atomicAdd(&send[a], 1u);
                    if (!first && (uint32_t)ap < (uint32_t)A)
                        atomicAdd(&bcnt[((uint32_t)ap * (uint32_t)A + (uint32_t)a) >> 12], 1u);
                }
            }
        }
        __syncthreads();
        for (int64_t k = threadIdx.x; k < nbk; k += kCB) ws.ecnt[k * nch + ch] = bcnt[k];
        __syncthreads();
    }
    __syncthreads();   // (a block without chunks: the zeroing above)
    if (__ballot(bad) != 0 && lane() == 0) set_status(status, PM4G_E_RANGE);
    const size_t ab = (size_t)blockIdx.x * A;
    for (int a = threadIdx.x; a < A; a += kCB) {
        ws.pstart[ab + a] = sstart[a];
        ws.pend[ab + a] = send[a];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ws.scal[0] = nbk * nch;
}

// Per chunk: every edge goes to its bucket's run (cursor seeded from the scan).
// Per 4096-event tile the edges are first grouped by bucket in LDS, then
// written out in bucket order, so each bucket's piece is one coalesced run.
// Span partial per block.  Dynamic LDS: 3 * nbk u32.
__global__ __launch_bounds__(kCB) void k_dfg_scatter(const int32_t* __restrict__ case_s,
                                                     const int32_t* __restrict__ act_s,
                                                     const int64_t* __restrict__ ts_s, int64_t n, int32_t A,
                                                     int64_t nbk, int64_t nch, int64_t chunk, DfgWs ws) {
    extern __shared__ uint32_t dsm[];
    uint32_t* cur = dsm;              // global cursor of each bucket
    uint32_t* lcnt = dsm + nbk;       // edges per bucket in this tile
    uint32_t* lstart = dsm + 2 * nbk; // their start in the staged tile
    __shared__ uint16_t s_cell[kDfgTile];
    __shared__ uint64_t s_gap[kDfgTile];
    __shared__ uint16_t s_bk[kDfgTile];
    __shared__ uint32_t tmp[kCB / kWave + 1];
    __shared__ uint64_t sspan[kCB / kWave];
    constexpr int kQ = kDfgTile / (4 * kCB);   // quads per thread per tile (2)
    const bool aligned = ((reinterpret_cast<uintptr_t>(case_s) | reinterpret_cast<uintptr_t>(act_s) |
                           reinterpret_cast<uintptr_t>(ts_s)) & 15) == 0;
    uint64_t span = 0;
    // chunks XCD-contiguous: a bucket's runs from neighbouring chunks are
    // neighbours in the output and meet in the same L2
    const XcdSplit xs = xcd_split(nch);
    for (int64_t ch = xs.first; ch < xs.end; ch += xs.stride) {
        for (int64_t k = threadIdx.x; k < nbk; k += kCB) cur[k] = ws.escan[k * nch + ch];
        const int64_t i1 = (ch + 1) * chunk < n ? (ch + 1) * chunk : n;
        for (int64_t t0 = ch * chunk; t0 < i1; t0 += kDfgTile) {
            for (int64_t k = threadIdx.x; k < nbk; k += kCB) lcnt[k] = 0;
            __syncthreads();
            // 1. edges of this thread's quads: bucket, slot in the bucket, cell, gap
            uint32_t eb[4 * kQ], ec[4 * kQ];
            uint64_t eg[4 * kQ];
#pragma unroll
            for (int h = 0; h < kQ; ++h) {
                const int64_t e0 = t0 + 4 * (h * kCB + (int64_t)threadIdx.x);
                Quad qd{};
                if (t0 + 4 * h * kCB < i1)   // block-uniform
                    qd = load_quad<true, false>(case_s, act_s, ts_s, e0, i1, n, aligned);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int u = 4 * h + j;
                    eb[u] = 0xFFFFFFFFu;
                    if (t0 + 4 * h * kCB >= i1) continue;
                    const int32_t cp = j ? qd.c[j - 1] : qd.cp;
                    const int32_t ap = j ? qd.a[j - 1] : qd.ap;
                    const int64_t tp = j ? qd.t[j - 1] : qd.tp;
                    if (e0 + j >= i1 || qd.c[j] != cp || (uint32_t)qd.a[j] >= (uint32_t)A ||
                        (uint32_t)ap >= (uint32_t)A)
                        continue;
                    const uint32_t cell = (uint32_t)ap * (uint32_t)A + (uint32_t)qd.a[j];
                    const uint64_t gap = (uint64_t)qd.t[j] - (uint64_t)tp;
                    span = sat_add63(span, cap63(gap));
                    const uint32_t b = cell >> 12;
                    const uint32_t slot = atomicAdd(&lcnt[b], 1u);
                    eb[u] = b | (slot << 16);   // nbk <= 4096, slot < 4096
                    ec[u] = cell & (kCellsPerTable - 1);
                    eg[u] = gap;
                }
            }
            __syncthreads();
            // 2. bucket starts inside the staged tile
            uint32_t E = 0;
            for (int64_t k0 = 0; k0 < nbk; k0 += kCB) {
                const int64_t k = k0 + threadIdx.x;
                const uint32_t v = k < nbk ? lcnt[k] : 0u;
                uint32_t total;
                const uint32_t ex = block_excl_sum<kCB>(v, tmp, &total);
                if (k < nbk) lstart[k] = E + ex;
                E += total;
            }
            __syncthreads();
            // 3. stage in bucket order
#pragma unroll
            for (int u = 0; u < 4 * kQ; ++u) {
                if (eb[u] == 0xFFFFFFFFu) continue;
                const uint32_t b = eb[u] & 0xFFFFu;
                const uint32_t at = lstart[b] + (eb[u] >> 16);
                s_cell[at] = (uint16_t)ec[u];
                s_gap[at] = eg[u];
                s_bk[at] = (uint16_t)b;
            }
            __syncthreads();
            // 4. coalesced runs out
            for (uint32_t i = threadIdx.x; i < E; i += kCB) {
                const uint32_t b = s_bk[i];
                const uint32_t g = cur[b] + (i - lstart[b]);
                ws.ecell[g] = s_cell[i];
                ws.egap[g] = s_gap[i];
            }
            __syncthreads();
            for (int64_t k = threadIdx.x; k < nbk; k += kCB) cur[k] += lcnt[k];
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) span = sat_add63(span, __shfl_xor(span, o));
    if (lane() == 0) sspan[threadIdx.x / kWave] = span;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int k = 0; k < kCB / kWave; ++k) s = sat_add63(s, sspan[k]);
        ws.pspan[blockIdx.x] = s;
    }
}

// Bucket bases and totals from the scan; every bucket cut into slots of about
// E/kDfgAggTarget edges.
__global__ __launch_bounds__(1024) void k_dfg_plan(int64_t nbk, int64_t nch, DfgWs ws) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
    const uint64_t all = *ws.utotal;
    uint64_t chunk = (all + kDfgAggTarget - 1) / kDfgAggTarget;
    if (chunk < 1) chunk = 1;
    uint32_t run = 0;
    for (int64_t b0 = 0; b0 < nbk; b0 += 1024) {
        const int64_t b = b0 + threadIdx.x;
        uint32_t sl = 0, tb = 0, base = 0;
        if (b < nbk && nch > 0) {   // no chunks (empty log): empty buckets
            base = ws.escan[b * nch];
            const uint32_t next = b + 1 < nbk ? ws.escan[(b + 1) * nch] : (uint32_t)all;
            tb = next - base;
            sl = (uint32_t)((tb + chunk - 1) / chunk);
        }
        uint32_t total;
        const uint32_t ex = block_excl_sum<1024>(sl, tmp, &total);
        if (b < nbk) {
            const uint32_t first = run + ex;
            ws.bbase[b] = base;
            ws.btotal[b] = tb;
            ws.bfirst[b] = first;
            ws.bslots[b] = sl;
            for (uint32_t s = 0; s < sl; ++s) {
                const uint64_t v0 = (uint64_t)s * chunk;
                const uint64_t v1 = v0 + chunk < tb ? v0 + chunk : tb;
                ws.plan[first + s] = make_int4((int)b, (int)v0, (int)v1, 0);
            }
        }
        run += total;
    }
    if (threadIdx.x == 0) *ws.nplan = run;
}

__device__ __forceinline__ void agg_edge(uint32_t* scount, uint64_t* ssum, int64_t* smin, int64_t* smax,
                                         uint32_t cell, uint64_t gap) {
    const int64_t gg = (int64_t)gap;
    atomicAdd(&scount[cell], 1u);
    atomicAdd(reinterpret_cast<unsigned long long*>(&ssum[cell]), (unsigned long long)gap);
    if (gg < __hip_atomic_load(&smin[cell], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
        __hip_atomic_fetch_min(&smin[cell], gg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (gg > __hip_atomic_load(&smax[cell], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
        __hip_atomic_fetch_max(&smax[cell], gg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One block per slot: its edges are one contiguous range of its bucket.
__global__ __launch_bounds__(kAB) void k_dfg_agg(DfgWs ws) {
    __shared__ uint32_t scount[kCellsPerTable];
    __shared__ uint64_t ssum[kCellsPerTable];
    __shared__ int64_t smin[kCellsPerTable];
    __shared__ int64_t smax[kCellsPerTable];

    const uint32_t g = blockIdx.x;
    if (g >= *ws.nplan) return;
    const int4 pl = ws.plan[g];
    for (int c = threadIdx.x; c < kCellsPerTable; c += kAB) {
        scount[c] = 0;
        ssum[c] = 0;
        smin[c] = INT64_MAX;
        smax[c] = INT64_MIN;
    }
    __syncthreads();
    const size_t at0 = (size_t)ws.bbase[pl.x];
    const int64_t v1 = pl.z;
    constexpr int kU = 4;   // edges in flight per thread
    int64_t v = pl.y + threadIdx.x;
    for (; v + (kU - 1) * kAB < v1; v += kU * kAB) {
        uint32_t cell[kU];
        uint64_t gap[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            cell[u] = ws.ecell[at0 + v + u * kAB];
            gap[u] = ws.egap[at0 + v + u * kAB];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) agg_edge(scount, ssum, smin, smax, cell[u], gap[u]);
    }
    for (; v < v1; v += kAB) agg_edge(scount, ssum, smin, smax, ws.ecell[at0 + v], ws.egap[at0 + v]);
    __syncthreads();
    const size_t slot = (size_t)g * kCellsPerTable;
    for (int c = threadIdx.x; c < kCellsPerTable; c += kAB) {
        ws.pcount[slot + c] = scount[c];
        ws.psum[slot + c] = ssum[c];
        ws.pmin[slot + c] = smin[c];
        ws.pmax[slot + c] = smax[c];
    }
}

// ---------------------------------------------------------------------------
// Fold partial tables into the dense outputs.
// direct_slots > 0: every cell's partials are slots 0..direct_slots-1 (LDS path).
// direct_slots == 0: cell -> bucket cell>>12 -> slots bfirst..bfirst+bslots.
__global__ __launch_bounds__(256) void k_dfg_reduce(int32_t A, int32_t direct_slots, DfgWs ws,
                                                    DfgOutDev out) {
    const int64_t cells = (int64_t)A * A;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= cells) return;
    int64_t lc, s0, s1;
    if (direct_slots > 0) {
        lc = e;
        s0 = 0;
        s1 = direct_slots;
    } else {
        const int64_t b = e >> 12;
        lc = e & (kCellsPerTable - 1);
        s0 = ws.bfirst[b];
        s1 = s0 + ws.bslots[b];
    }
    uint64_t cnt = 0, sum = 0;
    int64_t mn = INT64_MAX, mx = INT64_MIN;
    for (int64_t s = s0; s < s1; ++s) {
        const size_t at = (size_t)s * kCellsPerTable + lc;
        cnt += ws.pcount[at];
        sum += ws.psum[at];
        const int64_t a = ws.pmin[at], b = ws.pmax[at];
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    out.count[e] = (int64_t)cnt;
    out.dt_sum[e] = (int64_t)sum;
    out.dt_min[e] = mn;
    out.dt_max[e] = mx;
    if (out.dt_mean) out.dt_mean[e] = cnt ? (double)(int64_t)sum / (double)(int64_t)cnt : (double)NAN;
}

__global__ void k_dfg_zero_acts(int32_t A, DfgOutDev out) {
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < A; a += gridDim.x * blockDim.x)
        out.act_count[a] = out.start_count[a] = out.end_count[a] = 0;
}

// grid (ceil(A/256), kActRows): block (x, r) folds partial rows r, r+kActRows, ...
// freq_from_counts: every event of a valid log either starts its case or ends
// one directly-follows pair, so an activity's frequency is its start count plus
// its column of the pair counts (out.count, already reduced); rows of that
// column are folded as the partial rows are.
constexpr int kActRows = 32;
__global__ __launch_bounds__(256) void k_dfg_acts(int32_t A, int32_t nblk, bool freq_from_counts,
                                                  DfgWs ws, DfgOutDev out) {
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= A) return;
    uint64_t f = 0, st = 0, en = 0;
    for (int k = blockIdx.y; k < nblk; k += kActRows) {
        if (!freq_from_counts) f += ws.pfreq[(size_t)k * A + a];
        st += ws.pstart[(size_t)k * A + a];
        en += ws.pend[(size_t)k * A + a];
    }
    if (freq_from_counts) {
        f += st;
        for (int b = blockIdx.y; b < A; b += kActRows) f += (uint64_t)out.count[(size_t)b * A + a];
    }
    atomicAdd(reinterpret_cast<unsigned long long*>(&out.act_count[a]), (unsigned long long)f);
    atomicAdd(reinterpret_cast<unsigned long long*>(&out.start_count[a]), (unsigned long long)st);
    atomicAdd(reinterpret_cast<unsigned long long*>(&out.end_count[a]), (unsigned long long)en);
}

// One block: overflow flag from the span partials, n_cases = sum of start counts.
__global__ __launch_bounds__(1024) void k_dfg_final(int32_t A, int32_t nblk, DfgWs ws,
                                                    const int32_t* status_in, DfgOutDev out) {
    __shared__ uint64_t r1[1024 / kWave], r2[1024 / kWave];
    uint64_t sp = 0, c = 0;
    for (int k = threadIdx.x; k < nblk; k += 1024) sp = sat_add63(sp, ws.pspan[k]);
    for (int a = threadIdx.x; a < A; a += 1024) c += (uint64_t)out.start_count[a];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) sp = sat_add63(sp, __shfl_xor(sp, o));
    c = wave_sum(c);
    if (lane() == 0) {
        r1[threadIdx.x / kWave] = sp;
        r2[threadIdx.x / kWave] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0, t = 0;
        for (int k = 0; k < 1024 / kWave; ++k) {
            s = sat_add63(s, r1[k]);
            t += r2[k];
        }
        *out.overflow = s > (uint64_t)INT64_MAX ? 1 : 0;
        *out.n_cases = (int64_t)t;
        if (status_in && *status_in != 0) set_status(out.status, *status_in);
    }
}

static void launch_acts(int32_t A, int32_t nblk, bool freq_from_counts, DfgWs ws, const int32_t* status_in,
                        DfgOutDev out, hipStream_t s) {
    k_dfg_zero_acts<<<(unsigned)((A + 255) / 256), 256, 0, s>>>(A, out);
    k_dfg_acts<<<dim3((unsigned)((A + 255) / 256), kActRows), 256, 0, s>>>(A, nblk, freq_from_counts, ws, out);
    k_dfg_final<<<1, 1024, 0, s>>>(A, nblk, ws, status_in, out);
}

__global__ void k_status_init(int32_t* status) { *status = 0; }

hipError_t launch_dfg(const int32_t* case_s, const int32_t* act_s, const int64_t* ts_s, int64_t n,
                      int32_t A, const int32_t* status_in, DfgWs ws, DfgOutDev out, hipStream_t s) {
    k_status_init<<<1, 1, 0, s>>>(out.status);
    const int64_t cells = (int64_t)A * A;
    if (A <= kDfgLdsMaxA) {
        {
            ProfScope p(P_DFG_MAIN, s);
            k_dfg_lds<<<kDfgLdsBlocks, kLB, 0, s>>>(case_s, act_s, ts_s, n, A, ws, out.status);
        }
        ProfScope p(P_DFG_REDUCE, s);
        k_dfg_reduce<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(A, kDfgLdsBlocks, ws, out);
        launch_acts(A, kDfgLdsBlocks, false, ws, status_in, out, s);
    } else {
        const int64_t nbk = n_buckets(A);
        const int64_t nch = dfg_chunks(n, nbk);
        const int64_t chunk = dfg_chunk(nbk);
        const unsigned g = (unsigned)ws.n_act_blocks;
        {
            ProfScope p(P_DFG_COUNT, s);
            k_dfg_count<<<g, kCB, (size_t)(2 * A + nbk) * sizeof(uint32_t), s>>>(case_s, act_s, n, A, nbk, nch,
                                                                             chunk, ws, out.status);
            dev::excl_scan<uint32_t>(ws.ecnt, &ws.scal[0], ws.escan, ws.part32, ws.utotal, s);
        }
        {
            ProfScope p(P_DFG_MAIN, s);
            k_dfg_scatter<<<g, kCB, (size_t)3 * nbk * sizeof(uint32_t), s>>>(case_s, act_s, ts_s, n, A, nbk,
                                                                           nch, chunk, ws);
        }
        {
            ProfScope p(P_DFG_PLAN, s);
            k_dfg_plan<<<1, 1024, 0, s>>>(nbk, nch, ws);
        }
        {
            ProfScope p(P_DFG_AGG, s);
            k_dfg_agg<<<(unsigned)ws.n_slots_max, kAB, 0, s>>>(ws);
        }
        ProfScope p(P_DFG_REDUCE, s);
        k_dfg_reduce<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(A, 0, ws, out);
        launch_acts(A, ws.n_act_blocks, true, ws, status_in, out, s);
    }
    return hipGetLastError();
}

}  // namespace pm4g
