// Trace variants of a prepared log (Sec. 3, variant level: cases grouped by
// their activity sequence, an aggregation of the per-case aggregation; the
// cases dataframe carries numbers from which each case's variant follows).
//
// Grouping is exact: a 64-bit hash of each case's sequence (the numeric
// feature) only brings candidates together; every equal-hash neighbour pair
// is compared element by element, and a run of equal hashes holding more
// than one sequence is regrouped exactly.  Variant ids follow (count desc,
// representative asc) with the representative the smallest case id.
//
//   k_var_hash       per case: sum over positions of mix(position, activity), mixed
//                    with the length (wave-cooperative, coalesced)
//   radix (64 bits)  cases by hash; stable, so equal hashes keep case order
//   k_var_verify     neighbour sequences compared exactly -> group starts
//   k_var_fix        only after a true collision: exact regrouping of a run
//   scans            group ids; representatives (first member = smallest id)
//                    enumerated in case order = representative order
//   radix (count)    stable sort by descending count -> final ids
//   k_var_emit       counts, lengths, representatives, CSR sequences, ids
// All sizes (cases, variants) stay on the device; nothing synchronises.
#include "common.hpp"
#include "devsort.hpp"
#include "internal.hpp"
#include "prof.hpp"
#include "../../include/pm4g.h"

namespace pm4g {

VarWs var_ws_layout(Bump& b, int64_t n) {
    VarWs w{};
    const size_t m = (size_t)(n > 0 ? n : 1);
    w.hash = b.take<uint64_t>(m);
    w.hash2 = b.take<uint64_t>(m);
    w.idx = b.take<uint32_t>(m);
    w.idx2 = b.take<uint32_t>(m);
    w.hist = b.take<uint32_t>(256 * (size_t)(dev::tiles(n) + 1));
    w.rowsum = b.take<uint32_t>(256);
    w.flag = b.take<uint32_t>(m);
    w.sid = b.take<uint32_t>(m);
    w.sstart = b.take<uint32_t>(m + 1);
    w.repflag = b.take<uint32_t>(m);
    w.rrank = b.take<uint32_t>(m);
    w.vcr = b.take<uint2>(m);
    w.cvar = b.take<uint32_t>(m);
    w.vkey = b.take<uint32_t>(m);
    w.vkey2 = b.take<uint32_t>(m);
    w.vidx = b.take<uint32_t>(m);
    w.vidx2 = b.take<uint32_t>(m);
    w.fid = b.take<uint32_t>(m);
    w.lens = b.take<uint32_t>(m);
    w.part32 = b.take<uint32_t>(dev::kScanGrid);
    w.part64 = b.take<int64_t>(dev::kScanGrid);
    w.scal = b.take<int64_t>(8);
    w.u32scal = b.take<uint32_t>(8);
    return w;
}

namespace {

constexpr int kGrid = 2048;
constexpr int kBlk = 256;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ bool same_seq(const int32_t* act_s, const int64_t* case_off, uint32_t a, uint32_t b) {
    const int64_t a0 = case_off[a], a1 = case_off[a + 1];
    const int64_t b0 = case_off[b], b1 = case_off[b + 1];
    if (a1 - a0 != b1 - b0) return false;
    for (int64_t k = 0; k < a1 - a0; ++k)
        if (act_s[a0 + k] != act_s[b0 + k]) return false;
    return true;
}

__global__ void k_var_init(VarWs w, const int64_t* n_cases) {
    if (threadIdx.x == 0) {
        w.scal[0] = *n_cases;   // C
        w.scal[1] = 0;          // V (filled later)
        w.u32scal[0] = 0;       // collisions
        w.u32scal[1] = 0;       // V (u32)
    }
}

// Wave-cooperative walk over 64 consecutive segments: lane m holds the
// virtual start of segment m (INT64_MAX if absent); returns the segment that
// contains virtual position p (the last m with start_m <= p).  Starts are
// strictly increasing (segments are non-empty) and p >= start_0.  Must be
// called with all 64 lanes active (the shuffles read every lane).
__device__ __forceinline__ int seg_of(int64_t vstart, int64_t p) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int cand = lo + step;
        if (__shfl(vstart, cand) <= p) lo = cand;
    }
    return lo;
}

// The same search over 32-bit starts (one lane exchange per step instead of two).
__device__ __forceinline__ int seg_of32(int32_t vstart, int64_t p) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int cand = lo + step;
        if ((int64_t)__shfl(vstart, cand) <= p) lo = cand;
    }
    return lo;
}

// Sequence hash of every case: a sum over positions of mix(position, activity)
// (order-sensitive, computable in any order), mixed with the length.  A wave
// takes 64 consecutive cases; their events are read in 1024-event windows
// with coalesced 16-byte loads into LDS, then each lane sums 16 consecutive
// events, adding a case's partial sum to its LDS total when it leaves the case
// (so a case costs one or two LDS additions, not one per event).
constexpr int kHashWin = 1024;
__global__ __launch_bounds__(kBlk) void k_var_hash(const int32_t* __restrict__ act_s,
                                                   const int64_t* __restrict__ case_off, VarWs w,
                                                   uint64_t mask, int64_t n) {
    __shared__ unsigned long long hsum[kBlk / kWave][kWave];
    __shared__ int64_t sst[kBlk / kWave][kWave + 1];
    __shared__ int32_t sact[kBlk / kWave][kHashWin];
    const int64_t C = w.scal[0];
    const int wl = threadIdx.x / kWave;
    const int64_t wv = ((int64_t)blockIdx.x * kBlk + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * kBlk / kWave;
    const bool aligned = (reinterpret_cast<uintptr_t>(act_s) & 15) == 0;
    constexpr int kPer = kHashWin / kWave;   // 16 events per lane and window
    for (int64_t c0 = wv * kWave; c0 < C; c0 += nw * kWave) {
        const int64_t c = c0 + lane();
        const bool has = c < C;
        const int64_t st = has ? case_off[c] : INT64_MAX;
        const int64_t en = has ? case_off[c + 1] : 0;
        hsum[wl][lane()] = 0;
        sst[wl][lane()] = st;
        if (lane() == 0) sst[wl][kWave] = INT64_MAX;
        const int last = (C - 1 - c0) < (kWave - 1) ? (int)(C - 1 - c0) : (kWave - 1);
        const int64_t base = __shfl(st, 0);
        const int64_t end = __shfl(en, last);
        for (int64_t w0 = base & ~(int64_t)3; w0 < end; w0 += kHashWin) {   // wave-uniform
            // stage the window's activities (positions outside [base, end) are not used);
            // the 16-byte loads take in-bounds positions with no branch around them
            // and are all issued before the first store (a quad past n - 4 re-reads
            // the last aligned quad and is replaced below)
            constexpr int kQ = kHashWin / (4 * kWave);
            int4 v[kQ];
            const bool vec = aligned && n >= 4;
            const int64_t plast = (n - 4) & ~(int64_t)3;
#pragma unroll
            for (int k = 0; k < kQ; ++k) {
                const int64_t p = w0 + 4 * (k * kWave + lane());
                if (vec) v[k] = *reinterpret_cast<const int4*>(act_s + (p + 3 < n ? p : plast));
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < kQ; ++k) {
                const int o = 4 * (k * kWave + lane());
                const int64_t p = w0 + o;
                if (vec && p + 3 < n) {
                    sact[wl][o] = v[k].x;
                    sact[wl][o + 1] = v[k].y;
                    sact[wl][o + 2] = v[k].z;
                    sact[wl][o + 3] = v[k].w;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) sact[wl][o + j] = p + j < n ? act_s[p + j] : 0;
                }
            }
            // lane-contiguous sums
            const int64_t q0 = w0 + (int64_t)kPer * lane();
            const int64_t lo = q0 > base ? q0 : base;
            const int64_t hi = (q0 + kPer) < end ? (q0 + kPer) : end;
            int m = seg_of(st, lo < end ? lo : end - 1);   // all lanes active
            int64_t s_m = sst[wl][m], nxt = sst[wl][m + 1];
            uint64_t acc = 0;
            for (int64_t p = lo; p < hi; ++p) {
                if (p >= nxt) {   // cases are non-empty: one step at a time
                    atomicAdd(&hsum[wl][m], (unsigned long long)acc);
                    acc = 0;
                    ++m;
                    s_m = nxt;
                    nxt = sst[wl][m + 1];
                }
                acc += mix64(((uint64_t)(p - s_m) << 13) + (uint64_t)(uint32_t)sact[wl][p - w0] +
                             0x632be59bd9b4e019ull);
            }
            if (lo < hi) atomicAdd(&hsum[wl][m], (unsigned long long)acc);
        }
        if (has) {
            uint64_t h = mix64((uint64_t)hsum[wl][lane()] ^ mix64((uint64_t)(en - st) + 0x9e3779b97f4a7c15ull));
            if (mask) h &= mask;
            w.hash[c] = h;
            w.idx[c] = (uint32_t)c;
            w.repflag[c] = 0;
        }
    }
}

__global__ __launch_bounds__(kBlk) void k_var_verify(const uint64_t* __restrict__ hs,
                                                     const uint32_t* __restrict__ is,
                                                     const int32_t* __restrict__ act_s,
                                                     const int64_t* __restrict__ case_off, VarWs w) {
    const int64_t C = w.scal[0];
    for (int64_t p = (int64_t)blockIdx.x * kBlk + threadIdx.x; p < C; p += (int64_t)gridDim.x * kBlk) {
        uint32_t f = 1;
        if (p > 0 && hs[p] == hs[p - 1]) {
            if (same_seq(act_s, case_off, is[p], is[p - 1])) f = 0;
            else atomicOr(&w.u32scal[0], 1u);
        }
        w.flag[p] = f;
    }
}

// Exact regrouping of equal-hash runs that hold several sequences.  Only does
// work after a true hash collision; one thread per affected run.
__global__ __launch_bounds__(kBlk) void k_var_fix(const uint64_t* __restrict__ hs, uint32_t* is,
                                                  const int32_t* __restrict__ act_s,
                                                  const int64_t* __restrict__ case_off, VarWs w) {
    if (w.u32scal[0] == 0) return;
    const int64_t C = w.scal[0];
    uint32_t* out = w.vidx2;     // scratch
    uint32_t* mark = w.vkey2;    // scratch
    for (int64_t p = (int64_t)blockIdx.x * kBlk + threadIdx.x; p < C; p += (int64_t)gridDim.x * kBlk) {
        if (p > 0 && hs[p] == hs[p - 1]) continue;   // not a run start
        int64_t q = p + 1;
        bool mixed = false;
        while (q < C && hs[q] == hs[p]) {
            mixed |= w.flag[q] != 0;
            ++q;
        }
        if (!mixed) continue;
        for (int64_t a = p; a < q; ++a) mark[a] = 0;
        int64_t o = p;
        for (int64_t a = p; a < q; ++a) {
            if (mark[a]) continue;
            const uint32_t lead = is[a];
            mark[a] = 1;
            out[o] = lead;
            w.flag[o] = 1;
            ++o;
            for (int64_t b = a + 1; b < q; ++b) {
                if (!mark[b] && same_seq(act_s, case_off, is[b], lead)) {
                    mark[b] = 1;
                    out[o] = is[b];
                    w.flag[o] = 0;
                    ++o;
                }
            }
        }
        for (int64_t a = p; a < q; ++a) is[a] = out[a];
    }
}

// sid = inclusive group index (after the exclusive scan of flags + flag - 1).
__global__ __launch_bounds__(kBlk) void k_var_groups(const uint32_t* __restrict__ is, VarWs w) {
    const int64_t C = w.scal[0];
    for (int64_t p = (int64_t)blockIdx.x * kBlk + threadIdx.x; p < C; p += (int64_t)gridDim.x * kBlk) {
        if (w.flag[p]) {
            const uint32_t g = w.sid[p];       // exclusive count of starts before p
            w.sstart[g] = (uint32_t)p;
            w.repflag[is[p]] = 1;              // first member: smallest case index
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t V = w.u32scal[1];
        w.sstart[V] = (uint32_t)C;
        w.scal[1] = V;
    }
}

// Per group (hash order): count and representative, stored at the group's
// representative-order index v (one 8-byte scattered write); the group's v
// is kept in hash order (gv, coalesced) for the per-case pass.
__global__ __launch_bounds__(kBlk) void k_var_segments(const uint32_t* __restrict__ is, VarWs w) {
    const int64_t V = w.scal[1];
    uint32_t* gv = w.repflag;   // free again after the representative scan
    for (int64_t g = (int64_t)blockIdx.x * kBlk + threadIdx.x; g < V; g += (int64_t)gridDim.x * kBlk) {
        const uint32_t s0 = w.sstart[g], s1 = w.sstart[g + 1];
        const uint32_t rep = is[s0];
        const uint32_t v = w.rrank[rep];
        w.vcr[v] = make_uint2(s1 - s0, rep);
        gv[g] = v;
    }
}

// Sort input of the final order (ascending key = descending count, stable on
// the representative order), and every case's representative-order variant.
__global__ __launch_bounds__(kBlk) void k_var_keys(const uint32_t* __restrict__ is, VarWs w) {
    const int64_t C = w.scal[0];
    const int64_t V = w.scal[1];
    const uint32_t* gv = w.repflag;
    for (int64_t v = (int64_t)blockIdx.x * kBlk + threadIdx.x; v < V; v += (int64_t)gridDim.x * kBlk) {
        w.vkey[v] = (uint32_t)C - w.vcr[v].x;
        w.vidx[v] = (uint32_t)v;
    }
    for (int64_t p = (int64_t)blockIdx.x * kBlk + threadIdx.x; p < C; p += (int64_t)gridDim.x * kBlk) {
        // group of p: flags up to p, minus one
        const uint32_t g = w.sid[p] + w.flag[p] - 1;
        w.cvar[is[p]] = gv[g];
    }
}

__global__ __launch_bounds__(kBlk) void k_var_ids(const uint32_t* __restrict__ order, VarWs w,
                                                  const int64_t* __restrict__ case_off,
                                                  const int32_t* __restrict__ case_code, VarOutDev out) {
    const int64_t V = w.scal[1];
    for (int64_t k = (int64_t)blockIdx.x * kBlk + threadIdx.x; k < V; k += (int64_t)gridDim.x * kBlk) {
        const uint32_t v = order[k];
        w.fid[v] = (uint32_t)k;
        const uint2 cr = w.vcr[v];
        const uint32_t r = cr.y;
        const uint32_t L = (uint32_t)(case_off[r + 1] - case_off[r]);
        out.var_count[k] = cr.x;
        out.var_rep[k] = case_code[r];
        out.var_len[k] = (int32_t)L;
        w.lens[k] = L;
    }
}

// Sequences in final order: a wave takes 64 consecutive variants and copies
// their representatives' activities, writes coalesced over the output range.
__global__ __launch_bounds__(kBlk) void k_var_emit(const uint32_t* __restrict__ order,
                                                   const int32_t* __restrict__ act_s,
                                                   const int64_t* __restrict__ case_off, VarWs w,
                                                   const int32_t* status_in, VarOutDev out) {
    const int64_t C = w.scal[0];
    const int64_t V = w.scal[1];
    const int64_t wv = ((int64_t)blockIdx.x * kBlk + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * kBlk / kWave;
    for (int64_t k0 = wv * kWave; k0 < V; k0 += nw * kWave) {
        const int64_t k = k0 + lane();
        const bool has = k < V;
        int64_t src = 0, dst = INT64_MAX, len = 0;
        if (has) {
            const uint32_t r = w.vcr[order[k]].y;
            src = case_off[r];
            len = case_off[r + 1] - src;
            dst = out.var_off[k];
        }
        const int last = (V - 1 - k0) < (kWave - 1) ? (int)(V - 1 - k0) : (kWave - 1);
        const int64_t base = __shfl(dst, 0);
        const int64_t end = __shfl(dst + len, last);
        // event positions are below 2^31 (the log's size limit), so output
        // starts and the source-minus-output shift fit 32 bits: the search and
        // the shift take one lane exchange each instead of two
        const int32_t dst32 = has ? (int32_t)dst : INT32_MAX;
        const int32_t shift = (int32_t)(src - (has ? dst : 0));
        // wave-uniform trip count: every lane takes part in the shuffles;
        // four 64-element steps per trip, their loads issued first
        constexpr int kU = 4;
        for (int64_t p0 = base; p0 < end; p0 += kU * kWave) {
            int32_t av[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t p = p0 + u * kWave + lane();
                const int m = seg_of32(dst32, p);
                const int32_t sh = __shfl(shift, m);
                av[u] = p < end ? act_s[p + sh] : 0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t p = p0 + u * kWave + lane();
                if (p < end) out.var_acts[p] = av[u];
            }
        }
    }
    if (out.case_variant) {
        for (int64_t c = (int64_t)blockIdx.x * kBlk + threadIdx.x; c < C; c += (int64_t)gridDim.x * kBlk)
            out.case_variant[c] = (int32_t)w.fid[w.cvar[c]];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        out.var_off[V] = w.scal[2];
        *out.n_variants = V;
        *out.status = status_in ? *status_in : 0;
    }
}

int bits_for(int64_t n) {
    int b = 0;
    while (b < 63 && (int64_t(1) << b) <= n) ++b;
    return b;
}

}  // namespace

hipError_t launch_variants(const int32_t* act_s, const int64_t* case_off, const int32_t* case_code,
                           const int64_t* n_cases, const int32_t* status_in, int64_t n, VarWs w,
                           VarOutDev out, uint32_t debug_hash_bits, hipStream_t s) {
    const uint64_t mask = (debug_hash_bits == 0 || debug_hash_bits >= 64)
                              ? 0ull
                              : ((uint64_t(1) << debug_hash_bits) - 1);
    k_var_init<<<1, 1, 0, s>>>(w, n_cases);
    {
        ProfScope p(P_VAR_HASH, s);
        k_var_hash<<<kGrid, kBlk, 0, s>>>(act_s, case_off, w, mask, n);
    }
    bool in2;
    {
        ProfScope p(P_VAR_SORT, s);
        in2 = dev::sort_pairs<uint64_t>(w.hash, w.idx, w.hash2, w.idx2, &w.scal[0], n, 64, w.hist,
                                        w.rowsum, s);
    }
    const uint64_t* hs = in2 ? w.hash2 : w.hash;
    uint32_t* is = in2 ? w.idx2 : w.idx;
    {
        ProfScope p(P_VAR_GROUP, s);
        k_var_verify<<<kGrid, kBlk, 0, s>>>(hs, is, act_s, case_off, w);
        k_var_fix<<<kGrid, kBlk, 0, s>>>(hs, is, act_s, case_off, w);
        // group index of every group start; V
        dev::excl_scan<uint32_t>(w.flag, &w.scal[0], w.sid, w.part32, &w.u32scal[1], s);
        k_var_groups<<<kGrid, kBlk, 0, s>>>(is, w);
        // representative-order index of every representative case
        dev::excl_scan<uint32_t>(w.repflag, &w.scal[0], w.rrank, w.part32, (uint32_t*)nullptr, s);
        k_var_segments<<<kGrid, kBlk, 0, s>>>(is, w);
        k_var_keys<<<kGrid, kBlk, 0, s>>>(is, w);
    }
    bool o2;
    {
        ProfScope p(P_VAR_ORDER, s);
        o2 = dev::sort_pairs<uint32_t>(w.vkey, w.vidx, w.vkey2, w.vidx2, &w.scal[1], n, bits_for(n),
                                       w.hist, w.rowsum, s);
    }
    const uint32_t* order = o2 ? w.vidx2 : w.vidx;
    ProfScope p(P_VAR_EMIT, s);
    k_var_ids<<<kGrid, kBlk, 0, s>>>(order, w, case_off, case_code, out);
    dev::excl_scan<int64_t>(w.lens, &w.scal[1], out.var_off, w.part64, &w.scal[2], s);
    k_var_emit<<<kGrid, kBlk, 0, s>>>(order, act_s, case_off, w, status_in, out);
    return hipGetLastError();
}

}  // namespace pm4g
