// Eventually-follows graph and temporal profile of a prepared log (Sec. 3:
// the EFG / temporal-profile module).  Every pair of events (i, j) of a case
// with i before j in the (case, timestamp, row) order counts for cell
// (a_i, a_j) with gap d = t_j - t_i; per cell: the number of pairs, the exact
// sum of the gaps (128-bit), the sum of their squares modulo 2^128, and from
// them the FP64 mean and sample standard deviation.
//
// The work is the pairs (sum over cases of L(L-1)/2), not the events, so the
// kernels spread pairs, not events, over the chip:
//   k_efg_tail     per event: the number of later events of its case (a wave
//                  walks the events of 64 consecutive cases, coalesced)
//   buckets        when A*A exceeds one LDS table (4096 cells), the events
//                  that have a later event are grouped by bucket of R source
//                  activities (R*A <= 4096): k_efg_bcount, scan, k_efg_bscatter;
//                  otherwise the list is the log itself
//   scan           int64 pair offsets over the list
//   k_efg_plan     each bucket gets plan entries in proportion to its pairs,
//                  each an equal range of the bucket's pairs
//   k_efg_agg      a block per entry (LDS-bound: one per CU): each wave takes
//                  64 source events, flattens their pairs across its lanes and
//                  adds the gaps into the block's LDS table (count, gap sum
//                  with carry count, 128-bit square sum); the table goes to
//                  the entry's partial slot
//   k_efg_reduce   per cell: the partial slots of its bucket summed exactly,
//                  then mean and std
// Bytes: 4 B/event tail + (buckets) 8 B/event list and 4 B/event of counting
// pass, 8 B/list entry of offsets; per pair 12 B of (act, ts) read through the
// caches (the later events of a case are contiguous) and 3-5 LDS atomics,
// which bound the kernel.
#include "common.hpp"
#include "devsort.hpp"
#include "internal.hpp"
#include "prof.hpp"
#include "../../include/pm4g.h"

namespace pm4g {

namespace {

constexpr int kEfgAggGrid = 256;         // one block per CU (128 KB of LDS each)
constexpr int kEB = 1024;                // threads of an aggregation block
constexpr int64_t kEfgSeg = int64_t(1) << 31;   // pairs per LDS pass (u32 counters)

}  // namespace

int efg_rows(int32_t A) { return A * A <= kEfgCells ? A : (kEfgCells / A > 0 ? kEfgCells / A : 1); }

int64_t efg_buckets(int32_t A) {
    const int R = efg_rows(A);
    return (A + R - 1) / R;
}

EfgWs efg_ws_layout(Bump& b, int64_t n, int32_t A) {
    EfgWs w{};
    const size_t m = (size_t)(n > 0 ? n : 1);
    const int64_t nbk = efg_buckets(A);
    const int64_t nch = (n + kEfgChunk - 1) / kEfgChunk;
    w.tail = b.take<uint32_t>(m);
    w.poff = b.take<int64_t>(m + 1);
    if (nbk > 1) {
        w.list = b.take<uint32_t>(m);
        w.tl = b.take<uint32_t>(m);
        w.bcnt = b.take<uint32_t>((size_t)(nbk * (nch > 0 ? nch : 1)));
        w.boff = b.take<int64_t>((size_t)(nbk * (nch > 0 ? nch : 1)));
    }
    w.part64 = b.take<int64_t>(dev::kScanGrid);
    w.scal = b.take<int64_t>(8);
    w.bfirst = b.take<int64_t>((size_t)nbk);
    w.bnum = b.take<int64_t>((size_t)nbk);
    w.plan = b.take<EfgEntry>((size_t)(kEfgPlanBlocks + nbk));
    w.part = b.take<uint64_t>((size_t)(kEfgPlanBlocks + nbk) * kSlotWords);
    return w;
}

namespace {

// scal: [0] n, [1] list length, [2] total pairs, [3] plan entries, [4] bucket
// counters (nbk * chunks)
__global__ void k_efg_setup(EfgWs w, int64_t n, int64_t ncounters) {
    w.scal[0] = n;
    w.scal[1] = n;   // the log itself unless bucketed
    w.scal[4] = ncounters;
}

__global__ __launch_bounds__(256) void k_efg_tail(const int64_t* __restrict__ case_off, const int64_t* n_cases,
                                                  uint32_t* __restrict__ tail) {
    const int64_t C = *n_cases;
    const int64_t wv = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * 256 / kWave;
    for (int64_t c0 = wv * kWave; c0 < C; c0 += nw * kWave) {
        const int64_t c = c0 + lane();
        const bool has = c < C;
        const int64_t st = has ? case_off[c] : INT64_MAX;
        const int64_t en = has ? case_off[c + 1] : 0;
        const int last = (C - 1 - c0) < (kWave - 1) ? (int)(C - 1 - c0) : (kWave - 1);
        const int64_t base = __shfl(st, 0);
        const int64_t end = __shfl(en, last);
        for (int64_t p0 = base; p0 < end; p0 += kWave) {   // wave-uniform trip count
            const int64_t p = p0 + lane();
            const int m = seg_at(st, p);
            const int64_t e_m = __shfl(en, m);
            if (p < end) tail[p] = (uint32_t)(e_m - p - 1);
        }
    }
}

// Per chunk of the log, the events with a later event per bucket of source
// activity: bcnt[bucket * chunks + chunk].  Increments are wave-aggregated
// (one LDS atomic per distinct bucket of a wave): the Zipf-skewed activities
// put most of a wave into a few buckets.
__global__ __launch_bounds__(256) void k_efg_bcount(const int32_t* __restrict__ act_s,
                                                    const uint32_t* __restrict__ tail, int64_t n, int32_t R,
                                                    int64_t nbk, int32_t kbits, int64_t nch,
                                                    uint32_t* __restrict__ bcnt) {
    __shared__ uint32_t h[kEfgCells];
    for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        for (int64_t b = threadIdx.x; b < nbk; b += 256) h[b] = 0;
        __syncthreads();
        for (int q = 0; q < kEfgChunk / 256; ++q) {
            const int64_t p = ch * kEfgChunk + q * 256 + threadIdx.x;
            const bool has = p < n && tail[p] > 0;
            (void)wave_bump(h, has ? (uint32_t)(act_s[p] / R) : 0u, kbits, has);
        }
        __syncthreads();
        for (int64_t b = threadIdx.x; b < nbk; b += 256) bcnt[b * nch + ch] = h[b];
        __syncthreads();
    }
}

// The chunk's events go to LDS in bucket order first (wave-aggregated cursors),
// then out as one contiguous run per bucket, so the stores coalesce.
__global__ __launch_bounds__(256) void k_efg_bscatter(const int32_t* __restrict__ act_s,
                                                      const uint32_t* __restrict__ tail, int64_t n, int32_t R,
                                                      int64_t nbk, int32_t kbits, int64_t nch, EfgWs w) {
    __shared__ uint32_t cur[kEfgCells];      // staging cursor, then the global offset - local start
    __shared__ uint32_t lstart[kEfgCells];   // bucket's first staging slot
    __shared__ uint32_t st_p[kEfgChunk];
    __shared__ uint32_t st_t[kEfgChunk];
    __shared__ uint16_t st_b[kEfgChunk];
    __shared__ uint32_t tmp[256 / kWave + 1];
    const XcdSplit xs = xcd_split(nch);   // a bucket's runs of neighbouring chunks meet in one L2
    for (int64_t ch = xs.first; ch < xs.end; ch += xs.stride) {
        uint32_t run = 0;
        for (int64_t b0 = 0; b0 < nbk; b0 += 256) {
            const int64_t b = b0 + threadIdx.x;
            const uint32_t v = b < nbk ? w.bcnt[b * nch + ch] : 0u;
            uint32_t tot;
            const uint32_t ex = run + block_excl_sum<256>(v, tmp, &tot);
            if (b < nbk) {
                lstart[b] = ex;
                cur[b] = ex;
            }
            run += tot;
        }
        __syncthreads();
        for (int q = 0; q < kEfgChunk / 256; ++q) {
            const int64_t p = ch * kEfgChunk + q * 256 + threadIdx.x;
            const uint32_t t = p < n ? tail[p] : 0u;
            const bool has = t > 0;
            const uint32_t bk = has ? (uint32_t)(act_s[p] / R) : 0u;
            const uint32_t x = wave_bump(cur, bk, kbits, has);
            if (has) {
                st_p[x] = (uint32_t)p;
                st_t[x] = t;
                st_b[x] = (uint16_t)bk;
            }
        }
        __syncthreads();
        for (int64_t b = threadIdx.x; b < nbk; b += 256) cur[b] = (uint32_t)w.boff[b * nch + ch] - lstart[b];
        __syncthreads();
        for (uint32_t x = threadIdx.x; x < run; x += 256) {
            const uint32_t k = cur[st_b[x]] + x;
            w.list[k] = st_p[x];
            w.tl[k] = st_t[x];
        }
        __syncthreads();
    }
}

// Bucket b's list range [klo, khi) and its pairs [q0, q0 + pb).
__device__ __forceinline__ void efg_bucket(const EfgWs& w, int64_t b, int64_t nbk, int64_t nch, int64_t len,
                                           int64_t P, int64_t& klo, int64_t& khi, int64_t& q0, int64_t& pb) {
    klo = nbk > 1 ? w.boff[b * nch] : 0;
    khi = nbk > 1 ? (b + 1 < nbk ? w.boff[(b + 1) * nch] : len) : len;
    q0 = klo < len ? w.poff[klo] : P;
    const int64_t q1 = khi < len ? w.poff[khi] : P;
    pb = q1 - q0;
}

// One block of 1024 threads.  A bucket with pb pairs gets ceil(pb * G / P)
// entries (so at most G + buckets in all), equal shares of its pairs; first the
// per-bucket entry counts and their scan, then the entries in parallel.
__global__ __launch_bounds__(1024) void k_efg_plan(EfgWs w, int64_t nbk, int64_t nch, int32_t G) {
    __shared__ int64_t tmp[1024 / kWave + 1];
    __shared__ int64_t s_total;
    const int64_t len = w.scal[1], P = w.scal[2];
    if (threadIdx.x == 0) w.poff[len] = P;
    int64_t run = 0;
    for (int64_t b0 = 0; b0 < nbk; b0 += 1024) {
        const int64_t b = b0 + threadIdx.x;
        int64_t nb = 0;
        if (b < nbk && len > 0) {
            int64_t klo, khi, q0, pb;
            efg_bucket(w, b, nbk, nch, len, P, klo, khi, q0, pb);
            if (pb > 0) {
                const unsigned __int128 x = (unsigned __int128)pb * (unsigned)G;
                nb = (int64_t)((x + (unsigned __int128)(P - 1)) / (unsigned __int128)P);
                if (nb < 1) nb = 1;
            }
        }
        int64_t total;
        const int64_t first = run + block_excl_sum<1024>(nb, tmp, &total);
        if (b < nbk) {
            w.bfirst[b] = first;
            w.bnum[b] = nb;
        }
        run += total;
    }
    if (threadIdx.x == 0) {
        w.scal[3] = run;
        s_total = run;
    }
    __syncthreads();   // bfirst / bnum visible to the block
    const int64_t nplan = s_total;
    for (int64_t e = threadIdx.x; e < nplan; e += 1024) {
        // the last bucket whose first entry is <= e (buckets without entries share
        // their first entry with the next bucket, so this one has entries)
        int64_t lo = 0, hi = nbk;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (w.bfirst[mid] <= e) lo = mid;
            else hi = mid;
        }
        const int64_t b = lo, nb = w.bnum[b], r = e - w.bfirst[b];
        int64_t klo, khi, q0, pb;
        efg_bucket(w, b, nbk, nch, len, P, klo, khi, q0, pb);
        const int64_t base = pb / nb, rem = pb % nb;
        EfgEntry en;
        en.q0 = q0 + r * base + (r < rem ? r : rem);
        en.q1 = q0 + (r + 1) * base + (r + 1 < rem ? r + 1 : rem);
        en.klo = klo;
        en.khi = khi;
        en.b = (int32_t)b;
        en.pad = 0;
        w.plan[e] = en;
    }
}

__device__ __forceinline__ int64_t shfl64(int64_t v, int src) {
    const int lo = __shfl((int)(uint32_t)v, src);
    const int hi = __shfl((int)(uint32_t)((uint64_t)v >> 32), src);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__global__ __launch_bounds__(kEB) void k_efg_agg(const int32_t* __restrict__ act_s,
                                                 const int64_t* __restrict__ ts_s, EfgWs w, int32_t A, int32_t R,
                                                 int32_t bucketed, int64_t seg) {
    __shared__ uint32_t s_cnt[kEfgCells];
    __shared__ uint64_t s_slo[kEfgCells];
    __shared__ uint32_t s_shi[kEfgCells];   // carries out of s_slo
    __shared__ uint64_t s_qlo[kEfgCells];
    __shared__ uint64_t s_qhi[kEfgCells];
    __shared__ int64_t s_k0;
    const int64_t nplan = w.scal[3];
    const int cells = R * A;
    const int wv = threadIdx.x / kWave;
    constexpr int kNW = kEB / kWave;
    for (int64_t e = blockIdx.x; e < nplan; e += gridDim.x) {
        const EfgEntry en = w.plan[e];
        uint64_t* slot = w.part + e * (int64_t)kSlotWords;
        bool first = true;
        for (int64_t s0 = en.q0; s0 < en.q1; s0 += seg) {
            const int64_t s1 = (en.q1 - s0) < seg ? en.q1 : s0 + seg;
            for (int c = threadIdx.x; c < cells; c += kEB) {
                s_cnt[c] = 0;
                s_slo[c] = 0;
                s_shi[c] = 0;
                s_qlo[c] = 0;
                s_qhi[c] = 0;
            }
            if (threadIdx.x == 0) {   // the list entry whose pairs hold s0
                int64_t lo = en.klo, hi = en.khi;
                while (hi - lo > 1) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (w.poff[mid] <= s0) lo = mid;
                    else hi = mid;
                }
                s_k0 = lo;
            }
            __syncthreads();
            const int64_t kstart = s_k0;
            for (int64_t k0 = kstart + (int64_t)kWave * wv; k0 < en.khi; k0 += (int64_t)kWave * kNW) {
                if (w.poff[k0] >= s1) break;   // same address in every lane: wave-uniform
                const int64_t k = k0 + lane();
                const bool valid = k < en.khi;
                const int64_t beg = valid ? w.poff[k] : s1;
                const int64_t end = valid ? w.poff[k + 1] : s1;
                const int64_t lo = beg > s0 ? beg : s0;
                const int64_t hi = end < s1 ? end : s1;
                // within one pass the wave's pairs number at most s1 - s0 <= 2^31,
                // so the flattened offsets are 32-bit
                const uint32_t cnt = hi > lo ? (uint32_t)(hi - lo) : 0u;
                const uint32_t incl = wave_incl_sum(cnt);
                const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1);
                const int64_t src = valid ? (bucketed ? (int64_t)w.list[k] : k) : 0;
                const int32_t row = valid ? act_s[src] - en.b * R : 0;
                const int64_t ti = valid ? ts_s[src] : 0;
                // the p-th flattened pair of this lane's source is its event jb + p
                // (modulo 2^32; events are below 2^31)
                const uint32_t jb = (uint32_t)(src + 1 + (lo - beg)) - (incl - cnt);
                for (uint32_t p0 = 0; p0 < total; p0 += kWave) {   // wave-uniform trip count
                    const uint32_t p = p0 + lane();
                    int m = 0;   // lanes whose inclusive pair count is <= p
#pragma unroll
                    for (int step = 32; step > 0; step >>= 1)
                        if ((uint32_t)__shfl((int)incl, m + step - 1) <= p) m += step;
                    const int64_t jm = (int64_t)(uint32_t)((uint32_t)__shfl((int)jb, m) + p);
                    const int32_t rm = __shfl(row, m);
                    const int64_t tm = shfl64(ti, m);
                    if (p < total) {
                        const int cell = rm * A + act_s[jm];
                        const uint64_t d = (uint64_t)ts_s[jm] - (uint64_t)tm;
                        atomicAdd(&s_cnt[cell], 1u);
                        const unsigned long long os = atomicAdd((unsigned long long*)&s_slo[cell], (unsigned long long)d);
                        if (os + d < os) atomicAdd(&s_shi[cell], 1u);
                        const uint64_t ql = d * d, qh = __umul64hi(d, d);
                        const unsigned long long oq = atomicAdd((unsigned long long*)&s_qlo[cell], (unsigned long long)ql);
                        const uint64_t h = qh + (oq + ql < oq ? 1u : 0u);
                        if (h) atomicAdd((unsigned long long*)&s_qhi[cell], (unsigned long long)h);
                    }
                }
            }
            __syncthreads();
            for (int c = threadIdx.x; c < cells; c += kEB) {
                const uint64_t cn = s_cnt[c], sl = s_slo[c], sh = s_shi[c], ql = s_qlo[c], qh = s_qhi[c];
                if (first) {
                    slot[c] = cn;
                    slot[kEfgCells + c] = sl;
                    slot[2 * kEfgCells + c] = sh;
                    slot[3 * kEfgCells + c] = ql;
                    slot[4 * kEfgCells + c] = qh;
                } else {
                    slot[c] += cn;
                    const uint64_t a = slot[kEfgCells + c];
                    slot[kEfgCells + c] = a + sl;
                    slot[2 * kEfgCells + c] += sh + (a + sl < a ? 1u : 0u);
                    const uint64_t q = slot[3 * kEfgCells + c];
                    slot[3 * kEfgCells + c] = q + ql;
                    slot[4 * kEfgCells + c] += qh + (q + ql < q ? 1u : 0u);
                }
            }
            first = false;
            __syncthreads();
        }
        if (first)   // an entry with no pairs still owns a slot
            for (int c = threadIdx.x; c < cells; c += kEB)
                for (int f = 0; f < 5; ++f) slot[f * kEfgCells + c] = 0;
    }
}

// 256-bit unsigned arithmetic for the variance numerator n*Q - S*S.
struct U256 {
    uint64_t w[4];
};

__device__ __forceinline__ void add_to(U256& r, int k, uint64_t v) {
    for (; k < 4 && v; ++k) {
        const uint64_t s = r.w[k] + v;
        v = s < v ? 1u : 0u;
        r.w[k] = s;
    }
}

// (a1:a0) * (b1:b0), both 128-bit.
__device__ U256 mul128(uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1) {
    U256 r{{0, 0, 0, 0}};
    const uint64_t a[2] = {a0, a1}, b[2] = {b0, b1};
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) {
            add_to(r, x + y, a[x] * b[y]);
            add_to(r, x + y + 1, __umul64hi(a[x], b[y]));
        }
    return r;
}

__device__ U256 sub256(const U256& a, const U256& b) {
    U256 r;
    uint64_t borrow = 0;
    for (int k = 0; k < 4; ++k) {
        const uint64_t t = a.w[k] - b.w[k];
        const uint64_t nb = (a.w[k] < b.w[k]) || (t < borrow) ? 1u : 0u;
        r.w[k] = t - borrow;
        borrow = nb;
    }
    return r;
}

// Most significant limb first: x = x * 2^64 + limb, one rounding per step.
__device__ __forceinline__ double limbs_to_double(const uint64_t* w, int n) {
    const double two64 = 18446744073709551616.0;
    double x = (double)w[n - 1];
    for (int k = n - 2; k >= 0; --k) x = __dadd_rn(__dmul_rn(x, two64), (double)w[k]);
    return x;
}

// 64 cells per block, 16 lanes per cell splitting its bucket's partial slots;
// the 16 partial sums combine exactly in LDS.
constexpr int kRC = 64, kRL = 16;
__global__ __launch_bounds__(kRC * kRL) void k_efg_reduce(EfgWs w, int32_t A, int32_t R, EfgOutDev o,
                                                          const int32_t* status_in) {
    __shared__ uint64_t red[5][kRL][kRC];
    const int64_t cells = (int64_t)A * A;
    const int ci = threadIdx.x % kRC, li = threadIdx.x / kRC;
    for (int64_t c0 = (int64_t)blockIdx.x * kRC; c0 < cells; c0 += (int64_t)gridDim.x * kRC) {
        const int64_t cell = c0 + ci;
        uint64_t cn = 0, sl = 0, sh = 0, ql = 0, qh = 0;
        if (cell < cells) {
            const int32_t row = (int32_t)(cell / A), col = (int32_t)(cell % A);
            const int32_t b = row / R;
            const int64_t local = (int64_t)(row - b * R) * A + col;
            const int64_t e0 = w.bfirst[b], ne = w.bnum[b];
            for (int64_t e = e0 + li; e < e0 + ne; e += kRL) {
                const uint64_t* slot = w.part + e * (int64_t)kSlotWords;
                cn += slot[local];
                const uint64_t a = slot[kEfgCells + local];
                sh += slot[2 * kEfgCells + local] + (sl + a < sl ? 1u : 0u);
                sl += a;
                const uint64_t q = slot[3 * kEfgCells + local];
                qh += slot[4 * kEfgCells + local] + (ql + q < ql ? 1u : 0u);
                ql += q;
            }
        }
        red[0][li][ci] = cn;
        red[1][li][ci] = sl;
        red[2][li][ci] = sh;
        red[3][li][ci] = ql;
        red[4][li][ci] = qh;
        __syncthreads();
        if (li == 0 && cell < cells) {
            for (int l = 1; l < kRL; ++l) {
                cn += red[0][l][ci];
                const uint64_t a = red[1][l][ci];
                sh += red[2][l][ci] + (sl + a < sl ? 1u : 0u);
                sl += a;
                const uint64_t q = red[3][l][ci];
                qh += red[4][l][ci] + (ql + q < ql ? 1u : 0u);
                ql += q;
            }
            o.count[cell] = (int64_t)cn;
            o.sum_lo[cell] = sl;
            o.sum_hi[cell] = sh;
            o.sq_lo[cell] = ql;
            o.sq_hi[cell] = qh;
            const double nan = __longlong_as_double(0x7ff8000000000000ll);
            const uint64_t s2[2] = {sl, sh};
            if (o.mean) o.mean[cell] = cn ? __ddiv_rn(limbs_to_double(s2, 2), (double)cn) : nan;
            if (o.std) {
                double sd;
                if (cn == 0) {
                    sd = nan;
                } else if (cn == 1) {
                    sd = 0.0;
                } else {
                    const U256 nq = mul128(cn, 0, ql, qh);
                    const U256 ss = mul128(sl, sh, sl, sh);
                    const U256 dd = sub256(nq, ss);
                    const double D = limbs_to_double(dd.w, 4);
                    sd = __dsqrt_rn(__ddiv_rn(__ddiv_rn(D, (double)cn), (double)(cn - 1)));
                }
                o.std[cell] = sd;
            }
        }
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *o.n_pairs = w.scal[2];
        *o.status = (status_in && *status_in) ? *status_in : 0;
    }
}

}  // namespace

hipError_t launch_efg(const pm4g_prepared* p, EfgWs w, const EfgOutDev& o, int64_t pass_pairs, hipStream_t s) {
    ProfScope ps(P_EFG, s);
    const int64_t n = p->n_events;
    const int32_t A = p->n_activities;
    const int32_t R = efg_rows(A);
    const int64_t nbk = efg_buckets(A);
    const int64_t nch = (n + kEfgChunk - 1) / kEfgChunk;
    k_efg_setup<<<1, 1, 0, s>>>(w, n, nbk * nch);
    k_efg_tail<<<2048, 256, 0, s>>>(p->case_off, p->n_cases, w.tail);
    const unsigned gch = (unsigned)(nch < 2048 ? (nch < 1 ? 1 : nch) : 2048);
    int kbits = 0;
    while ((int64_t(1) << kbits) < nbk) ++kbits;
    if (nbk > 1) {
        k_efg_bcount<<<gch, 256, 0, s>>>(p->act_s, w.tail, n, R, nbk, kbits, nch, w.bcnt);
        // bucket-major offsets; the list length (events with a later event) -> scal[1]
        dev::excl_scan<int64_t>(w.bcnt, &w.scal[4], w.boff, w.part64, &w.scal[1], s);
        k_efg_bscatter<<<gch, 256, 0, s>>>(p->act_s, w.tail, n, R, nbk, kbits, nch, w);
        dev::excl_scan<int64_t>(w.tl, &w.scal[1], w.poff, w.part64, &w.scal[2], s);
    } else {
        dev::excl_scan<int64_t>(w.tail, &w.scal[1], w.poff, w.part64, &w.scal[2], s);
    }
    k_efg_plan<<<1, 1024, 0, s>>>(w, nbk, nch, kEfgPlanBlocks);
    const int64_t seg = (pass_pairs > 0 && pass_pairs < kEfgSeg) ? pass_pairs : kEfgSeg;
    k_efg_agg<<<kEfgAggGrid, kEB, 0, s>>>(p->act_s, p->ts_s, w, A, R, nbk > 1 ? 1 : 0, seg);
    const int64_t cells = (int64_t)A * A;
    const int64_t gr = (cells + kRC - 1) / kRC;
    k_efg_reduce<<<(unsigned)(gr < 2048 ? gr : 2048), kRC * kRL, 0, s>>>(w, A, R, o, p->status);
    return hipGetLastError();
}

}  // namespace pm4g
