// Per-case ordering (Sec. 3, first formatting step: within a case, events are
// ordered by timestamp, then by absolute row index).
//
// Input: the radix output, grouped by case, each case's events in row order
// (the passes are stable).  Block w owns the cases that START inside window
// [w*1024, (w+1)*1024); their events (at most 1023 + 2049 = 3072 when no case
// is longer than 2049 events) are staged in LDS.  The staged region is cut
// into 64-event chunks; each wave sorts its chunks in registers with a
// bitonic network on (case, timestamp, staging position) -- the staging
// position is the row order inside a case.  A case that fits in one chunk is
// then ordered; a case spanning k chunks has k sorted portions, and an event's
// rank in its case is its rank in its own portion plus, for each other
// portion, the number of smaller events found by binary search:
// O(L/64 * log 64) comparisons per event instead of O(L).
// A region longer than the LDS window sets RangeInfo::long_case and the
// host switches to the full-key fallback.
//
// Also writes the prepared columns: case id (unbiased), activity, timestamp.
// Bytes per event: 16 read + 16 write.
#include "common.hpp"
#include "internal.hpp"
#include "prof.hpp"

namespace pm4g {

constexpr int kSB = 512;
constexpr int kSI = kSegCap / kSB;   // 6 items per thread

__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t* red) {
    v = wave_min(v);
    const int w = threadIdx.x / kWave;
    if (lane() == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t m = red[0];
        for (int i = 1; i < kSB / kWave; ++i) m = red[i] < m ? red[i] : m;
        red[kSB / kWave] = m;
    }
    __syncthreads();
    const int64_t r = red[kSB / kWave];
    __syncthreads();
    return r;
}

__device__ __forceinline__ int32_t wave_incl_max_i32(int32_t v) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int32_t u = __shfl_up(v, o);
        if (lane() >= o) v = u > v ? u : v;
    }
    return v;
}

// act_shift > 0: packed keys (case bits below act_shift, activity above).
__global__ __launch_bounds__(kSB) void k_segsort(SortBufs in, int64_t n, RangeInfo* info,
                                                 int32_t* __restrict__ case_s,
                                                 int32_t* __restrict__ act_s,
                                                 int64_t* __restrict__ ts_s, int act_shift) {
    __shared__ uint32_t lkey[kSegCap];
    __shared__ int64_t lts[kSegCap];
    __shared__ uint16_t lact[kSegCap];
    __shared__ uint16_t lidx[kSegCap];   // staging position of the event now at i
    __shared__ uint16_t lcs[kSegCap];
    __shared__ uint16_t lce[kSegCap + 1];
    __shared__ int64_t red[kSB / kWave + 1];
    __shared__ int32_t wred[kSB / kWave];

    const uint32_t* __restrict__ key = in.key;
    const uint32_t kmask = act_shift > 0 ? ((1u << act_shift) - 1u) : 0xFFFFFFFFu;
    const int64_t w0 = (int64_t)blockIdx.x * kSegWindow;
    const int64_t w1 = (w0 + kSegWindow) < n ? (w0 + kSegWindow) : n;

    // 1. first case start inside the window
    int64_t cand = INT64_MAX;
    for (int64_t p = w0 + threadIdx.x; p < w1; p += kSB) {
        if (p == 0 || ((key[p] ^ key[p - 1]) & kmask) != 0) {
            cand = p;
            break;
        }
    }
    const int64_t s = block_min_i64(cand, red);
    if (s == INT64_MAX) return;   // a long case covers the whole window (block-uniform)

    // 2. first case start at or after the window end (n counts as a start)
    int64_t e = INT64_MAX;
    for (int64_t base = w1; base <= n && base - s <= kSegCap; base += kSB) {
        const int64_t p = base + threadIdx.x;
        int64_t c = INT64_MAX;
        if (p == n) c = n;
        else if (p < n && ((key[p] ^ key[p - 1]) & kmask) != 0) c = p;
        const int64_t m = block_min_i64(c, red);
        if (m != INT64_MAX) {
            e = m;
            break;
        }
    }
    if (e == INT64_MAX || e - s > kSegCap) {
        if (threadIdx.x == 0) atomicOr(&info->long_case, 1);
        return;
    }
    const int R = (int)(e - s);

    // 3. stage the region
    for (int i = threadIdx.x; i < R; i += kSB) {
        const uint32_t kr = key[s + i];
        lkey[i] = kr & kmask;
        lts[i] = in.ts[s + i];
        lact[i] = (uint16_t)(act_shift > 0 ? (kr >> act_shift) : in.act[s + i]);
    }
    __syncthreads();

    // 4. case start of every event: inclusive max-scan of start positions
    //    (blocked layout: thread t owns items 8t .. 8t+7)
    {
        int32_t loc[kSI];
        int32_t m = 0;
#pragma unroll
        for (int q = 0; q < kSI; ++q) {
            const int i = threadIdx.x * kSI + q;
            if (i < R && (i == 0 || lkey[i] != lkey[i - 1])) m = i;
            loc[q] = m;
        }
        const int w = threadIdx.x / kWave;
        int32_t inc = wave_incl_max_i32(m);
        if (lane() == kWave - 1) wred[w] = inc;
        __syncthreads();
        int32_t before = 0;
        for (int i = 0; i < w; ++i) before = wred[i] > before ? wred[i] : before;
        int32_t excl = __shfl_up(inc, 1);
        if (lane() == 0) excl = 0;
        excl = excl > before ? excl : before;
#pragma unroll
        for (int q = 0; q < kSI; ++q) {
            const int i = threadIdx.x * kSI + q;
            if (i < R) lcs[i] = (uint16_t)(loc[q] > excl ? loc[q] : excl);
        }
    }
    __syncthreads();
    // case end, stored at the case start: the last event of each case writes it
    for (int i = threadIdx.x; i < R; i += kSB) {
        if (i == R - 1 || lkey[i + 1] != lkey[i]) lce[lcs[i]] = (uint16_t)(i + 1);
    }
    __syncthreads();

    // 5. sort every 64-event chunk in registers by (case, ts, staging position)
    {
        const int w = threadIdx.x / kWave;
        const int l = lane();
        for (int ch = w; ch * kWave < R; ch += kSB / kWave) {
            const int i = ch * kWave + l;
            uint32_t k = 0xFFFFFFFFu, id = 0x10000u + (uint32_t)l;   // padding sorts last
            int64_t t = INT64_MAX;
            if (i < R) {
                k = lkey[i];
                t = lts[i];
                id = (uint32_t)i;
            }
#pragma unroll
            for (int m = 2; m <= kWave; m <<= 1) {
#pragma unroll
                for (int j = m >> 1; j > 0; j >>= 1) {
                    const uint32_t pk = __shfl_xor(k, j);
                    const int64_t pt = __shfl_xor(t, j);
                    const uint32_t pid = __shfl_xor(id, j);
                    // branch-free compare-exchange: keep the partner iff it belongs here
                    const bool pless = (pk < k) | ((pk == k) & ((pt < t) | ((pt == t) & (pid < id))));
                    const bool flip = ((l & m) == 0) != ((l & j) == 0);
                    const bool take = pless != flip;
                    k = take ? pk : k;
                    t = take ? pt : t;
                    id = take ? pid : id;
                }
            }
            if (i < R) {
                lkey[i] = k;   // unchanged: the chunk was already grouped by case
                lts[i] = t;
                lidx[i] = (uint16_t)id;
            }
        }
    }
    __syncthreads();

    // 6. rank inside the case: own portion + binary searches in the other portions
    int32_t pos[kSI];
    uint32_t kv[kSI];
    int64_t tv[kSI];
    uint16_t av[kSI];
#pragma unroll
    for (int q = 0; q < kSI; ++q) {
        const int i = threadIdx.x + q * kSB;
        pos[q] = -1;
        if (i < R) {
            const int cs = lcs[i];
            const int ce = lce[cs];
            const int64_t t = lts[i];
            const uint32_t id = lidx[i];
            const int ch = i >> 6;
            int r = i - (cs > (ch << 6) ? cs : (ch << 6));
            const int c_last = (ce - 1) >> 6;
            for (int c2 = cs >> 6; c2 <= c_last; ++c2) {
                if (c2 == ch) continue;
                const int p0 = cs > (c2 << 6) ? cs : (c2 << 6);
                int lo = p0, hi = ce < (c2 << 6) + kWave ? ce : (c2 << 6) + kWave;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const int64_t tm = lts[mid];
                    if (tm < t || (tm == t && (uint32_t)lidx[mid] < id)) lo = mid + 1;
                    else hi = mid;
                }
                r += lo - p0;
            }
            pos[q] = cs + r;
            kv[q] = lkey[i];
            tv[q] = t;
            av[q] = lact[id];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSI; ++q) {
        if (pos[q] >= 0) {
            lkey[pos[q]] = kv[q];
            lts[pos[q]] = tv[q];
            lact[pos[q]] = av[q];
        }
    }
    __syncthreads();

    // 7. write the prepared columns
    const uint32_t bias = (uint32_t)info->case_min;
    for (int i = threadIdx.x; i < R; i += kSB) {
        case_s[s + i] = (int32_t)(lkey[i] + bias);
        act_s[s + i] = (int32_t)lact[i];
        ts_s[s + i] = lts[i];
    }
}

__global__ void k_unbias_copy(SortBufs in, int64_t n, const RangeInfo* info, int32_t* case_s,
                              int32_t* act_s, int64_t* ts_s, int act_shift) {
    const uint32_t bias = (uint32_t)info->case_min;
    const uint32_t kmask = act_shift > 0 ? ((1u << act_shift) - 1u) : 0xFFFFFFFFu;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t k = in.key[i];
        case_s[i] = (int32_t)((k & kmask) + bias);
        act_s[i] = (int32_t)(act_shift > 0 ? (k >> act_shift) : in.act[i]);
        ts_s[i] = in.ts[i];
    }
}

__global__ void k_copy_log(const int32_t* c, const int32_t* a, const int64_t* t, int64_t n,
                           int32_t* case_s, int32_t* act_s, int64_t* ts_s) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        case_s[i] = c[i];
        act_s[i] = a[i];
        ts_s[i] = t[i];
    }
}

static unsigned copy_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

hipError_t launch_segsort(SortBufs in, int64_t n, RangeInfo* info, int32_t* case_s, int32_t* act_s,
                          int64_t* ts_s, int act_shift, hipStream_t s) {
    ProfScope p(P_SEGSORT, s);
    if (n > 0) k_segsort<<<(unsigned)segsort_blocks(n), kSB, 0, s>>>(in, n, info, case_s, act_s, ts_s, act_shift);
    return hipGetLastError();
}

hipError_t launch_unbias_copy(SortBufs in, int64_t n, const RangeInfo* info, int32_t* case_s,
                              int32_t* act_s, int64_t* ts_s, int act_shift, hipStream_t s) {
    if (n > 0) k_unbias_copy<<<copy_grid(n), 256, 0, s>>>(in, n, info, case_s, act_s, ts_s, act_shift);
    return hipGetLastError();
}

hipError_t launch_copy_log(const int32_t* c, const int32_t* a, const int64_t* t, int64_t n,
                           int32_t* case_s, int32_t* act_s, int64_t* ts_s, hipStream_t s) {
    if (n > 0) k_copy_log<<<copy_grid(n), 256, 0, s>>>(c, a, t, n, case_s, act_s, ts_s);
    return hipGetLastError();
}

}  // namespace pm4g
