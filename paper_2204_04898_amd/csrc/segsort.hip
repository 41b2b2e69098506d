// Per-case ordering (Sec. 3, first formatting step: within a case, events are
// ordered by timestamp, then by absolute row index).
//
// Input: the radix output, grouped by case, each case's events in row order
// (the passes are stable).  Block w owns the cases that START inside window
// [w*W, (w+1)*W); their events (at most W - 1 + 2049 = kSegCap when no case
// is longer than 2049 events) are staged in LDS.  The staged region is cut
// into 64-event chunks; each wave sorts its chunks in registers with a
// bitonic network on (case, timestamp, staging position) -- the staging
// position is the row order inside a case.  A case that fits in one chunk is
// then ordered; a case spanning k chunks has k sorted portions, and an event's
// rank in its case is its rank in its own portion plus, for each other
// portion, the number of smaller events found by binary search:
// O(L/64 * log 64) comparisons per event instead of O(L).
//
// Sort key.  When every staged event lies within 2^51 time units of its
// case's first staged event (block-uniform check; ns timestamps: 26 days per
// case), the three fields fold into one u64 per event:
//   [63:58] case slot in the chunk (count of case starts before it)
//   [57:6]  timestamp - case base + 2^51
//   [5:0]   lane (= staging order inside the chunk)
// and the network moves 2 dwords per stage with one 64-bit compare; the lane
// bits name the event, the timestamp is rebuilt from the base.  Otherwise the
// network compares (case start, timestamp, staging position) field by field.
// Lane exchanges: quad permutes and a row rotate (DPP) for distances 1, 2, 8,
// swizzles for 4 and 16, a permute for 32.
//
// A region longer than the LDS window sets RangeInfo::long_case and the
// host switches to the full-key fallback.
//
// Also writes the prepared columns: case id (unbiased), activity, timestamp,
// and, when the caller asks for it (ROW), the original row of each position
// (read from the row the radix passes carried, at its staging position).
// Bytes per event: 16 read + 16 write (12 + 16 packed; + 4 + 4 with rows).
#include "common.hpp"
#include "internal.hpp"
#include "prof.hpp"

namespace pm4g {

constexpr int kSB = 512;
constexpr int kSW = kSB / kWave;     // waves per block
constexpr int kSI = kSegCap / kSB;   // items per thread = chunks per wave
constexpr int kPre = 3;              // window + lookahead read in the first load round
static_assert(kSI < 8, "a thread's case starts are counted in three bits");
static_assert(kSegCap % kSB == 0, "staging capacity must be a multiple of the block");
static_assert(kSegCap <= 4096, "cross keys hold the staging position in 12 bits");
static_assert(kPre * kSB >= kSegWindow, "the first load round covers the window");

__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t* red) {
    v = wave_min(v);
    if (lane() == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    int64_t m = red[0];
#pragma unroll
    for (int i = 1; i < kSW; ++i) m = red[i] < m ? red[i] : m;
    __syncthreads();
    return m;
}

// Value of lane (lane ^ J); every lane of the wave must be active.
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
    if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad [1,0,3,2]
    else if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad [2,3,0,1]
    else if constexpr (J == 8) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false); // row rotate 8
    else if constexpr (J == 4 || J == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (J << 10) | 0x1F);
    else return (uint32_t)__shfl_xor((int)v, J);
}

template <int J>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v) {
    const uint32_t lo = xor_lane<J>((uint32_t)v);
    const uint32_t hi = xor_lane<J>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Lanes that take the larger of the pair at stage (M, J) of the ascending
// network: lane l's block of M runs downward, or l is the upper lane of its
// pair, but not both.  A compile-time lane mask: with inverse_ballot it stays
// in scalar registers (no per-wave computation of the 21 masks).
constexpr uint64_t flip_mask(int M, int J) {
    uint64_t m = 0;
    for (int l = 0; l < 64; ++l)
        if (((l & M) == 0) != ((l & J) == 0)) m |= uint64_t(1) << l;
    return m;
}

// One bitonic merge level (block size M) on one u64 key per lane, ascending.
template <int M, int J>
__device__ __forceinline__ void merge_u64(uint64_t& k) {
    if constexpr (J > 0) {
        const uint64_t p = xor_lane64<J>(k);
        const bool flip = __builtin_amdgcn_inverse_ballot_w64(flip_mask(M, J));
        k = ((p < k) != flip) ? p : k;
        merge_u64<M, J / 2>(k);
    }
}

__device__ __forceinline__ void bitonic64_u64(uint64_t& k) {
    merge_u64<2, 1>(k);
    merge_u64<4, 2>(k);
    merge_u64<8, 4>(k);
    merge_u64<16, 8>(k);
    merge_u64<32, 16>(k);
    merge_u64<64, 32>(k);
}

// Field-by-field network: (case start c, timestamp t, staging position id).
template <int M, int J>
__device__ __forceinline__ void merge_3(uint32_t& c, int64_t& t, uint32_t& id) {
    if constexpr (J > 0) {
        const uint32_t pc = xor_lane<J>(c);
        const int64_t pt = (int64_t)xor_lane64<J>((uint64_t)t);
        const uint32_t pid = xor_lane<J>(id);
        const bool pless = (pc < c) | ((pc == c) & ((pt < t) | ((pt == t) & (pid < id))));
        const bool flip = __builtin_amdgcn_inverse_ballot_w64(flip_mask(M, J));
        const bool take = pless != flip;
        c = take ? pc : c;
        t = take ? pt : t;
        id = take ? pid : id;
        merge_3<M, J / 2>(c, t, id);
    }
}

__device__ __forceinline__ void bitonic64_3(uint32_t& c, int64_t& t, uint32_t& id) {
    merge_3<2, 1>(c, t, id);
    merge_3<4, 2>(c, t, id);
    merge_3<8, 4>(c, t, id);
    merge_3<16, 8>(c, t, id);
    merge_3<32, 16>(c, t, id);
    merge_3<64, 32>(c, t, id);
}

constexpr uint64_t kOffBias = 1ull << 51;
constexpr uint64_t kOffMask = (1ull << 52) - 1;

// act_shift > 0: packed keys (case bits below act_shift, activity above).
template <bool ROW>
__global__ __launch_bounds__(kSB) void k_segsort(SortBufs in, int64_t n, RangeInfo* info,
                                                 int32_t* __restrict__ case_s,
                                                 int32_t* __restrict__ act_s,
                                                 int64_t* __restrict__ ts_s, int act_shift,
                                                 uint32_t* __restrict__ wincnt,
                                                 int32_t* __restrict__ row_s) {
    __shared__ int64_t lts[kSegCap];     // timestamps; on the fast path the sorted cross keys
    __shared__ uint16_t lact[kSegCap];
    __shared__ uint16_t lidx[kSegCap];   // field-by-field path: staging position of the event now at i
    __shared__ uint16_t lcs[kSegCap];    // case start of position i
    __shared__ uint16_t lce[kSegCap];    // case end, stored at the case start
    __shared__ int64_t red[2 * kSW];
    __shared__ int32_t wred[kSW];
    __shared__ int32_t wst[kSW];
    __shared__ uint32_t wfirst[2][kSW];

    const uint32_t* __restrict__ key = in.key;
    const uint32_t kmask = act_shift > 0 ? ((1u << act_shift) - 1u) : 0xFFFFFFFFu;
    // one window per block, XCD-contiguous: a window's lookahead is the next
    // window's start, read by the same XCD at about the same time (its L2)
    const int64_t win = xcd_split(gridDim.x).first;
    const int64_t w0 = win * kSegWindow;
    const int64_t w1 = (w0 + kSegWindow) < n ? (w0 + kSegWindow) : n;

    // 1. one load round: the window and a lookahead are read into registers; the
    //    first case start inside the window (s) and the first at or after its end
    //    (e; n counts) come from them.  Item q of thread t is position
    //    w0 + q*kSB + t, so within a wave positions grow with q, then with the
    //    lane: the first q whose ballot is not empty holds the wave's first
    //    start (wave-uniform, scalar work); the block takes the smallest over
    //    its waves.  Offsets from w0 fit in 32 bits.
    // The loads take clamped (in-bounds) positions with no branch around them
    // and all are issued before any is used; values past n are never used.
    uint32_t pk[kPre], pa[kPre], pkm1[kPre];
    int64_t pt[kPre];
    bool pst[kPre];
    const int wv0 = threadIdx.x / kWave;
    uint32_t s_off = UINT32_MAX, e_off = UINT32_MAX;
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
        const int64_t P = w0 + threadIdx.x + q * kSB;
        const int64_t Pc = P < n ? P : n - 1;
        pk[q] = key[Pc];
        pkm1[q] = key[Pc > 0 ? Pc - 1 : 0];
        pt[q] = in.ts[Pc];
        pa[q] = 0;
        if (act_shift <= 0) pa[q] = in.act[Pc];   // block-uniform: no activity column when packed
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
        const int64_t P = w0 + threadIdx.x + q * kSB;
        if (act_shift > 0) pa[q] = pk[q] >> act_shift;
        pst[q] = P < n && (P == 0 || ((pk[q] ^ pkm1[q]) & kmask) != 0);
        const uint64_t bs = __ballot(pst[q] && P < w1);
        const uint64_t be = __ballot((pst[q] && P >= w1) || P == n);
        const uint32_t base = (uint32_t)(q * kSB + wv0 * kWave);
        if (s_off == UINT32_MAX && bs) s_off = base + (uint32_t)__ffsll((unsigned long long)bs) - 1u;
        if (e_off == UINT32_MAX && be) e_off = base + (uint32_t)__ffsll((unsigned long long)be) - 1u;
    }
    if (lane() == 0) {
        wfirst[0][wv0] = s_off;
        wfirst[1][wv0] = e_off;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSW; ++k) {
        s_off = wfirst[0][k] < s_off ? wfirst[0][k] : s_off;
        e_off = wfirst[1][k] < e_off ? wfirst[1][k] : e_off;
    }
    int64_t s = s_off == UINT32_MAX ? INT64_MAX : w0 + (int64_t)s_off;
    int64_t e = e_off == UINT32_MAX ? INT64_MAX : w0 + (int64_t)e_off;
    if (s == INT64_MAX) {   // a long case covers the whole window (block-uniform): no case starts here
        if (threadIdx.x == 0) wincnt[win] = 0;
        return;
    }
    for (int64_t base = w0 + kPre * kSB; e == INT64_MAX && base <= n && base - s <= kSegCap; base += kSB) {
        const int64_t p = base + threadIdx.x;
        int64_t c = INT64_MAX;
        if (p == n) c = n;
        else if (p < n && ((key[p] ^ key[p - 1]) & kmask) != 0) c = p;
        e = block_min_i64(c, red);
    }
    if (e == INT64_MAX || e - s > kSegCap) {
        if (threadIdx.x == 0) atomicOr(&info->long_case, 1);
        return;
    }
    const int R = (int)(e - s);

    // 2. stage the region [s, e): prefetched events, then any beyond the lookahead
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
        const int64_t P = w0 + threadIdx.x + q * kSB;
        if (P >= s && P < e) {
            const int i = (int)(P - s);
            lts[i] = pt[q];
            lact[i] = (uint16_t)pa[q];
            lcs[i] = (uint16_t)(pst[q] ? i : 0);
        }
    }
    for (int64_t P = w0 + kPre * kSB + threadIdx.x; P < e; P += kSB) {
        const int i = (int)(P - s);
        const uint32_t kr = key[P];
        lts[i] = in.ts[P];
        lact[i] = (uint16_t)(act_shift > 0 ? (kr >> act_shift) : in.act[P]);
        lcs[i] = (uint16_t)((((kr ^ key[P - 1]) & kmask) != 0) ? i : 0);
    }
    // case ids of the output positions (striped), in flight during the sort:
    // position i keeps the case of staging position i
    uint32_t ck[kSI];
#pragma unroll
    for (int q = 0; q < kSI; ++q) {
        const int i = threadIdx.x + q * kSB;
        ck[q] = key[s + (i < R ? i : R - 1)];   // in bounds, no branch; masked at the write
    }
    __syncthreads();

    // 3. case start of every event: inclusive max-scan of the start positions
    //    (blocked layout: thread t owns items kSI*t .. kSI*t + kSI - 1)
    {
        int32_t loc[kSI];
        int32_t m = 0, nst = 0;
#pragma unroll
        for (int q = 0; q < kSI; ++q) {
            const int i = threadIdx.x * kSI + q;
            if (i < R) {
                m = (int32_t)lcs[i] > m ? (int32_t)lcs[i] : m;
                nst += (int32_t)lcs[i] == i;   // a case starts at i
            }
            loc[q] = m;
        }
        const int w = threadIdx.x / kWave;
        // inclusive max over the lanes: where m is not zero it is the last start
        // among the lane's items, so it grows with the lane; the max is the m of
        // the highest lane at or below this one with m > 0
        const uint64_t nz = __ballot(m > 0) & (lanes_below() | (uint64_t(1) << lane()));
        const int32_t inc = nz ? __shfl(m, 63 - __clzll((long long)nz)) : 0;
        // the wave's starts: nst < 8, so three ballots of its bits
        const int32_t wn = __popcll(__ballot(nst & 1)) + 2 * __popcll(__ballot(nst & 2)) +
                           4 * __popcll(__ballot(nst & 4));
        if (lane() == kWave - 1) wred[w] = inc;
        if (lane() == 0) wst[w] = wn;
        __syncthreads();
        if (threadIdx.x == 0) {   // the region's cases are the cases starting in the window
            int32_t t = 0;
            for (int k = 0; k < kSW; ++k) t += wst[k];
            wincnt[win] = (uint32_t)t;
        }
        int32_t before = 0;
        for (int i = 0; i < w; ++i) before = wred[i] > before ? wred[i] : before;
        // lane l - 1's inclusive max (DPP wave shift right by one; lane 0 reads 0)
        int32_t excl = __builtin_amdgcn_update_dpp(0, inc, 0x138, 0xF, 0xF, false);
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
        if (i == R - 1 || lcs[i + 1] == i + 1) lce[lcs[i]] = (uint16_t)(i + 1);
    }

    // 4. sort every 64-event chunk in registers (wave w: chunks w, w + kSW, ...;
    //    chunk w + q*kSW, lane l is position threadIdx.x + q*kSB, as in step 5)
    const int w = threadIdx.x / kWave;
    const int l = lane();
    uint64_t sk[kSI];
    int64_t sb[kSI];
    bool fits = true;
#pragma unroll
    for (int q = 0; q < kSI; ++q) {
        const int ch = w + q * kSW;
        const int i = ch * kWave + l;
        sk[q] = ~0ull;   // padding sorts last
        sb[q] = 0;
        if (ch * kWave < R) {   // wave-uniform
            const bool valid = i < R;
            const int cs = valid ? (int)lcs[i] : 0;
            const bool first = l == 0 || (valid && cs == i);
            const uint64_t starts = __ballot(first);
            const uint32_t slot = (uint32_t)__popcll(starts & lanes_below()) + (first ? 1u : 0u) - 1u;
            if (valid) {
                const int64_t base = lts[cs];
                const int64_t t = lts[i];
                const bool ok = t >= base ? ((uint64_t)t - (uint64_t)base < kOffBias)
                                          : ((uint64_t)base - (uint64_t)t <= kOffBias);
                fits &= ok;
                sk[q] = ((uint64_t)slot << 58) | ((((uint64_t)t - (uint64_t)base + kOffBias) & kOffMask) << 6) |
                        (uint64_t)l;
                sb[q] = base;
            }
        }
    }
    const bool fast = __syncthreads_and(fits);   // also: every read of step 4 precedes the writes below
    int32_t pos[kSI];
    int64_t tv[kSI];
    uint16_t av[kSI];
    uint16_t sv[kSI];   // staging position of the event (ROW)
    if (fast) {
        // sorted position i holds cross key (offset << 12 | staging position):
        // unique, and ordered as (timestamp, row) across the chunks of a case
#pragma unroll
        for (int q = 0; q < kSI; ++q) {
            const int ch = w + q * kSW;
            if (ch * kWave >= R) continue;   // wave-uniform
            uint64_t k = sk[q];
            bitonic64_u64(k);
            const int i = ch * kWave + l;
            if (i < R) lts[i] = (int64_t)((((k >> 6) & kOffMask) << 12) | (uint64_t)(ch * kWave + (int)(k & 63u)));
        }
        __syncthreads();
        // 5. rank inside the case: own portion + binary searches in the other portions
#pragma unroll
        for (int q = 0; q < kSI; ++q) {
            const int i = threadIdx.x + q * kSB;
            pos[q] = -1;
            if (i < R) {
                const int cs = lcs[i];
                const int ce = lce[cs];
                const uint64_t x = (uint64_t)lts[i];
                const int ch = i >> 6;
                int r = i - (cs > (ch << 6) ? cs : (ch << 6));
                const int c_last = (ce - 1) >> 6;
                for (int c2 = cs >> 6; c2 <= c_last; ++c2) {
                    if (c2 == ch) continue;
                    const int p0 = cs > (c2 << 6) ? cs : (c2 << 6);
                    int lo = p0, hi = ce < (c2 << 6) + kWave ? ce : (c2 << 6) + kWave;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if ((uint64_t)lts[mid] < x) lo = mid + 1;
                        else hi = mid;
                    }
                    r += lo - p0;
                }
                pos[q] = cs + r;
                tv[q] = (int64_t)((uint64_t)sb[q] + (x >> 12) - kOffBias);
                av[q] = lact[x & 0xFFFu];
                sv[q] = (uint16_t)(x & 0xFFFu);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < kSI; ++q) {
            const int ch = w + q * kSW;
            if (ch * kWave >= R) continue;   // wave-uniform
            const int i = ch * kWave + l;
            uint32_t c = 0xFFFFFFFFu, id = 0x10000u + (uint32_t)l;   // padding sorts last
            int64_t t = INT64_MAX;
            if (i < R) {
                c = lcs[i];
                t = lts[i];
                id = (uint32_t)i;
            }
            bitonic64_3(c, t, id);
            if (i < R) {
                lts[i] = t;
                lidx[i] = (uint16_t)id;
            }
        }
        __syncthreads();
        // 5. rank inside the case: own portion + binary searches in the other portions
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
                tv[q] = t;
                av[q] = lact[id];
                sv[q] = (uint16_t)id;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSI; ++q) {
        if (pos[q] >= 0) {
            lts[pos[q]] = tv[q];
            lact[pos[q]] = av[q];
            if (ROW) lidx[pos[q]] = sv[q];
        }
    }
    __syncthreads();

    // 6. write the prepared columns
    const uint32_t bias = (uint32_t)info->case_min;
#pragma unroll
    for (int q = 0; q < kSI; ++q) {
        const int i = threadIdx.x + q * kSB;
        if (i < R) {
            case_s[s + i] = (int32_t)((ck[q] & kmask) + bias);
            act_s[s + i] = (int32_t)lact[i];
            ts_s[s + i] = lts[i];
            if (ROW) row_s[s + i] = (int32_t)in.row[s + lidx[i]];
        }
    }
}

__global__ void k_unbias_copy(SortBufs in, int64_t n, const RangeInfo* info, int32_t* case_s,
                              int32_t* act_s, int64_t* ts_s, int act_shift, int32_t* row_s) {
    const uint32_t bias = (uint32_t)info->case_min;
    const uint32_t kmask = act_shift > 0 ? ((1u << act_shift) - 1u) : 0xFFFFFFFFu;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t k = in.key[i];
        case_s[i] = (int32_t)((k & kmask) + bias);
        act_s[i] = (int32_t)(act_shift > 0 ? (k >> act_shift) : in.act[i]);
        ts_s[i] = in.ts[i];
        if (row_s) row_s[i] = (int32_t)in.row[i];
    }
}

__global__ void k_copy_log(const int32_t* c, const int32_t* a, const int64_t* t, int64_t n,
                           int32_t* case_s, int32_t* act_s, int64_t* ts_s, int32_t* row_s) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        case_s[i] = c[i];
        act_s[i] = a[i];
        ts_s[i] = t[i];
        if (row_s) row_s[i] = (int32_t)i;   // presorted: position k is row k
    }
}

static unsigned copy_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

hipError_t launch_segsort(SortBufs in, int64_t n, RangeInfo* info, int32_t* case_s, int32_t* act_s,
                          int64_t* ts_s, int act_shift, uint32_t* wincnt, int32_t* row_s, hipStream_t s) {
    ProfScope p(P_SEGSORT, s);
    if (n > 0) {
        if (row_s)
            k_segsort<true><<<(unsigned)segsort_blocks(n), kSB, 0, s>>>(in, n, info, case_s, act_s, ts_s,
                                                                         act_shift, wincnt, row_s);
        else
            k_segsort<false><<<(unsigned)segsort_blocks(n), kSB, 0, s>>>(in, n, info, case_s, act_s, ts_s,
                                                                          act_shift, wincnt, nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_unbias_copy(SortBufs in, int64_t n, const RangeInfo* info, int32_t* case_s,
                              int32_t* act_s, int64_t* ts_s, int act_shift, int32_t* row_s, hipStream_t s) {
    if (n > 0) k_unbias_copy<<<copy_grid(n), 256, 0, s>>>(in, n, info, case_s, act_s, ts_s, act_shift, row_s);
    return hipGetLastError();
}

hipError_t launch_copy_log(const int32_t* c, const int32_t* a, const int64_t* t, int64_t n,
                           int32_t* case_s, int32_t* act_s, int64_t* ts_s, int32_t* row_s, hipStream_t s) {
    if (n > 0) k_copy_log<<<copy_grid(n), 256, 0, s>>>(c, a, t, n, case_s, act_s, ts_s, row_s);
    return hipGetLastError();
}

}  // namespace pm4g
