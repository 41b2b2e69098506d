// Stable LSD radix passes over (key u32, ts i64, act u32) elements, 8-bit
// digits, reduce-then-scan:
//   k_radix_hist     per-tile digit histograms, digit-major [256][tiles]
//   k_radix_scan     exclusive scan of each digit row, row totals
//   k_radix_scatter  wave64 ballot ranking (stable: wave, item, lane order),
//                    LDS staging in digit order, coalesced-run writes; tiles
//                    laid out XCD-contiguously over the grid
// The first pass reads the raw log columns directly (case id biased by the
// case minimum), so the caller's arrays are never copied.
//
// This is the grouping step of Sec. 3's first formatting step: events of a
// case become adjacent while keeping their row order (stability); the
// per-case timestamp order is applied afterwards in LDS (segsort.hip).
// Packed layout (PACKED): when the case bits and the activity bits fit in 32,
// the activity rides in the key above the case bits (key_mask selects the
// case bits) and no activity column moves: 12 bytes per element.
// Bytes per event per pass: 4 (hist) + 16 read + 16 write (12 + 12 packed).
// Row order (ROW): when the caller asks for the permutation, each element
// also carries its original row (the first pass takes it from its position),
// 4 more bytes read and written per element; otherwise nothing moves for it.
#include "common.hpp"
#include "internal.hpp"
#include "prof.hpp"

namespace pm4g {

constexpr int kRB = 512;               // threads per block
constexpr int kRI = kRadixTile / kRB;  // items per thread (8)
constexpr int kRW = kRB / kWave;       // waves per block (8)

template <int SRC>
__device__ __forceinline__ uint32_t digit_of(uint32_t key, int64_t ts, int shift, int64_t ts_min,
                                             uint32_t key_mask) {
    if (SRC == 0) return ((key & key_mask) >> shift) & 255u;
    return (uint32_t)(((uint64_t)ts - (uint64_t)ts_min) >> shift) & 255u;
}

// The first pass reads the raw columns: key = case - case_min (| act << act_shift when packed).
template <bool FIRST, bool PACKED>
__device__ __forceinline__ uint32_t load_key(const SortBufs& in, int64_t i, int32_t case_min, int act_shift) {
    if (FIRST) {
        uint32_t k = (uint32_t)reinterpret_cast<const int32_t*>(in.key)[i] - (uint32_t)case_min;
        if (PACKED) k |= (uint32_t)reinterpret_cast<const int32_t*>(in.act)[i] << act_shift;
        return k;
    }
    return in.key[i];
}

template <int SRC, bool FIRST>
__global__ __launch_bounds__(kRB) void k_radix_hist(SortBufs in, int64_t n, int shift,
                                                    const RangeInfo* info, uint32_t* hist,
                                                    int64_t nb, uint32_t key_mask) {
    __shared__ uint32_t h[256];
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const int32_t case_min = info->case_min;
    const int64_t ts_min = info->ts_min;
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    const bool vec = SRC == 0 && base + kRadixTile <= n && (reinterpret_cast<uintptr_t>(in.key) & 15) == 0;
    if (vec) {
        // full tile: 16-byte loads of four keys
        const uint4* k4 = reinterpret_cast<const uint4*>(in.key + base);
#pragma unroll
        for (int q = 0; q < kRI / 4; ++q) {
            const uint4 v = k4[q * kRB + threadIdx.x];
            const uint32_t bias = FIRST ? (uint32_t)case_min : 0u;
            atomicAdd(&h[digit_of<0>(v.x - bias, 0, shift, 0, key_mask)], 1u);
            atomicAdd(&h[digit_of<0>(v.y - bias, 0, shift, 0, key_mask)], 1u);
            atomicAdd(&h[digit_of<0>(v.z - bias, 0, shift, 0, key_mask)], 1u);
            atomicAdd(&h[digit_of<0>(v.w - bias, 0, shift, 0, key_mask)], 1u);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kRI; ++k) {
            const int64_t i = base + k * kRB + threadIdx.x;
            if (i < n) {
                uint32_t d;
                if (SRC == 0) d = digit_of<0>(load_key<FIRST, false>(in, i, case_min, 0), 0, shift, 0, key_mask);
                else d = digit_of<1>(0, in.ts[i], shift, ts_min, key_mask);
                atomicAdd(&h[d], 1u);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 256) hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: exclusive scan of hist[d][0..nb) in place, row total.
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t* hist, int64_t nb, uint32_t* rowsum) {
    __shared__ uint32_t tmp[256 / kWave + 1];
    uint32_t* row = hist + (int64_t)blockIdx.x * nb;
    uint32_t run = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += 256 * 4) {
        uint32_t v[4];
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = c0 + threadIdx.x * 4 + q;
            v[q] = i < nb ? row[i] : 0u;
            s += v[q];
        }
        uint32_t total;
        uint32_t ex = block_excl_sum<256>(s, tmp, &total);
        uint32_t r = run + ex;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = c0 + threadIdx.x * 4 + q;
            if (i < nb) row[i] = r;
            r += v[q];
        }
        run += total;
    }
    if (threadIdx.x == 0) rowsum[blockIdx.x] = run;
}

// First case pass with the range scan's histograms of the raw low byte u:
// digit d of case - case_min is u = (d + case_min) & 255, so row d is the
// scan of raw row (d + case_min) & 255.
__global__ __launch_bounds__(256) void k_radix_scan_rot(const uint32_t* hist_raw, uint32_t* hist, int64_t nb,
                                                        uint32_t* rowsum, const RangeInfo* info) {
    __shared__ uint32_t tmp[256 / kWave + 1];
    const uint32_t u = (blockIdx.x + (uint32_t)info->case_min) & 255u;
    const uint32_t* in = hist_raw + (int64_t)u * nb;
    uint32_t* row = hist + (int64_t)blockIdx.x * nb;
    uint32_t run = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += 256 * 4) {
        uint32_t v[4];
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = c0 + threadIdx.x * 4 + q;
            v[q] = i < nb ? in[i] : 0u;
            s += v[q];
        }
        uint32_t total;
        uint32_t r = run + block_excl_sum<256>(s, tmp, &total);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = c0 + threadIdx.x * 4 + q;
            if (i < nb) row[i] = r;
            r += v[q];
        }
        run += total;
    }
    if (threadIdx.x == 0) rowsum[blockIdx.x] = run;
}

template <int SRC, bool FIRST, bool PACKED, bool ROW>
__global__ __launch_bounds__(kRB) void k_radix_scatter(SortBufs in, SortBufs out, int64_t n, int shift,
                                                       const RangeInfo* info, const uint32_t* hist,
                                                       const uint32_t* rowsum, int64_t nb,
                                                       uint32_t key_mask, int act_shift) {
    __shared__ uint32_t cnt[kRW * 256];       // per-wave running digit counts
    __shared__ uint32_t tstart[256];          // tile-local start of each digit
    __shared__ int64_t gshift[256];           // global position - tile position
    __shared__ uint32_t skey[kRadixTile];
    __shared__ int64_t sts[kRadixTile];
    __shared__ uint32_t sact[PACKED ? 1 : kRadixTile];
    __shared__ uint32_t srow[ROW ? kRadixTile : 1];
    __shared__ uint32_t tmp[kRB / kWave + 1];

    const int32_t case_min = info->case_min;
    const int64_t ts_min = info->ts_min;
    const int w = threadIdx.x / kWave;
    // one tile per block, XCD-contiguous: the runs of neighbouring tiles meet
    // in the same L2, where their shared boundary lines are completed
    const int64_t tile = xcd_split(nb).first;
    const int64_t tile0 = tile * kRadixTile;
    const int64_t wbase = tile0 + (int64_t)w * (kWave * kRI);

    for (int i = threadIdx.x; i < kRW * 256; i += kRB) cnt[i] = 0;

    uint32_t key[kRI], act[kRI], dg[kRI], rk[kRI], rw[kRI];
    int64_t tv[kRI];
    if constexpr (FIRST) {
        // all loads of the tile first: forming each key from its two raw
        // columns right after their loads (as the compiler schedules it
        // otherwise) made every item's loads wait for the previous item's
        uint32_t rc[kRI], ra[kRI];
#pragma unroll
        for (int k = 0; k < kRI; ++k) {
            const int64_t i = wbase + k * kWave + lane();
            if (i < n) {
                rc[k] = reinterpret_cast<const uint32_t*>(in.key)[i];
                ra[k] = in.act[i];
                tv[k] = in.ts[i];
            } else {
                rc[k] = (uint32_t)case_min;
                ra[k] = 0;
                tv[k] = ts_min;
            }
            rw[k] = (uint32_t)i;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < kRI; ++k) {
            key[k] = rc[k] - (uint32_t)case_min;   // 0 past the end
            if (PACKED) key[k] |= ra[k] << act_shift;
            act[k] = PACKED ? 0u : ra[k];
            dg[k] = digit_of<SRC>(key[k], tv[k], shift, ts_min, key_mask);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kRI; ++k) {
            const int64_t i = wbase + k * kWave + lane();
            if (i < n) {
                key[k] = load_key<FIRST, PACKED>(in, i, case_min, act_shift);
                tv[k] = in.ts[i];
                act[k] = PACKED ? 0u : in.act[i];
                rw[k] = ROW ? in.row[i] : 0u;
            } else {
                key[k] = 0;
                tv[k] = ts_min;
                act[k] = 0;
                rw[k] = 0;
            }
            dg[k] = digit_of<SRC>(key[k], tv[k], shift, ts_min, key_mask);
        }
    }
    __syncthreads();

    // Stable ranks within the wave's contiguous chunk, in (item, lane) order.
#pragma unroll
    for (int k = 0; k < kRI; ++k) {
        const int64_t i = wbase + k * kWave + lane();
        const bool valid = i < n;
        const uint64_t active = __ballot(valid);
        const uint64_t peers = match_digit8(dg[k], active);
        const uint32_t below = __popcll(peers & lanes_below());
        uint32_t c = 0;
        if (valid) c = cnt[w * 256 + dg[k]];
        rk[k] = c + below;
        if (valid && below == 0) cnt[w * 256 + dg[k]] = c + __popcll(peers);
    }
    __syncthreads();

    // Per digit: exclusive offsets of the waves, the tile's digit totals.
    uint32_t tot = 0;
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
        uint32_t run = 0;
        for (int ww = 0; ww < kRW; ++ww) {
            const uint32_t x = cnt[ww * 256 + d];
            cnt[ww * 256 + d] = run;
            run += x;
        }
        tot = run;
    }
    uint32_t all;
    const uint32_t ts_excl = block_excl_sum<kRB>(tot, tmp, &all);
    const uint32_t rs = threadIdx.x < 256 ? rowsum[threadIdx.x] : 0u;
    const uint32_t digit_base = block_excl_sum<kRB>(rs, tmp, &all);
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
        tstart[d] = ts_excl;
        gshift[d] = (int64_t)digit_base + (int64_t)hist[(int64_t)d * nb + tile] - (int64_t)ts_excl;
    }
    __syncthreads();

#pragma unroll
    for (int k = 0; k < kRI; ++k) {
        const int64_t i = wbase + k * kWave + lane();
        if (i < n) {
            const uint32_t pos = tstart[dg[k]] + cnt[w * 256 + dg[k]] + rk[k];
            skey[pos] = key[k];
            sts[pos] = tv[k];
            if (!PACKED) sact[pos] = act[k];
            if (ROW) srow[pos] = rw[k];
        }
    }
    __syncthreads();

    const int64_t valid_count = (n - tile0) < kRadixTile ? (n - tile0) : kRadixTile;
    for (int i = threadIdx.x; i < valid_count; i += kRB) {
        const uint32_t k = skey[i];
        const int64_t t = sts[i];
        const uint32_t d = digit_of<SRC>(k, t, shift, ts_min, key_mask);
        const int64_t g = gshift[d] + i;
        out.key[g] = k;
        out.ts[g] = t;
        if (!PACKED) out.act[g] = sact[i];
        if (ROW) out.row[g] = srow[i];
    }
}

template <int SRC, bool FIRST, bool PACKED, bool ROW>
static void run_pass(SortBufs in, SortBufs out, int64_t n, int shift, const RangeInfo* info,
                     uint32_t* hist, uint32_t* rowsum, uint32_t key_mask, int act_shift,
                     const uint32_t* hist_raw, hipStream_t s) {
    const int64_t nb = radix_blocks(n);
    if (hist_raw) {
        ProfScope p(P_RADIX_SCAN, s);
        k_radix_scan_rot<<<256, 256, 0, s>>>(hist_raw, hist, nb, rowsum, info);
    } else {
        {
            ProfScope p(P_RADIX_HIST, s);
            k_radix_hist<SRC, FIRST><<<(unsigned)nb, kRB, 0, s>>>(in, n, shift, info, hist, nb, key_mask);
        }
        ProfScope p(P_RADIX_SCAN, s);
        k_radix_scan<<<256, 256, 0, s>>>(hist, nb, rowsum);
    }
    ProfScope p(P_RADIX_SCATTER, s);
    k_radix_scatter<SRC, FIRST, PACKED, ROW><<<(unsigned)nb, kRB, 0, s>>>(in, out, n, shift, info, hist, rowsum,
                                                                      nb, key_mask, act_shift);
}

hipError_t launch_radix_pass(SortBufs in, SortBufs out, int64_t n, int digit_src, int shift,
                             bool first, const RangeInfo* info, uint32_t* hist, uint32_t* rowsum,
                             int act_shift, const uint32_t* hist_raw, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const bool packed = act_shift > 0;
    const uint32_t key_mask = packed ? ((act_shift >= 32) ? 0xFFFFFFFFu : ((1u << act_shift) - 1u)) : 0xFFFFFFFFu;
    // the raw-byte histograms describe the first case pass only
    if (!(digit_src == 0 && first && shift == 0)) hist_raw = nullptr;
    // the row order is carried iff the output has a row array
#define PM4G_PASS(SRC, FIRST, PACKED)                                                                        \
    do {                                                                                                    \
        if (out.row)                                                                                        \
            run_pass<SRC, FIRST, PACKED, true>(in, out, n, shift, info, hist, rowsum, key_mask, act_shift, \
                                               hist_raw, s);                                                \
        else                                                                                                \
            run_pass<SRC, FIRST, PACKED, false>(in, out, n, shift, info, hist, rowsum, key_mask, act_shift, \
                                                hist_raw, s);                                               \
    } while (0)
    if (digit_src == 0) {
        if (first) { if (packed) PM4G_PASS(0, true, true); else PM4G_PASS(0, true, false); }
        else { if (packed) PM4G_PASS(0, false, true); else PM4G_PASS(0, false, false); }
    } else {
        if (first) { if (packed) PM4G_PASS(1, true, true); else PM4G_PASS(1, true, false); }
        else { if (packed) PM4G_PASS(1, false, true); else PM4G_PASS(1, false, false); }
    }
#undef PM4G_PASS
    return hipGetLastError();
}

}  // namespace pm4g
