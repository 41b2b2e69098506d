// Range scan of a raw log: case-id and timestamp extremes (they fix the
// radix key widths), activity validation, and the order check for a log
// that claims to be presorted (Sec. 3: (case, timestamp, row) order).
//
// Streaming pass, HBM-bound: 8 bytes/event (case, activity), 16 with the
// timestamp.  Block reductions into per-block partials, folded by one block
// (no same-address atomics: across the 8 XCDs they serialise).
#include "common.hpp"
#include "internal.hpp"
#include "prof.hpp"
#include "../../include/pm4g.h"

namespace pm4g {

__global__ void k_range_init(RangeInfo* info) {
    info->case_min = INT32_MAX;
    info->case_max = INT32_MIN;
    info->status = 0;
    info->long_case = 0;
    info->ts_min = INT64_MAX;
    info->ts_max = INT64_MIN;
}

template <bool PRESORTED, bool WANT_TS>
__global__ __launch_bounds__(256) void k_range_scan(const int32_t* __restrict__ case_id,
                                                    const int32_t* __restrict__ act,
                                                    const int64_t* __restrict__ ts, int64_t n,
                                                    int32_t A, RangePart* part) {
    __shared__ RangePart red[256 / kWave];
    int32_t cmin = INT32_MAX, cmax = INT32_MIN;
    int64_t tmin = INT64_MAX, tmax = INT64_MIN;
    bool bad_act = false, unsorted = false;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    auto visit = [&](int64_t i, int32_t c, int32_t a) {
        bad_act |= (uint32_t)a >= (uint32_t)A;
        cmin = c < cmin ? c : cmin;
        cmax = c > cmax ? c : cmax;
        if (WANT_TS || PRESORTED) {
            const int64_t t = ts[i];
            tmin = t < tmin ? t : tmin;
            tmax = t > tmax ? t : tmax;
            if (PRESORTED && i > 0) {
                const int32_t c0 = case_id[i - 1];
                const int64_t t0 = ts[i - 1];
                unsorted |= (c0 > c) || (c0 == c && t0 > t);
            }
        }
    };
    if (!WANT_TS && !PRESORTED) {
        // 16-byte loads of four ids and four activities (the columns are 16-byte aligned
        // torch/hip allocations; a misaligned start falls back to the scalar loop)
        const bool aligned = ((reinterpret_cast<uintptr_t>(case_id) | reinterpret_cast<uintptr_t>(act)) & 15) == 0;
        const int64_t n4 = aligned ? n / 4 : 0;
        const int4* c4 = reinterpret_cast<const int4*>(case_id);
        const int4* a4 = reinterpret_cast<const int4*>(act);
        int64_t q = tid;
        for (; q + stride < n4; q += 2 * stride) {   // two loads of each column in flight
            const int4 c = c4[q], cb = c4[q + stride];
            const int4 a = a4[q], ab = a4[q + stride];
            visit(4 * q, c.x, a.x);
            visit(4 * q + 1, c.y, a.y);
            visit(4 * q + 2, c.z, a.z);
            visit(4 * q + 3, c.w, a.w);
            visit(4 * (q + stride), cb.x, ab.x);
            visit(4 * (q + stride) + 1, cb.y, ab.y);
            visit(4 * (q + stride) + 2, cb.z, ab.z);
            visit(4 * (q + stride) + 3, cb.w, ab.w);
        }
        for (; q < n4; q += stride) {
            const int4 c = c4[q];
            const int4 a = a4[q];
            visit(4 * q, c.x, a.x);
            visit(4 * q + 1, c.y, a.y);
            visit(4 * q + 2, c.z, a.z);
            visit(4 * q + 3, c.w, a.w);
        }
        for (int64_t i = 4 * n4 + tid; i < n; i += stride) visit(i, case_id[i], act[i]);
    } else {
        for (int64_t i = tid; i < n; i += stride) visit(i, case_id[i], act[i]);
    }
    RangePart r;
    r.cmin = wave_min(cmin);
    r.cmax = wave_max(cmax);
    r.tmin = wave_min(tmin);
    r.tmax = wave_max(tmax);
    r.bad = __ballot(bad_act) != 0;
    r.unsorted = __ballot(unsorted) != 0;
    if (lane() == 0) red[threadIdx.x / kWave] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 256 / kWave; ++k) {
            const RangePart& o = red[k];
            r.cmin = o.cmin < r.cmin ? o.cmin : r.cmin;
            r.cmax = o.cmax > r.cmax ? o.cmax : r.cmax;
            r.tmin = o.tmin < r.tmin ? o.tmin : r.tmin;
            r.tmax = o.tmax > r.tmax ? o.tmax : r.tmax;
            r.bad |= o.bad;
            r.unsorted |= o.unsorted;
        }
        part[blockIdx.x] = r;
    }
}

// The formatting step's range scan over radix tiles (kRadixTile events per
// block, no timestamps): besides the partials, each tile's histogram of the
// low 8 bits of the raw case id.  The first radix pass digit is the low byte
// of case - case_min, a rotation of that byte by case_min, so this histogram
// replaces the first pass's histogram kernel (k_radix_scan_rot rotates it).
__global__ __launch_bounds__(kRangeTileThreads) void k_range_tiles(const int32_t* __restrict__ case_id,
                                                                   const int32_t* __restrict__ act, int64_t n,
                                                                   int32_t A, RangePart* part,
                                                                   uint32_t* hist_raw, int64_t nb) {
    __shared__ uint32_t h[256];
    __shared__ RangePart red[kRangeTileThreads / kWave];
    constexpr int kT = kRangeTileThreads;
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    int32_t cmin = INT32_MAX, cmax = INT32_MIN;
    bool bad = false;
    auto visit = [&](int32_t c, int32_t a) {
        bad |= (uint32_t)a >= (uint32_t)A;
        cmin = c < cmin ? c : cmin;
        cmax = c > cmax ? c : cmax;
        atomicAdd(&h[(uint32_t)c & 255u], 1u);
    };
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    const bool vec = base + kRadixTile <= n &&
                     ((reinterpret_cast<uintptr_t>(case_id) | reinterpret_cast<uintptr_t>(act)) & 15) == 0;
    if (vec) {
        const int4* c4 = reinterpret_cast<const int4*>(case_id + base);
        const int4* a4 = reinterpret_cast<const int4*>(act + base);
#pragma unroll
        for (int q = 0; q < kRadixTile / (4 * kT); ++q) {
            const int4 c = c4[q * kT + threadIdx.x];
            const int4 a = a4[q * kT + threadIdx.x];
            visit(c.x, a.x);
            visit(c.y, a.y);
            visit(c.z, a.z);
            visit(c.w, a.w);
        }
    } else {
        for (int64_t i = base + threadIdx.x; i < n && i < base + kRadixTile; i += kT) visit(case_id[i], act[i]);
    }
    RangePart r{wave_min(cmin), wave_max(cmax), __ballot(bad) != 0, 0, INT64_MAX, INT64_MIN};
    if (lane() == 0) red[threadIdx.x / kWave] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kT / kWave; ++k) {
            r.cmin = red[k].cmin < r.cmin ? red[k].cmin : r.cmin;
            r.cmax = red[k].cmax > r.cmax ? red[k].cmax : r.cmax;
            r.bad |= red[k].bad;
        }
        part[blockIdx.x] = r;
    }
    if (threadIdx.x < 256) hist_raw[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// One block folds the per-block partials into the RangeInfo.
__global__ __launch_bounds__(1024) void k_range_final(const RangePart* part, int nparts, RangeInfo* info) {
    __shared__ RangePart red[1024 / kWave];
    RangePart r{INT32_MAX, INT32_MIN, 0, 0, INT64_MAX, INT64_MIN};
    for (int k = threadIdx.x; k < nparts; k += 1024) {
        const RangePart o = part[k];
        r.cmin = o.cmin < r.cmin ? o.cmin : r.cmin;
        r.cmax = o.cmax > r.cmax ? o.cmax : r.cmax;
        r.tmin = o.tmin < r.tmin ? o.tmin : r.tmin;
        r.tmax = o.tmax > r.tmax ? o.tmax : r.tmax;
        r.bad |= o.bad;
        r.unsorted |= o.unsorted;
    }
    r.cmin = wave_min(r.cmin);
    r.cmax = wave_max(r.cmax);
    r.tmin = wave_min(r.tmin);
    r.tmax = wave_max(r.tmax);
    r.bad = __ballot(r.bad != 0) != 0;
    r.unsorted = __ballot(r.unsorted != 0) != 0;
    if (lane() == 0) red[threadIdx.x / kWave] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 1024 / kWave; ++k) {
            const RangePart& o = red[k];
            r.cmin = o.cmin < r.cmin ? o.cmin : r.cmin;
            r.cmax = o.cmax > r.cmax ? o.cmax : r.cmax;
            r.tmin = o.tmin < r.tmin ? o.tmin : r.tmin;
            r.tmax = o.tmax > r.tmax ? o.tmax : r.tmax;
            r.bad |= o.bad;
            r.unsorted |= o.unsorted;
        }
        info->case_min = r.cmin;
        info->case_max = r.cmax;
        info->ts_min = r.tmin;
        info->ts_max = r.tmax;
        info->status = r.bad ? PM4G_E_RANGE : (r.unsorted ? PM4G_E_NOT_SORTED : 0);
    }
}

__global__ __launch_bounds__(256) void k_ts_range(const int64_t* __restrict__ ts, int64_t n,
                                                  RangeInfo* info) {
    int64_t tmin = INT64_MAX, tmax = INT64_MIN;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t t = ts[i];
        tmin = t < tmin ? t : tmin;
        tmax = t > tmax ? t : tmax;
    }
    tmin = wave_min(tmin);
    tmax = wave_max(tmax);
    if (lane() == 0) {
        __hip_atomic_fetch_min(&info->ts_min, tmin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_max(&info->ts_max, tmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

static int range_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > kRangeParts) g = kRangeParts;
    return g < 1 ? 1 : (int)g;
}

hipError_t launch_range_scan(const int32_t* case_id, const int32_t* act, const int64_t* ts, int64_t n,
                             int32_t A, bool presorted, bool want_ts, RangeInfo* info, RangePart* part,
                             uint32_t* hist_raw, hipStream_t s) {
    ProfScope p(P_RANGE, s);
    k_range_init<<<1, 1, 0, s>>>(info);
    if (n > 0) {
        if (hist_raw && !presorted && !want_ts) {
            const int64_t nb = radix_blocks(n);
            k_range_tiles<<<(unsigned)nb, kRangeTileThreads, 0, s>>>(case_id, act, n, A, part, hist_raw, nb);
            k_range_final<<<1, 1024, 0, s>>>(part, (int)nb, info);
            return hipGetLastError();
        }
        const int g = range_grid(n);
        if (presorted)
            k_range_scan<true, true><<<g, 256, 0, s>>>(case_id, act, ts, n, A, part);
        else if (want_ts)
            k_range_scan<false, true><<<g, 256, 0, s>>>(case_id, act, ts, n, A, part);
        else
            k_range_scan<false, false><<<g, 256, 0, s>>>(case_id, act, ts, n, A, part);
        k_range_final<<<1, 1024, 0, s>>>(part, g, info);
    }
    return hipGetLastError();
}

hipError_t launch_ts_range(const int64_t* ts, int64_t n, RangeInfo* info, hipStream_t s) {
    if (n > 0) k_ts_range<<<range_grid(n), 256, 0, s>>>(ts, n, info);
    return hipGetLastError();
}

}  // namespace pm4g
