// One drill-down view of a prepared log materialised as a prepared log of its
// own (Sec. 3: timestamp filter on events and attribute filter, applied on
// the formatted log, whose (case, timestamp, row) order the kept events
// keep).  Stream compaction over the view's slice [p0, p1) (whole cases):
//   k_filter_slice   p0, p1 from the case range (binary search), on the device
//   k_filter_count   per-tile kept counts (persistent grid over the slice)
//   scan             tile offsets, kept total
//   k_filter_emit    kept events written in order
//   case table       of the kept events (cases.hip); case_off[C] = kept total
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

__device__ __forceinline__ bool keep(const pm4g_view& v, const uint64_t* mask, int32_t a, int64_t t) {
    return t >= v.t_lo && t <= v.t_hi && ((mask[a >> 6] >> (a & 63)) & 1ull);
}

__global__ __launch_bounds__(kFB) void k_filter_count(const int32_t* __restrict__ act_s,
                                                      const int64_t* __restrict__ ts_s, const pm4g_view* view,
                                                      const uint64_t* mask, FilterWs w) {
    __shared__ uint32_t tmp[kFB / kWave + 1];
    const pm4g_view v = *view;
    const int64_t p0 = w.scal[0], p1 = w.scal[1], nt = w.scal[2];
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        uint32_t c = 0;
        for (int q = 0; q < kFI; ++q) {
            const int64_t i = p0 + t * kFilterTile + q * kFB + threadIdx.x;
            if (i < p1 && keep(v, mask, act_s[i], ts_s[i])) ++c;
        }
        uint32_t total;
        block_excl_sum<kFB>(c, tmp, &total);
        if (threadIdx.x == 0) w.tile_cnt[t] = total;
    }
}

__global__ __launch_bounds__(kFB) void k_filter_emit(const int32_t* __restrict__ case_s,
                                                     const int32_t* __restrict__ act_s,
                                                     const int64_t* __restrict__ ts_s, const pm4g_view* view,
                                                     const uint64_t* mask, FilterWs w, int32_t* o_case,
                                                     int32_t* o_act, int64_t* o_ts) {
    __shared__ uint32_t tmp[kFB / kWave + 1];
    const pm4g_view v = *view;
    const int64_t p0 = w.scal[0], p1 = w.scal[1], nt = w.scal[2];
    for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
        // blocked: thread owns 16 consecutive events, so ranks follow positions
        const int64_t base = p0 + t * kFilterTile + (int64_t)threadIdx.x * kFI;
        uint32_t flags = 0;
        for (int q = 0; q < kFI; ++q) {
            const int64_t i = base + q;
            if (i < p1 && keep(v, mask, act_s[i], ts_s[i])) flags |= 1u << q;
        }
        uint32_t total;
        int64_t r = w.tile_off[t] + block_excl_sum<kFB>((uint32_t)__popc(flags), tmp, &total);
        for (int q = 0; q < kFI; ++q) {
            if (!(flags & (1u << q))) continue;
            const int64_t i = base + q;
            o_case[r] = case_s[i];
            o_act[r] = act_s[i];
            o_ts[r] = ts_s[i];
            ++r;
        }
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
                                                          const int64_t* blockoff, int64_t* case_off,
                                                          int32_t* case_code, int64_t* n_cases) {
    __shared__ uint32_t tmp[256 / kWave + 1];
    const int64_t n = w.scal[3];
    const int64_t nb = (n + kCaseTile - 1) / kCaseTile;
    constexpr int kCI = kCaseTile / 256;
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int64_t base = b * kCaseTile + (int64_t)threadIdx.x * kCI;
        uint32_t flags = 0;
        for (int q = 0; q < kCI; ++q) {
            const int64_t i = base + q;
            if (i < n && (i == 0 || c[i] != c[i - 1])) flags |= 1u << q;
        }
        uint32_t total;
        int64_t r = blockoff[b] + block_excl_sum<256>((uint32_t)__popc(flags), tmp, &total);
        for (int q = 0; q < kCI; ++q) {
            if (!(flags & (1u << q))) continue;
            case_off[r] = base + q;
            case_code[r] = c[base + q];
            ++r;
        }
    }
}

__global__ void k_filter_case_done(FilterWs w, const int64_t* ncase_total, int64_t* case_off, int64_t* n_cases,
                                   int32_t* status, const int32_t* status_in) {
    const int64_t C = *ncase_total;
    case_off[C] = w.scal[3];
    *n_cases = C;
    *status = (status_in && *status_in) ? *status_in : (w.scal[7] ? PM4G_E_CAPACITY : 0);
}

}  // namespace

hipError_t launch_filter_view(const pm4g_prepared* p, const pm4g_view* view, const uint64_t* mask,
                              const pm4g_prepared* out, FilterWs w, hipStream_t s) {
    ProfScope ps(P_VIEW_FILTER, s);
    const int64_t n = p->n_events;
    const int64_t ntiles = (n + kFilterTile - 1) / kFilterTile;
    const unsigned grid = (unsigned)(ntiles < 2048 ? (ntiles < 1 ? 1 : ntiles) : 2048);
    k_filter_slice<<<1, 1, 0, s>>>(view, p->case_off, p->case_code, p->n_cases, out->n_events, w);
    k_filter_count<<<grid, kFB, 0, s>>>(p->act_s, p->ts_s, view, mask, w);
    // tile offsets: tile_cnt has scal[2] valid entries; total -> scal[3]
    dev::excl_scan<int64_t>(w.tile_cnt, &w.scal[2], w.tile_off, w.part64, &w.scal[3], s);
    k_filter_emit<<<grid, kFB, 0, s>>>(p->case_s, p->act_s, p->ts_s, view, mask, w, out->case_s, out->act_s,
                                       out->ts_s);
    const int64_t nbc = case_blocks(n);
    const unsigned g2 = (unsigned)(nbc < 2048 ? (nbc < 1 ? 1 : nbc) : 2048);
    k_filter_case_count<<<g2, 256, 0, s>>>(out->case_s, w, w.caseblk, nbc + 1);
    // per-block case offsets into tile_off (free again after the emit); total cases -> scal[5]
    k_filter_nblocks<<<1, 1, 0, s>>>(w);
    dev::excl_scan<int64_t>(w.caseblk, &w.scal[6], w.tile_off, w.part64, &w.scal[5], s);
    k_filter_case_emit<<<g2, 256, 0, s>>>(out->case_s, w, w.tile_off, out->case_off, out->case_code, out->n_cases);
    k_filter_case_done<<<1, 1, 0, s>>>(w, &w.scal[5], out->case_off, out->n_cases, out->status, p->status);
    return hipGetLastError();
}

}  // namespace pm4g
