// Case table of a prepared log (Sec. 3, third formatting step, "cases
// dataframe"; Sec. 2.1 group identification): case_code[j] is the j-th
// distinct case id in order and case_off[j] the position of its first event.
// Reduce-then-scan compaction of the boundary flags
// flag(i) = (i == 0) || case_s[i] != case_s[i-1]:
//   k_case_count  per-tile flag counts (or k_case_tiles: from the per-window
//                 case counts the per-case sort already produced)
//   k_case_scan   exclusive scan of the tile counts, n_cases, case_off[C] = N
//   k_case_emit   per-tile ranks -> case_off / case_code
// Bytes per event: 4 + 4 read (the column is read twice).
#include "common.hpp"
#include "internal.hpp"
#include "prof.hpp"

namespace pm4g {

constexpr int kCB = 256;
constexpr int kCI = kCaseTile / kCB;   // 16

__global__ __launch_bounds__(kCB) void k_case_count(const int32_t* __restrict__ case_s, int64_t n,
                                                    uint32_t* blockcnt) {
    __shared__ uint32_t tmp[kCB / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kCaseTile;
    // loads at clamped positions (n >= 1), all issued before any is used
    int32_t cv[kCI], pv[kCI];
#pragma unroll
    for (int k = 0; k < kCI; ++k) {
        const int64_t i = base + k * kCB + threadIdx.x;
        const int64_t ic = i < n ? i : n - 1;
        cv[k] = case_s[ic];
        pv[k] = case_s[ic > 0 ? ic - 1 : 0];
    }
    __builtin_amdgcn_sched_barrier(0);
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kCI; ++k) {
        const int64_t i = base + k * kCB + threadIdx.x;
        if (i < n && (i == 0 || cv[k] != pv[k])) ++c;
    }
    uint32_t total;
    block_excl_sum<kCB>(c, tmp, &total);
    if (threadIdx.x == 0) blockcnt[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_case_scan(uint32_t* blockcnt, int64_t nb, int64_t n,
                                                    int64_t* case_off, int64_t* n_cases) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
    uint32_t run = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        const int64_t i = c0 + threadIdx.x;
        const uint32_t v = i < nb ? blockcnt[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_sum<1024>(v, tmp, &total);
        if (i < nb) blockcnt[i] = run + ex;
        run += total;
    }
    if (threadIdx.x == 0) {
        *n_cases = run;
        case_off[run] = n;
    }
}

// Tile counts from per-window counts (kCaseTile / kSegWindow windows per tile),
// written by the per-case sort.
__global__ __launch_bounds__(1024) void k_case_tiles(const uint32_t* wincnt, int64_t nwin, uint32_t* blockcnt,
                                                     int64_t nb) {
    constexpr int kPerTile = kCaseTile / kSegWindow;
    for (int64_t t = (int64_t)blockIdx.x * 1024 + threadIdx.x; t < nb; t += (int64_t)gridDim.x * 1024) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < kPerTile; ++k) {
            const int64_t w = t * kPerTile + k;
            if (w < nwin) c += wincnt[w];
        }
        blockcnt[t] = c;
    }
}

__global__ __launch_bounds__(kCB) void k_case_emit(const int32_t* __restrict__ case_s, int64_t n,
                                                   const uint32_t* blockoff, int64_t* case_off,
                                                   int32_t* case_code) {
    // striped layout (coalesced loads): item k of thread t is position base + k*256 + t,
    // so position order is (k, wave, lane) order; ranks from ballots + one small scan
    constexpr int kNW = kCB / kWave;
    __shared__ uint32_t wcnt[kCI * kNW];
    __shared__ uint32_t tmp[kCB / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kCaseTile;
    const int w = threadIdx.x / kWave;
    uint64_t masks[kCI];
    // loads at clamped positions (n >= 1), all issued before any is used
    int32_t cv[kCI], pv[kCI];
#pragma unroll
    for (int k = 0; k < kCI; ++k) {
        const int64_t i = base + k * kCB + threadIdx.x;
        const int64_t ic = i < n ? i : n - 1;
        cv[k] = case_s[ic];
        pv[k] = case_s[ic > 0 ? ic - 1 : 0];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kCI; ++k) {
        const int64_t i = base + k * kCB + threadIdx.x;
        const bool f = i < n && (i == 0 || cv[k] != pv[k]);
        masks[k] = __ballot(f);
        if (lane() == 0) wcnt[k * kNW + w] = (uint32_t)__popcll(masks[k]);
    }
    __syncthreads();
    // exclusive scan of the kCI * kNW (k-major) wave counts; kCI * kNW = 64 <= kCB
    uint32_t total;
    const uint32_t v = threadIdx.x < kCI * kNW ? wcnt[threadIdx.x] : 0u;
    const uint32_t ex = block_excl_sum<kCB>(v, tmp, &total);
    if (threadIdx.x < kCI * kNW) wcnt[threadIdx.x] = ex;
    __syncthreads();
    const uint32_t b0 = blockoff[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kCI; ++k) {
        if ((masks[k] >> lane()) & 1ull) {
            const uint32_t r = b0 + wcnt[k * kNW + w] + (uint32_t)__popcll(masks[k] & lanes_below());
            case_off[r] = base + k * kCB + threadIdx.x;
            case_code[r] = cv[k];
        }
    }
}

hipError_t launch_case_table(const int32_t* case_s, int64_t n, uint32_t* blockcnt, int64_t* case_off,
                             int32_t* case_code, int64_t* n_cases, const uint32_t* wincnt, hipStream_t s) {
    static_assert(kCaseTile % kSegWindow == 0, "case tiles hold whole sort windows");
    ProfScope p(P_CASE_TABLE, s);
    const int64_t nb = case_blocks(n);
    if (nb > 0) {
        if (wincnt) {
            const int64_t g = (nb + 1023) / 1024;
            k_case_tiles<<<(unsigned)(g < 1024 ? g : 1024), 1024, 0, s>>>(wincnt, segsort_blocks(n), blockcnt, nb);
        } else {
            k_case_count<<<(unsigned)nb, kCB, 0, s>>>(case_s, n, blockcnt);
        }
    }
    k_case_scan<<<1, 1024, 0, s>>>(blockcnt, nb, n, case_off, n_cases);
    if (nb > 0) k_case_emit<<<(unsigned)nb, kCB, 0, s>>>(case_s, n, blockcnt, case_off, case_code);
    return hipGetLastError();
}

}  // namespace pm4g
