// Sampling of a prepared log (Sec. 3: the sampling module, a sample by a
// number of cases or of events).  The k units (cases by id, or events by their
// position in the formatted log) with the smallest SplitMix64 keys are kept;
// the keys are distinct, so the sample is unique and nested in k.
//
// The k-th smallest key is found by an MSD radix select over 8-bit digits:
// each pass recomputes the keys (no memory traffic for events; 4 B per case
// code), histograms the next digit of the keys that match the prefix found so
// far, and one block picks the digit that holds the k-th.  The kept units are
// then materialised by the event-filter compaction or the case-filter copy.
#include "common.hpp"
#include "internal.hpp"
#include "prof.hpp"
#include "../../include/pm4g.h"

namespace pm4g {
namespace {

constexpr int kSB = 256;

__global__ void k_sel_init(SelState* sel, int64_t k, const int64_t* count_dev, int64_t count_host) {
    const int64_t count = count_dev ? *count_dev : count_host;
    sel->prefix = 0;
    sel->krem = k;
    sel->T = ~0ull;
    sel->none = k <= 0 ? 1 : 0;
    sel->all = (k > 0 && k >= count) ? 1 : 0;
    for (int d = 0; d < 256; ++d) sel->hist[d] = 0;
}

// Digit `pass` (most significant first) of the keys whose higher digits equal
// the prefix.
__global__ __launch_bounds__(kSB) void k_sel_hist(const int32_t* __restrict__ case_code, const int64_t* count_dev,
                                                  int64_t count_host, uint64_t seed, int pass, SelState* sel) {
    __shared__ uint32_t h[256];
    if (sel->none || sel->all) return;   // uniform: nothing to select
    const int64_t count = count_dev ? *count_dev : count_host;
    const uint64_t prefix = sel->prefix;
    const int hi_shift = 64 - 8 * pass;   // bits above the digit
    const int shift = 56 - 8 * pass;
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t u = (int64_t)blockIdx.x * kSB + threadIdx.x; u < count; u += (int64_t)gridDim.x * kSB) {
        const uint64_t x = case_code ? (uint64_t)(uint32_t)case_code[u] : (uint64_t)u;
        const uint64_t key = splitmix64(seed, x);
        if (pass == 0 || (key >> hi_shift) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&sel->hist[threadIdx.x], h[threadIdx.x]);
}

// One block of 256: the digit whose bin holds the krem-th smallest candidate.
__global__ __launch_bounds__(256) void k_sel_pick(SelState* sel, int last) {
    __shared__ uint32_t tmp[256 / kWave + 1];
    if (sel->none || sel->all) return;
    const uint32_t v = sel->hist[threadIdx.x];
    uint32_t total;
    const uint32_t ex = block_excl_sum<256>(v, tmp, &total);
    const int64_t krem = sel->krem;
    __syncthreads();
    if ((int64_t)ex < krem && krem <= (int64_t)ex + (int64_t)v) {   // exactly one thread
        const uint64_t np = (sel->prefix << 8) | (uint64_t)threadIdx.x;
        sel->krem = krem - (int64_t)ex;
        sel->prefix = np;
        if (last) sel->T = np;
    }
    __syncthreads();
    sel->hist[threadIdx.x] = 0;
}

}  // namespace

hipError_t launch_sample_select(const pm4g_prepared* p, int64_t k, uint64_t seed, bool by_events, SelState* sel,
                                hipStream_t s) {
    const int64_t* count_dev = by_events ? nullptr : p->n_cases;
    const int64_t count_host = p->n_events;   // events, or an upper bound of the cases
    const int32_t* codes = by_events ? nullptr : p->case_code;
    const int64_t g = (count_host + kSB - 1) / kSB;
    const unsigned grid = (unsigned)(g < 2048 ? (g < 1 ? 1 : g) : 2048);
    k_sel_init<<<1, 1, 0, s>>>(sel, k, count_dev, count_host);
    for (int pass = 0; pass < 8; ++pass) {
        k_sel_hist<<<grid, kSB, 0, s>>>(codes, count_dev, count_host, seed, pass, sel);
        k_sel_pick<<<1, 256, 0, s>>>(sel, pass == 7 ? 1 : 0);
    }
    return hipGetLastError();
}

}  // namespace pm4g
