// Device helpers shared by the pm4g kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm4g {

constexpr int kWave = 64;

__device__ __forceinline__ int lane() { return __lane_id(); }

// XCD-contiguous work split.  The dispatcher deals a grid's blocks
// round-robin to the 8 XCDs (block b runs on XCD b % 8), and each XCD has its
// own L2.  Items [0, n) are cut into 8 contiguous ranges, one per XCD; the
// blocks of an XCD stride over its range.  Neighbouring items (whose outputs
// share cache lines at run boundaries) then meet in the same L2.  A bijection
// for any grid; grids below 8 blocks keep the plain split.
struct XcdSplit {
    int64_t first, end, stride;
};
__device__ __forceinline__ XcdSplit xcd_split(int64_t n) {
    const int64_t G = gridDim.x, b = blockIdx.x;
    if (G < 8) return XcdSplit{b, n, G};
    const int64_t x = b % 8, j = b / 8;
    const int64_t blocks = G / 8 + (x < G % 8 ? 1 : 0);   // blocks on XCD x
    const int64_t q = n / 8, r = n % 8;
    const int64_t begin = x * q + (x < r ? x : r);
    return XcdSplit{begin + j, begin + q + (x < r ? 1 : 0), blocks};
}

// Mask of the lanes below this one.
__device__ __forceinline__ uint64_t lanes_below() {
    return (uint64_t(1) << lane()) - uint64_t(1);
}

// Lanes of this wave whose 8-bit digit equals this lane's, among `active`.
// Per bit: the lanes agreeing with this lane are ~(ballot ^ s), s this lane's
// bit spread over the word (0 or all ones), which gfx950 folds with the and
// into one three-input bit operation per 32-bit half.
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, uint64_t active) {
    uint32_t lo = (uint32_t)active, hi = (uint32_t)(active >> 32);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint32_t s = 0u - ((d >> b) & 1u);
        const uint64_t m = __ballot(s != 0u);
        lo &= ~((uint32_t)m ^ s);
        hi &= ~((uint32_t)(m >> 32) ^ s);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Lanes of this wave whose value agrees with this lane's in the low `bits`
// bits, among `active`.  Every lane of the wave must execute it (`bits` is
// wave-uniform).
__device__ __forceinline__ uint64_t match_bits(uint32_t v, int bits, uint64_t active) {
    uint32_t lo = (uint32_t)active, hi = (uint32_t)(active >> 32);
    for (int b = 0; b < bits; ++b) {
        const uint32_t s = 0u - ((v >> b) & 1u);   // as in match_digit8
        const uint64_t m = __ballot(s != 0u);
        lo &= ~((uint32_t)m ^ s);
        hi &= ~((uint32_t)(m >> 32) ^ s);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Wave-aggregated LDS counter increment: the lanes with `has` set add one to
// counter[key]; each gets the counter's value before its own increment (one
// atomic per distinct key).  Every lane of the wave must execute it.
__device__ __forceinline__ uint32_t wave_bump(uint32_t* counter, uint32_t key, int key_bits, bool has) {
    const uint64_t active = __ballot(has);
    const uint64_t peers = match_bits(has ? key : 0u, key_bits, active);
    const uint32_t rank = (uint32_t)__popcll(peers & lanes_below());
    const int leader = has ? (int)__ffsll((unsigned long long)peers) - 1 : 0;
    uint32_t base = 0;
    if (has && rank == 0) base = atomicAdd(&counter[key], (uint32_t)__popcll(peers));
    base = (uint32_t)__shfl((int)base, leader);
    return base + rank;
}

// SplitMix64 (Steele, Lea and Flood, 2014): the x-th output (x = 0, 1, ...)
// of the generator started from state `seed`.  A bijection of x for a fixed
// seed, so distinct inputs never share a key.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t x) {
    uint64_t z = seed + (x + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Segment of position p among 64 consecutive segments (lane m holds the start
// of segment m, INT64_MAX if absent; p >= start of segment 0): the last m
// whose start is <= p.  Every lane of the wave must execute it.
__device__ __forceinline__ int seg_at(int64_t vstart, int64_t p) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int cand = lo + step;
        if (__shfl(vstart, cand) <= p) lo = cand;
    }
    return lo;
}

template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T u = __shfl_up(v, o);
        if (lane() >= o) v += u;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u < v ? u : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

// Exclusive prefix sum over a block of BLOCK threads (one value per thread).
// `tmp` must hold BLOCK/64 + 1 entries of T in LDS.  Returns the exclusive
// sum; *total receives the block total.  Contains __syncthreads().
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_sum(T v, T* tmp, T* total) {
    constexpr int NW = BLOCK / kWave;
    const int w = threadIdx.x / kWave;
    T inc = wave_incl_sum(v);
    if (lane() == kWave - 1) tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < NW; ++i) {
            T x = tmp[i];
            tmp[i] = run;
            run += x;
        }
        tmp[NW] = run;
    }
    __syncthreads();
    T r = tmp[w] + inc - v;
    *total = tmp[NW];
    __syncthreads();
    return r;
}

// Saturating add of non-negative 64-bit amounts, capped at 2^63 (any value
// >= 2^63 means "exceeds INT64_MAX").  Inputs must already be <= 2^63.
__device__ __forceinline__ uint64_t sat_add63(uint64_t a, uint64_t b) {
    constexpr uint64_t cap = uint64_t(1) << 63;
    return (a > cap - b) ? cap : a + b;
}
__device__ __forceinline__ uint64_t cap63(uint64_t a) {
    constexpr uint64_t cap = uint64_t(1) << 63;
    return a > cap ? cap : a;
}

// Record a data-dependent error; the first one wins.
__device__ __forceinline__ void set_status(int32_t* status, int32_t code) {
    atomicCAS(status, 0, code);
}

}  // namespace pm4g
