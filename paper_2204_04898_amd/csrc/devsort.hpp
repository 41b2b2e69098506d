// Device-sized building blocks: the element count lives in device memory
// (it is data-dependent, e.g. the number of cases); persistent grids visit
// only the tiles that hold data.
//   - stable LSD radix sort of (key, u32 value) pairs, 8-bit digits,
//     ballot ranking in wave64, LDS staging (same scheme as radix.hip);
//   - exclusive prefix sum, reduce-then-scan over a fixed grid.
#pragma once

#include "common.hpp"

#pragma clang diagnostic ignored "-Wunneeded-internal-declaration"

namespace pm4g {
namespace dev {
// internal linkage: every including file gets its own kernels
namespace {

constexpr int kB = 512;
constexpr int kI = 8;
constexpr int kTile = kB * kI;
constexpr int kW = kB / kWave;

inline int64_t tiles(int64_t nmax) { return (nmax + kTile - 1) / kTile; }

constexpr int kMaxGrid = 2048;   // persistent blocks; tiles are visited grid-stride

inline unsigned grid_for(int64_t nb) { return (unsigned)(nb < kMaxGrid ? (nb < 1 ? 1 : nb) : kMaxGrid); }

// hist is digit-major with row stride nb (an upper bound); only the first
// ceil(n/kTile) tiles of each row are written and scanned.
template <typename K>
__global__ __launch_bounds__(kB) void k_hist(const K* __restrict__ key, const int64_t* n_dev, int shift,
                                             uint32_t* hist, int64_t nb) {
    __shared__ uint32_t h[256];
    const int64_t n = *n_dev;
    const int64_t tiles_n = (n + kTile - 1) / kTile;
    for (int64_t tile = blockIdx.x; tile < tiles_n; tile += gridDim.x) {
        if (threadIdx.x < 256) h[threadIdx.x] = 0;
        __syncthreads();
        const int64_t base = tile * kTile;
        // keys at clamped positions (n >= 1 here), all loaded before the first atomic
        K kv[kI];
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            const int64_t i = base + k * kB + threadIdx.x;
            kv[k] = key[i < n ? i : n - 1];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            const int64_t i = base + k * kB + threadIdx.x;
            if (i < n) atomicAdd(&h[(uint32_t)(kv[k] >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x < 256) hist[(int64_t)threadIdx.x * nb + tile] = h[threadIdx.x];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_hist_scan(uint32_t* hist, const int64_t* n_dev, int64_t nb_stride,
                                                   uint32_t* rowsum) {
    __shared__ uint32_t tmp[256 / kWave + 1];
    const int64_t nb = (*n_dev + kTile - 1) / kTile;
    uint32_t* row = hist + (int64_t)blockIdx.x * nb_stride;
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

template <typename K>
__global__ __launch_bounds__(kB) void k_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                const int64_t* n_dev, int shift, const uint32_t* hist,
                                                const uint32_t* rowsum, int64_t nb) {
    __shared__ uint32_t cnt[kW * 256];
    __shared__ uint32_t tstart[256];
    __shared__ int64_t gshift[256];
    __shared__ K skey[kTile];
    __shared__ uint32_t sval[kTile];
    __shared__ uint32_t tmp[kB / kWave + 1];

    const int64_t n = *n_dev;
    const int64_t tiles_n = (n + kTile - 1) / kTile;
    const int w = threadIdx.x / kWave;
    uint32_t all;
    const uint32_t rs = threadIdx.x < 256 ? rowsum[threadIdx.x] : 0u;
    const uint32_t digit_base = block_excl_sum<kB>(rs, tmp, &all);

    const XcdSplit xs = xcd_split(tiles_n);   // neighbouring tiles' digit runs meet in one L2
    for (int64_t tile = xs.first; tile < xs.end; tile += xs.stride) {
        const int64_t tile0 = tile * kTile;
        const int64_t wbase = tile0 + (int64_t)w * (kWave * kI);
        for (int i = threadIdx.x; i < kW * 256; i += kB) cnt[i] = 0;

        K key[kI];
        uint32_t val[kI], dg[kI], rk[kI];
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            const int64_t i = wbase + k * kWave + lane();
            key[k] = i < n ? kin[i] : K(0);
            val[k] = i < n ? vin[i] : 0u;
            dg[k] = (uint32_t)(key[k] >> shift) & 255u;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kI; ++k) {
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
        uint32_t tot = 0;
        if (threadIdx.x < 256) {
            uint32_t run = 0;
            for (int ww = 0; ww < kW; ++ww) {
                const uint32_t x = cnt[ww * 256 + threadIdx.x];
                cnt[ww * 256 + threadIdx.x] = run;
                run += x;
            }
            tot = run;
        }
        const uint32_t ts_excl = block_excl_sum<kB>(tot, tmp, &all);
        if (threadIdx.x < 256) {
            tstart[threadIdx.x] = ts_excl;
            gshift[threadIdx.x] =
                (int64_t)digit_base + (int64_t)hist[(int64_t)threadIdx.x * nb + tile] - (int64_t)ts_excl;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            const int64_t i = wbase + k * kWave + lane();
            if (i < n) {
                const uint32_t pos = tstart[dg[k]] + cnt[w * 256 + dg[k]] + rk[k];
                skey[pos] = key[k];
                sval[pos] = val[k];
            }
        }
        __syncthreads();
        const int64_t vc = (n - tile0) < kTile ? (n - tile0) : kTile;
        for (int i = threadIdx.x; i < vc; i += kB) {
            const K k = skey[i];
            const int64_t g = gshift[(uint32_t)(k >> shift) & 255u] + i;
            kout[g] = k;
            vout[g] = sval[i];
        }
        __syncthreads();
    }
}

// Stable sort of (k0, v0) by the key bits [0, bits); ping-pongs with (k1, v1).
// Returns true if the result ended in (k1, v1).
template <typename K>
inline bool sort_pairs(K* k0, uint32_t* v0, K* k1, uint32_t* v1, const int64_t* n_dev, int64_t nmax,
                       int bits, uint32_t* hist, uint32_t* rowsum, hipStream_t s) {
    const int64_t nb = tiles(nmax);
    if (nb == 0) return false;
    bool flip = false;
    for (int shift = 0; shift < bits; shift += 8) {
        K* ki = flip ? k1 : k0;
        uint32_t* vi = flip ? v1 : v0;
        K* ko = flip ? k0 : k1;
        uint32_t* vo = flip ? v0 : v1;
        k_hist<K><<<grid_for(nb), kB, 0, s>>>(ki, n_dev, shift, hist, nb);
        k_hist_scan<<<256, 256, 0, s>>>(hist, n_dev, nb, rowsum);
        k_scatter<K><<<grid_for(nb), kB, 0, s>>>(ki, vi, ko, vo, n_dev, shift, hist, rowsum, nb);
        flip = !flip;
    }
    return flip;
}

// ---- exclusive prefix sum of u32 values into T (u32 or u64) ----------------
constexpr int kScanGrid = 1024;

template <typename T>
__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* in, const int64_t* n_dev,
                                                     T* partial) {
    __shared__ T red[256 / kWave];
    const int64_t n = *n_dev;
    const int64_t chunk = (n + kScanGrid - 1) / kScanGrid;
    const int64_t b0 = blockIdx.x * chunk;
    const int64_t b1 = (b0 + chunk) < n ? (b0 + chunk) : n;
    T s = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) s += in[i];
    s = wave_sum(s);
    if (lane() == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int k = 0; k < 256 / kWave; ++k) t += red[k];
        partial[blockIdx.x] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(kScanGrid) void k_scan_top(T* partial, T* total_out) {
    __shared__ T tmp[kScanGrid / kWave + 1];
    T total;
    const T v = partial[threadIdx.x];
    const T ex = block_excl_sum<kScanGrid>(v, tmp, &total);
    partial[threadIdx.x] = ex;
    if (threadIdx.x == 0 && total_out) *total_out = total;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* in, const int64_t* n_dev,
                                                    const T* partial, T* out) {
    __shared__ T tmp[256 / kWave + 1];
    const int64_t n = *n_dev;
    const int64_t chunk = (n + kScanGrid - 1) / kScanGrid;
    const int64_t b0 = blockIdx.x * chunk;
    const int64_t b1 = (b0 + chunk) < n ? (b0 + chunk) : n;
    T run = partial[blockIdx.x];
    for (int64_t c0 = b0; c0 < b1; c0 += 256) {
        const int64_t i = c0 + threadIdx.x;
        const T v = i < b1 ? (T)in[i] : (T)0;
        T total;
        const T ex = block_excl_sum<256>(v, tmp, &total);
        if (i < b1) out[i] = run + ex;
        run += total;
    }
}

// out[i] = sum of in[0..i), i < n; *total = sum of all (if not NULL).
// `partial` needs kScanGrid entries of T.
template <typename T>
inline void excl_scan(const uint32_t* in, const int64_t* n_dev, T* out, T* partial, T* total,
                      hipStream_t s) {
    k_scan_reduce<T><<<kScanGrid, 256, 0, s>>>(in, n_dev, partial);
    k_scan_top<T><<<1, kScanGrid, 0, s>>>(partial, total);
    k_scan_apply<T><<<kScanGrid, 256, 0, s>>>(in, n_dev, partial, out);
}

}  // namespace
}  // namespace dev
}  // namespace pm4g
