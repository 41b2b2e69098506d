// CSV ingestion into the columns of an event log (Sec. 2.2: a CSV holds a
// header row and data rows of separator-delimited values; the GPU parses
// different parts of the text at once).
//
//   lines     quote characters toggle a quoted state wherever they stand; a
//             line ends at a newline outside quotes (or at the end of the
//             text), without a trailing carriage return; empty lines are
//             skipped; with a header the first non-empty line is skipped.
//   values    fields split at separators outside quotes; a field's value
//             drops the delimiting quotes of its quoted runs and reads a
//             doubled quote inside a run as one quote.
//   columns   case and activity values coded 0, 1, ... in order of first
//             appearance (byte-exact); timestamps integers or ISO-8601
//             date-times in units of 10^-scale s.
//
// Kernels:
//   k_csv_scan_text  per 4096-byte tile: quote parity, and the ends of
//                    non-empty lines for both quote states the tile may start
//                    in (16-bit masks per 16 bytes)
//   scan             quote parity at each tile's start; line counts of the
//                    state each tile starts in; their scan
//   k_csv_lines      line-end positions from the masks
//   k_csv_close      the unterminated last line, row count, capacity
//   k_csv_parse      a thread per data row: field ranges, value hashes, the
//                    timestamp; values enter open-addressing tables keyed by
//                    64-bit hash, each slot keeping its first row; the slots
//                    claimed (one per distinct value) are listed per table
//   k_csv_verify     every row's value against its slot's first row, byte by
//                    byte (a hash collision is detected, and the call is
//                    repeated with another hash seed)
//   codes            the listed slots sorted by first row: the code is the rank
//   k_csv_emit       codes per row
// Bytes: the text is read once by the tile pass and once more by the row
// pass (plus the first rows' values once); 16 B/row written.
#include "common.hpp"
#include "devsort.hpp"
#include "internal.hpp"
#include "prof.hpp"
#include "../../include/pm4g.h"

namespace pm4g {

namespace {

constexpr int kCT = 4096;              // bytes per tile
constexpr int kCTB = 256;              // threads per tile block
constexpr int kCPer = kCT / kCTB;      // 16 bytes per thread
constexpr int kTsMax = 64;             // longest timestamp value

int64_t pow2_at_least(int64_t x) {
    int64_t p = 1024;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

CsvWs csv_ws_layout(Bump& b, int64_t n_bytes, int64_t max_rows) {
    CsvWs w{};
    const int64_t tiles = (n_bytes + kCT - 1) / kCT;
    const size_t t1 = (size_t)(tiles > 0 ? tiles : 1) + 1;
    const size_t rows = (size_t)(max_rows > 0 ? max_rows : 1);
    w.tsize = pow2_at_least(2 * (max_rows > 0 ? max_rows : 1));
    w.qpar = b.take<uint32_t>(t1);
    w.qpre = b.take<uint32_t>(t1);
    w.lcnt = b.take<uint32_t>(t1);
    w.lcnt1 = b.take<uint32_t>(t1);
    w.emask = b.take<uint32_t>((t1 - 1) * kCTB);
    w.loff = b.take<int64_t>(t1);
    w.line_end = b.take<int64_t>(rows + 2);
    w.foff = b.take<int64_t>(2 * rows);
    w.flen = b.take<int32_t>(2 * rows);
    w.slot = b.take<uint32_t>(2 * rows);
    w.table = b.take<CsvSlot>((size_t)(2 * w.tsize));
    w.max_rows = (int64_t)rows;
    w.dlist = b.take<uint32_t>(2 * rows);
    w.k0 = b.take<uint32_t>(rows);
    w.v0 = b.take<uint32_t>(rows);
    w.k1 = b.take<uint32_t>(rows);
    w.v1 = b.take<uint32_t>(rows);
    w.hist = b.take<uint32_t>((size_t)256 * (size_t)dev::tiles((int64_t)rows));
    w.rowsum = b.take<uint32_t>(256);
    w.part32 = b.take<uint32_t>(dev::kScanGrid);
    w.part64 = b.take<int64_t>(dev::kScanGrid);
    w.scal = b.take<int64_t>(16);
    return w;
}

namespace {

// scal: [0] tiles, [1] lines found by the tile pass, [2] data rows, [3] first
// bad row (INT64_MAX: none), [4] hash collision seen, [5] distinct values (case
// table, then activity table), [6] rows over capacity, [7] quote parity at
// the end, [8] table slots, [9] line capacity, [10], [11] slots listed in the
// case and activity tables
__global__ void k_csv_init(CsvWs w, int64_t n_bytes, int64_t max_lines) {
    w.scal[0] = (n_bytes + kCT - 1) / kCT;
    w.scal[1] = 0;
    w.scal[2] = 0;
    w.scal[3] = INT64_MAX;
    w.scal[4] = 0;
    w.scal[5] = 0;
    w.scal[6] = 0;
    w.scal[7] = 0;
    w.scal[8] = w.tsize;
    w.scal[9] = max_lines;
    w.scal[10] = 0;
    w.scal[11] = 0;
}

__global__ __launch_bounds__(256) void k_csv_clear(CsvWs w) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {   // this attempt's retry flag and slot lists
        w.scal[4] = 0;
        w.scal[10] = 0;
        w.scal[11] = 0;
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < 2 * w.tsize; i += (int64_t)gridDim.x * 256) {
        w.table[i].hash = 0;
        w.table[i].first = 0xffffffffu;
        w.table[i].code = 0;
    }
}

// High bit of each byte of x that equals the byte repeated in c8 (exact per
// byte: the 7-bit add cannot carry into the next byte).
__device__ __forceinline__ uint64_t eq_bytes(uint64_t x, uint64_t c8) {
    const uint64_t y = x ^ c8;
    const uint64_t t = (y & 0x7F7F7F7F7F7F7F7Full) + 0x7F7F7F7F7F7F7F7Full;
    return ~(t | y | 0x7F7F7F7F7F7F7F7Full);
}

// The eight byte flags of eq_bytes as bits 0..7: after the shift, byte i's flag
// is bit 8i; the multiplier's byte j holds 2^(7-j), so the products land on
// distinct bits 8i + 7j + 7 (no carries) and i + j = 7 puts flag i at bit 56 + i.
__device__ __forceinline__ uint32_t pack8(uint64_t m) {
    return (uint32_t)(((m >> 7) * 0x0102040810204080ull) >> 56);
}

constexpr uint64_t kRep8 = 0x0101010101010101ull;

// Bit k: byte k of the 16 (lo: bytes 0-7, hi: 8-15) equals ch.
__device__ __forceinline__ uint32_t byte_mask16(uint64_t lo, uint64_t hi, uint8_t ch) {
    return pack8(eq_bytes(lo, kRep8 * ch)) | (pack8(eq_bytes(hi, kRep8 * ch)) << 8);
}

// The 16 bytes at p as two little-endian words (zero past the end).
__device__ __forceinline__ void load16w(const uint8_t* __restrict__ text, int64_t n, int64_t p, uint64_t* lo,
                                        uint64_t* hi) {
    if (p + kCPer <= n && ((reinterpret_cast<uintptr_t>(text + p) & 15) == 0)) {
        const uint4 v = *reinterpret_cast<const uint4*>(text + p);
        *lo = (uint64_t)v.x | ((uint64_t)v.y << 32);
        *hi = (uint64_t)v.z | ((uint64_t)v.w << 32);
    } else {
        uint64_t a = 0, b = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (p + k < n) a |= (uint64_t)text[p + k] << (8 * k);
            if (p + 8 + k < n) b |= (uint64_t)text[p + 8 + k] << (8 * k);
        }
        *lo = a;
        *hi = b;
    }
}

// Inclusive prefix XOR of a 16-bit mask: bit k = parity of bits 0..k.
__device__ __forceinline__ uint32_t prefix_xor16(uint32_t x) {
    x ^= x << 1;
    x ^= x << 2;
    x ^= x << 4;
    x ^= x << 8;
    return x & 0xFFFFu;
}

// One pass over the text, tile by tile (16 bytes per thread): the tile's
// quote parity, and the non-empty line ends outside quotes for both parities
// the tile may start with (it is known only after the scan of the parities).
// A line end is empty when the line is "" or "\r" after a line end; bytes
// before the text count as line ends.  Writes qpar, lcnt (start outside
// quotes), lcnt1 (inside) and each thread's two 16-bit end masks.
__global__ __launch_bounds__(kCTB) void k_csv_scan_text(const uint8_t* __restrict__ text, int64_t n, CsvWs w) {
    __shared__ uint32_t tmp[kCTB / kWave + 1];
    const int64_t tiles = w.scal[0];
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int64_t p0 = t * kCT + (int64_t)threadIdx.x * kCPer;
        uint64_t lo, hi;
        load16w(text, n, p0, &lo, &hi);
        const uint32_t qm = byte_mask16(lo, hi, '"');
        const uint32_t nm = byte_mask16(lo, hi, '\n');
        const uint32_t cm = byte_mask16(lo, hi, '\r');
        // bytes p0 - 2 and p0 - 1: the top two of the thread below (DPP wave
        // shift right by one); lane 0 reads them
        uint32_t prev = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(hi >> 48), 0x138, 0xF, 0xF, false);
        if (lane() == 0) {
            prev = 0x0A0Au;   // before the text: line ends
            if (p0 >= 2 && p0 - 1 < n) prev = (uint32_t)text[p0 - 2] | ((uint32_t)text[p0 - 1] << 8);
        }
        const uint32_t pn = ((prev & 0xFFu) == '\n' ? 1u : 0u) | ((prev >> 8) == '\n' ? 2u : 0u);
        const uint32_t pc = ((prev & 0xFFu) == '\r' ? 1u : 0u) | ((prev >> 8) == '\r' ? 2u : 0u);
        const uint32_t en = (nm << 2) | pn;   // bit k + 2: byte k is a line end
        const uint32_t ec = (cm << 2) | pc;
        const uint32_t empty = ((en >> 1) | ((ec >> 1) & en)) & 0xFFFFu;
        const uint32_t cand = nm & ~empty;   // bytes past the end are zero: no line ends
        uint32_t qt;
        const uint32_t qx = block_excl_sum<kCTB>((uint32_t)__popc(qm), tmp, &qt);
        const uint32_t inq = ((qx & 1u) ? 0xFFFFu : 0u) ^ prefix_xor16(qm);   // inside quotes, tile starting outside
        const uint32_t e0 = cand & ~inq, e1 = cand & inq;
        uint32_t ct;
        (void)block_excl_sum<kCTB>((uint32_t)__popc(e0) | ((uint32_t)__popc(e1) << 16), tmp, &ct);
        w.emask[t * kCTB + threadIdx.x] = e0 | (e1 << 16);
        if (threadIdx.x == 0) {
            w.qpar[t] = qt & 1u;
            w.lcnt[t] = ct & 0xFFFFu;
            w.lcnt1[t] = ct >> 16;
        }
    }
}

// Line ends of each tile for the parity it starts with.
__global__ void k_csv_pick(CsvWs w) {
    const int64_t tiles = w.scal[0];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tiles; t += (int64_t)gridDim.x * blockDim.x)
        if (w.qpre[t] & 1u) w.lcnt[t] = w.lcnt1[t];
}

// Positions of the line ends, from the end masks.
__global__ __launch_bounds__(kCTB) void k_csv_lines(CsvWs w) {
    __shared__ uint32_t tmp[kCTB / kWave + 1];
    const int64_t tiles = w.scal[0];
    const int64_t cap = w.scal[9];
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int64_t p0 = t * kCT + (int64_t)threadIdx.x * kCPer;
        const uint32_t m = w.emask[t * kCTB + threadIdx.x];
        uint32_t ends = (w.qpre[t] & 1u) ? (m >> 16) : (m & 0xFFFFu);
        uint32_t lt;
        int64_t r = w.loff[t] + block_excl_sum<kCTB>((uint32_t)__popc(ends), tmp, &lt);
        while (ends) {
            if (r < cap) w.line_end[r] = p0 + __builtin_ctz(ends);
            ++r;
            ends &= ends - 1;
        }
    }
}

// The last line when the text does not end with a line end, the data rows,
// capacity, and an open quoted run at the end (an error on the last row).
__global__ void k_csv_close(const uint8_t* __restrict__ text, int64_t n, CsvWs w, int has_header,
                            int64_t max_rows) {
    int64_t L = w.scal[1];
    const uint32_t par_end = w.scal[7] & 1;
    if (n > 0) {
        const uint8_t c1 = text[n - 1];
        const bool ends_on_newline = c1 == '\n' && par_end == 0;
        const bool only_cr = c1 == '\r' && (n == 1 || text[n - 2] == '\n') && par_end == 0;
        if (!ends_on_newline && !only_cr) {
            if (L < w.scal[9]) w.line_end[L] = n;
            ++L;
        }
    }
    const int64_t rows = L - ((has_header && L > 0) ? 1 : 0);
    w.scal[1] = L;
    w.scal[2] = rows;
    if (rows > max_rows) {
        w.scal[6] = 1;
        w.scal[2] = 0;   // nothing parsed
    } else if (par_end && rows > 0) {
        w.scal[3] = rows - 1;
    }
}

// ---- values ----

// Sequential reader of the text through one cached 16-byte chunk: aligned
// vector loads, except for the chunk that crosses the end of the text, which
// is read byte by byte (nothing past the text is touched).
struct Bytes {
    static constexpr bool kStaged = false;
    const uint8_t* t;
    int64_t n;
    int64_t chunk;
    uint64_t lo, hi;   // the cached chunk as two 64-bit halves (kept in registers)
    bool vec;
    __device__ __forceinline__ Bytes(const uint8_t* text, int64_t n_)
        : t(text), n(n_), chunk(-1), lo(0), hi(0), vec((reinterpret_cast<uintptr_t>(text) & 15) == 0) {}
    __device__ __forceinline__ uint8_t at(int64_t p) {
        const int64_t c = p >> 4;
        if (c != chunk) {
            chunk = c;
            const int64_t b = c << 4;
            if (vec && b + 16 <= n) {
                const uint4 v = *reinterpret_cast<const uint4*>(t + b);
                lo = (uint64_t)v.x | ((uint64_t)v.y << 32);
                hi = (uint64_t)v.z | ((uint64_t)v.w << 32);
            } else {
                uint64_t l = 0, h = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (b + k < n) l |= (uint64_t)t[b + k] << (8 * k);
                    if (b + 8 + k < n) h |= (uint64_t)t[b + 8 + k] << (8 * k);
                }
                lo = l;
                hi = h;
            }
        }
        const int o = (int)(p & 15);
        // a mask blend, not a select of the two halves: no address to index
        const uint64_t m = (uint64_t)0 - (uint64_t)(o >> 3);
        return (uint8_t)(((lo & ~m) | (hi & m)) >> (8 * (o & 7)));
    }
};

// Iterates the value bytes of a raw field (quoted runs unwrapped).
struct Unquote {
    Bytes B;   // its own copy of the reader: no reference to a local object
    int64_t i, e;
    bool in;
    __device__ __forceinline__ Unquote(const Bytes& bytes, int64_t b, int64_t end) : B(bytes), i(b), e(end), in(false) {}
    // next value byte into *c; false at the end
    __device__ __forceinline__ bool next(uint8_t* c) {
        while (i < e) {
            const uint8_t x = B.at(i++);
            if (x != '"') {
                *c = x;
                return true;
            }
            if (in && i < e && B.at(i) == '"') {
                ++i;
                *c = '"';
                return true;
            }
            in = !in;
        }
        return false;
    }
};

__device__ __forceinline__ bool same_value(const Bytes& B1, int64_t b1, int64_t e1, const Bytes& B2, int64_t b2, int64_t e2) {
    Unquote u1(B1, b1, e1), u2(B2, b2, e2);
    uint8_t c1, c2;
    for (;;) {
        const bool m1 = u1.next(&c1), m2 = u2.next(&c2);
        if (m1 != m2) return false;
        if (!m1) return true;
        if (c1 != c2) return false;
    }
}

// FNV-1a over the value bytes from a seeded basis, then a SplitMix64 finish.
constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull, kFnvPrime = 0x100000001b3ull;

__device__ __forceinline__ uint64_t finish_hash(uint64_t h, uint64_t seed, uint64_t mask) {
    h = splitmix64(seed, h) & mask;
    return h ? h : 1;
}

// ---- timestamps ----

// Days between 1970-01-01 and y-m-d (proleptic Gregorian), H. Hinnant's
// published days-from-civil algorithm: years counted from March so that
// February's leap day closes a year, 400-year eras of 146097 days.
__device__ __forceinline__ int64_t days_since_epoch(int64_t y, int64_t m, int64_t d) {
    const int64_t yy = m <= 2 ? y - 1 : y;
    const int64_t era = (yy >= 0 ? yy : yy - 399) / 400;
    const int64_t yoe = yy - era * 400;
    const int64_t mp = m > 2 ? m - 3 : m + 9;                  // months since March
    const int64_t doy = (153 * mp + 2) / 5 + d - 1;
    const int64_t doe = 365 * yoe + yoe / 4 - yoe / 100 + doy;
    return era * 146097 + doe - 719468;
}

__device__ __forceinline__ bool leap(int64_t y) { return (y % 4 == 0 && y % 100 != 0) || y % 400 == 0; }

__device__ __forceinline__ int month_days(int64_t y, int64_t m) {
    if (m == 2) return leap(y) ? 29 : 28;
    return (m == 4 || m == 6 || m == 9 || m == 11) ? 30 : 31;
}

// The value bytes of a raw field (quoted runs unwrapped) with one byte of
// lookahead: c is the current byte, -1 at the end.
template <class Src>
struct ValueCursor {
    Src B;   // its own copy of the reader: no reference to a local object
    int64_t i, e;
    bool in;
    int c;
    __device__ __forceinline__ ValueCursor(const Src& bytes, int64_t b, int64_t end)
        : B(bytes), i(b), e(end), in(false), c(-1) {
        adv();
    }
    __device__ __forceinline__ void adv() {
        while (i < e) {
            const uint8_t x = B.at(i++);
            if (x != '"') {
                c = x;
                return;
            }
            if (in && i < e && B.at(i) == '"') {
                ++i;
                c = '"';
                return;
            }
            in = !in;
        }
        c = -1;
    }
    __device__ __forceinline__ bool end() const { return c < 0; }
    __device__ __forceinline__ bool is(int ch) const { return c == ch; }
    __device__ __forceinline__ bool digit() const { return c >= '0' && c <= '9'; }
    __device__ __forceinline__ bool take(int ch) {
        if (c != ch) return false;
        adv();
        return true;
    }
    __device__ __forceinline__ bool digits(int k, int64_t* out) {
        int64_t x = 0;
        for (int j = 0; j < k; ++j) {
            if (!digit()) return false;
            x = x * 10 + (c - '0');
            adv();
        }
        *out = x;
        return true;
    }
};

// The bytes of a staged field that holds no quote character, with one byte
// of lookahead: the cursor of ValueCursor's interface without its unquoting.
struct PlainCursor {
    const uint8_t* s;   // the field's first byte in the stage
    int64_t i, e;       // offsets from s
    int c;
    __device__ __forceinline__ PlainCursor(const uint8_t* first, int64_t len) : s(first), i(0), e(len), c(-1) {
        adv();
    }
    __device__ __forceinline__ void adv() { c = i < e ? (int)s[i++] : -1; }
    __device__ __forceinline__ bool end() const { return c < 0; }
    __device__ __forceinline__ bool is(int ch) const { return c == ch; }
    __device__ __forceinline__ bool digit() const { return c >= '0' && c <= '9'; }
    __device__ __forceinline__ bool take(int ch) {
        if (c != ch) return false;
        adv();
        return true;
    }
    __device__ __forceinline__ bool digits(int k, int64_t* out) {
        int64_t x = 0;
        for (int j = 0; j < k; ++j) {
            if (!digit()) return false;
            x = x * 10 + (c - '0');
            adv();
        }
        *out = x;
        return true;
    }
};

template <class Cur>
__device__ __forceinline__ bool iso_value(Cur& c, int scale, int64_t* out) {
    int64_t y, mo, d, hh = 0, mi = 0, ss = 0, frac = 0, off = 0;
    if (!c.digits(4, &y) || !c.take('-') || !c.digits(2, &mo) || !c.take('-') || !c.digits(2, &d)) return false;
    if (mo < 1 || mo > 12 || d < 1 || d > month_days(y, mo)) return false;
    int nf = 0;
    if (c.is('T') || c.is(' ')) {
        c.adv();
        if (!c.digits(2, &hh) || !c.take(':') || !c.digits(2, &mi)) return false;
        if (c.take(':')) {
            if (!c.digits(2, &ss)) return false;
            if (c.is('.') || c.is(',')) {
                c.adv();
                while (c.digit()) {
                    if (nf == 9) return false;
                    if (nf < scale) frac = frac * 10 + (c.c - '0');
                    ++nf;
                    c.adv();
                }
                if (nf == 0) return false;
            }
        }
        if (hh > 23 || mi > 59 || ss > 59) return false;
        if (c.take('Z')) {
        } else if (c.is('+') || c.is('-')) {
            const int64_t sg = c.is('-') ? -1 : 1;
            c.adv();
            int64_t oh, om = 0;
            if (!c.digits(2, &oh)) return false;
            c.take(':');
            if (!c.end() && !c.digits(2, &om)) return false;
            if (oh > 23 || om > 59) return false;
            off = sg * (oh * 3600 + om * 60);
        }
    }
    if (!c.end()) return false;
    for (int k = nf < scale ? nf : scale; k < scale; ++k) frac *= 10;
    const int64_t secs = days_since_epoch(y, mo, d) * 86400 + hh * 3600 + mi * 60 + ss - off;
    __int128 p10 = 1;
    for (int k = 0; k < scale; ++k) p10 *= 10;
    const __int128 x = (__int128)secs * p10 + frac;   // must stay in int64
    if (x > (__int128)INT64_MAX || x < (__int128)INT64_MIN) return false;
    *out = (int64_t)x;
    return true;
}

template <class Cur>
__device__ __forceinline__ bool int_value(Cur& c, int64_t* out) {
    bool neg = false;
    if (c.is('+') || c.is('-')) {
        neg = c.is('-');
        c.adv();
    }
    if (c.end()) return false;
    uint64_t x = 0;
    const uint64_t lim = neg ? (uint64_t)INT64_MAX + 1 : (uint64_t)INT64_MAX;
    while (!c.end()) {
        if (!c.digit()) return false;
        const uint64_t dgt = (uint64_t)(c.c - '0');
        if (x > (lim - dgt) / 10) return false;
        x = x * 10 + dgt;
        c.adv();
    }
    *out = neg ? (int64_t)(0 - x) : (int64_t)x;
    return true;
}

__device__ __forceinline__ void flag_bad(const CsvWs& w, int64_t r) {
    atomicMin(reinterpret_cast<unsigned long long*>(&w.scal[3]), (unsigned long long)r);
}

// Eight bytes of the text from p: the two aligned words around them, funnel-
// shifted (both words end before p + 16, which the caller keeps <= n).
__device__ __forceinline__ uint64_t word_at(const uint8_t* __restrict__ text, int64_t p) {
    const int64_t a = p & ~(int64_t)7;
    const uint64_t* t64 = reinterpret_cast<const uint64_t*>(text + a);
    const int sh = (int)(p - a) * 8;
    const uint64_t lo = t64[0];
    if (sh == 0) return lo;
    const uint64_t hi = t64[1];
    return (lo >> sh) | (hi << (64 - sh));
}

// Raw fields [b1, b1 + len) and [b2, b2 + len) byte for byte, eight at a time
// (equal raw bytes are equal values; unequal ones may still be, by quoting).
__device__ __forceinline__ bool raw_equal(const uint8_t* __restrict__ text, int64_t n, int64_t b1, int64_t b2,
                                          int64_t len, bool aligned) {
    int64_t i = 0;
    if (aligned) {
        for (; i + 8 <= len && b1 + i + 16 <= n && b2 + i + 16 <= n; i += 8)
            if (word_at(text, b1 + i) != word_at(text, b2 + i)) return false;
    }
    for (; i < len; ++i)
        if (text[b1 + i] != text[b2 + i]) return false;
    return true;
}

// Slot of value hash h in table `tab` (linear probing); the slot keeps the
// smallest row that holds the value.  A slot is read before any atomic: a
// value already in the table (nearly every row) costs no atomic unless this
// row is smaller than the first row seen, so hot values (few activities over
// millions of rows) do not serialise on their slot.  Sets *claimed when this
// row's compare-and-swap took an empty slot (the value's first insert).
__device__ __forceinline__ uint32_t insert(CsvSlot* tab, int64_t tsize, uint64_t h, uint32_t r, bool* claimed) {
    uint64_t i = h & (uint64_t)(tsize - 1);
    for (;;) {   // the table has more slots than rows: an empty or equal slot exists
        unsigned long long cur = __hip_atomic_load(reinterpret_cast<unsigned long long*>(&tab[i].hash),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == 0) {
            cur = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[i].hash), 0ull, (unsigned long long)h);
            *claimed = cur == 0;
        }
        if (cur == 0 || cur == h) {
            if (r < __hip_atomic_load(&tab[i].first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMin(&tab[i].first, r);
            return (uint32_t)i;
        }
        i = (i + 1) & (uint64_t)(tsize - 1);
    }
}

// Both values of a row: when each is already at its home slot (the common
// case: the tables are at least twice the rows) the two lookups share their
// memory round trips; otherwise one insert after the other.
__device__ __forceinline__ void insert2(CsvSlot* t0, CsvSlot* t1, int64_t tsize, uint64_t h0, uint64_t h1,
                                        uint32_t r, bool* claimed, uint32_t* s0, uint32_t* s1) {
    const uint64_t i0 = h0 & (uint64_t)(tsize - 1), i1 = h1 & (uint64_t)(tsize - 1);
    const unsigned long long c0 = __hip_atomic_load(reinterpret_cast<unsigned long long*>(&t0[i0].hash),
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long c1 = __hip_atomic_load(reinterpret_cast<unsigned long long*>(&t1[i1].hash),
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (c0 == h0 && c1 == h1) {
        const uint32_t f0 = __hip_atomic_load(&t0[i0].first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t f1 = __hip_atomic_load(&t1[i1].first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (r < f0) atomicMin(&t0[i0].first, r);
        if (r < f1) atomicMin(&t1[i1].first, r);
        *s0 = (uint32_t)i0;
        *s1 = (uint32_t)i1;
        return;
    }
    *s0 = insert(t0, tsize, h0, r, &claimed[0]);
    *s1 = insert(t1, tsize, h1, r, &claimed[1]);
}

// Bytes of the text already staged in LDS: [lo, lo + len) at stage[0..).
struct StagedBytes {
    static constexpr bool kStaged = true;
    const uint8_t* stage;
    int64_t lo;
    __device__ __forceinline__ uint8_t at(int64_t p) const { return stage[p - lo]; }
};

// Hash of a value: its bytes packed little-endian into 64-bit words (the last
// one zero-padded), each folded in by xor and multiply, then the length and a
// SplitMix64 finish.  Fed a byte at a time (quoted values, unwrapped) or a
// word at a time (values without quotes): the same bytes give the same hash.
struct ValueHash {
    uint64_t h, acc;
    uint32_t n;
    __device__ __forceinline__ explicit ValueHash(uint64_t seed) : h(kFnvBasis ^ seed), acc(0), n(0) {}
    __device__ __forceinline__ void byte(uint8_t x) {
        acc |= (uint64_t)x << (8 * (n & 7));
        if ((++n & 7) == 0) {
            h = (h ^ acc) * kFnvPrime;
            acc = 0;
        }
    }
    __device__ __forceinline__ void word(uint64_t x) {   // eight bytes; n is a multiple of 8
        h = (h ^ x) * kFnvPrime;
        n += 8;
    }
    __device__ __forceinline__ uint64_t done(uint64_t seed, uint64_t mask) {
        if (n & 7) h = (h ^ acc) * kFnvPrime;
        return finish_hash(h ^ (uint64_t)n, seed, mask);
    }
};

// Eight staged bytes from stage offset o: the two aligned words around them,
// funnel-shifted (the stage keeps 16 bytes of room past its capacity).
__device__ __forceinline__ uint64_t stage_word(const uint8_t* stage, int64_t o) {
    const int64_t a = o & ~(int64_t)7;
    const uint64_t* s64 = reinterpret_cast<const uint64_t*>(stage + a);
    const int sh = (int)(o - a) * 8;
    const uint64_t lo = s64[0];
    return sh ? ((lo >> sh) | (s64[1] << (64 - sh))) : lo;
}

// 0x80 in each byte of x equal to the byte repeated in c8, 0 elsewhere.

// A staged row with no quote character, eight bytes at a time: separators
// from byte masks, the case and activity values hashed a word at a time.
// Fills the field ranges and hashes the byte walk would; false (nothing
// written) when the row holds a quote.
__device__ __forceinline__ bool split_fast(const uint8_t* stage, int64_t lo, int64_t a, int64_t e,
                                           const pm4g_csv_schema& sc, int32_t need, uint64_t seed, uint64_t mask,
                                           int64_t* fr, int32_t* nf, uint64_t* hc, uint64_t* ha) {
    const uint64_t sep8 = 0x0101010101010101ull * (uint8_t)sc.sep;
    const uint64_t quo8 = 0x0101010101010101ull * (uint8_t)'"';
    for (int64_t p = a; p < e; p += 8)
        if (eq_bytes(stage_word(stage, p - lo), quo8) & (e - p >= 8 ? ~0ull : ((1ull << (8 * (e - p))) - 1)))
            return false;
    int32_t f = 0;
    int64_t fs = a;
    for (int64_t p = a; p < e && f <= need; p += 8) {
        uint64_t sm = eq_bytes(stage_word(stage, p - lo), sep8) & (e - p >= 8 ? ~0ull : ((1ull << (8 * (e - p))) - 1));
        while (sm && f <= need) {
            const int64_t i = p + (__builtin_ctzll(sm) >> 3);
            if (f == sc.case_col) { fr[0] = fs; fr[1] = i; }
            if (f == sc.act_col) { fr[2] = fs; fr[3] = i; }
            if (f == sc.ts_col) { fr[4] = fs; fr[5] = i; }
            ++f;
            fs = i + 1;
            sm &= sm - 1;
        }
    }
    if (f <= need) {   // the end of the line closes the last field
        if (f == sc.case_col) { fr[0] = fs; fr[1] = e; }
        if (f == sc.act_col) { fr[2] = fs; fr[3] = e; }
        if (f == sc.ts_col) { fr[4] = fs; fr[5] = e; }
        ++f;
    }
    *nf = f;
    if (f <= need) return true;
    for (int k = 0; k < 2; ++k) {
        const int64_t b = fr[2 * k], en = fr[2 * k + 1];
        ValueHash hv(seed);
        int64_t p = b;
        for (; p + 8 <= en; p += 8) hv.word(stage_word(stage, p - lo));
        for (; p < en; ++p) hv.byte(stage[p - lo]);
        (k == 0 ? *hc : *ha) = hv.done(seed, mask);
    }
    return true;
}

// One walk over row r: fields split at separators outside quoted runs; the
// case and activity values are hashed and the timestamp value copied as the
// walk unwraps their runs (a doubled quote inside a run is one quote and
// leaves the run open, as two toggles would).  A staged row without quotes
// takes split_fast instead of the byte walk.
template <class Src>
__device__ __forceinline__ void parse_row(Src B, int64_t r, int64_t a, int64_t e, const CsvWs w,
                                         const pm4g_csv_schema& sc, int32_t need, uint64_t seed, uint64_t mask,
                                         int64_t* __restrict__ ts_out, bool* claimed) {
    const uint8_t sep = (uint8_t)sc.sep;
    // skip the empty lines in between ("\n" or "\r\n" each)
    while (a < e && (B.at(a) == '\n' || (B.at(a) == '\r' && a + 1 < e && B.at(a + 1) == '\n'))) ++a;
    if (e > a && B.at(e - 1) == '\r') --e;
    int64_t cb = -1, ce = -1, ab = -1, ae = -1, tb = -1, te = -1;
    int32_t f = 0;
    uint64_t hc = 0, ha = 0;
    bool fast = false;
    if constexpr (Src::kStaged) {
        int64_t fr[6] = {-1, -1, -1, -1, -1, -1};
        fast = split_fast(B.stage, B.lo, a, e, sc, need, seed, mask, fr, &f, &hc, &ha);
        if (fast) {
            cb = fr[0]; ce = fr[1]; ab = fr[2]; ae = fr[3]; tb = fr[4]; te = fr[5];
        }
    }
    if (!fast) {
    ValueHash h0(seed), h1(seed);
    bool q = false;
    int64_t fs = a;
    for (int64_t i = a; i <= e; ++i) {
        if (i < e) {
            uint8_t x = B.at(i);
            bool lit = false;
            if (x == '"') {
                if (q && i + 1 < e && B.at(i + 1) == '"') {
                    ++i;   // a doubled quote inside a run: one quote, still in the run
                    lit = true;
                } else {
                    q = !q;
                    continue;
                }
            }
            if (lit || x != sep || q) {
                if (f == sc.case_col) h0.byte(x);
                if (f == sc.act_col) h1.byte(x);
                continue;
            }
        }
        // a separator outside quotes, or the end of the line, closes field f
        if (f == sc.case_col) { cb = fs; ce = i; }
        if (f == sc.act_col) { ab = fs; ae = i; }
        if (f == sc.ts_col) { tb = fs; te = i; }
        ++f;
        fs = i + 1;
    }
    hc = h0.done(seed, mask);
    ha = h1.done(seed, mask);
    }
    if (f <= need) {
        flag_bad(w, r);
        w.slot[2 * r] = w.slot[2 * r + 1] = 0;
        return;
    }
    w.foff[2 * r] = cb;
    w.flen[2 * r] = (int32_t)(ce - cb);
    w.foff[2 * r + 1] = ab;
    w.flen[2 * r + 1] = (int32_t)(ae - ab);
    uint32_t s0, s1;
    insert2(w.table, w.table + w.tsize, w.tsize, hc, ha, (uint32_t)r, claimed, &s0, &s1);
    w.slot[2 * r] = s0;
    w.slot[2 * r + 1] = s1;
    bool ok = te - tb <= kTsMax;
    if (ok) {
        int64_t t;
        if constexpr (Src::kStaged) {
            if (fast) {   // no quote in the row: the field's bytes are its value
                PlainCursor pc(B.stage + (tb - B.lo), te - tb);
                ok = sc.ts_iso ? iso_value(pc, sc.ts_scale, &t) : int_value(pc, &t);
            } else {
                ValueCursor<Src> vc(B, tb, te);
                ok = sc.ts_iso ? iso_value(vc, sc.ts_scale, &t) : int_value(vc, &t);
            }
        } else {
            ValueCursor<Src> vc(B, tb, te);
            ok = sc.ts_iso ? iso_value(vc, sc.ts_scale, &t) : int_value(vc, &t);
        }
        if (ok) ts_out[r] = t;
    }
    if (!ok) flag_bad(w, r);
}

constexpr int kStage = 32768;   // bytes of text staged per block of rows

// A block takes 256 consecutive rows; their bytes (one contiguous range) are
// copied to LDS with coalesced 16-byte loads and walked there; a range longer
// than the stage is walked through the chunk reader instead.
__global__ __launch_bounds__(256) void k_csv_parse(const uint8_t* __restrict__ text, int64_t n_bytes, CsvWs w,
                                                   pm4g_csv_schema sc, uint64_t seed, uint64_t mask,
                                                   int64_t* __restrict__ ts_out) {
    __shared__ uint4 stage4[kStage / 16 + 1];   // + 16 bytes of room for the word reads
    __shared__ uint32_t s_new[2][256];   // slots this block's rows claimed, per table
    __shared__ uint32_t s_cnt[2];
    __shared__ int64_t s_base[2];
    uint8_t* stage = reinterpret_cast<uint8_t*>(stage4);
    const int64_t rows = w.scal[2];
    const int64_t hdr = (sc.has_header && w.scal[1] > 0) ? 1 : 0;
    const int32_t need = sc.case_col > sc.act_col ? (sc.case_col > sc.ts_col ? sc.case_col : sc.ts_col)
                                                   : (sc.act_col > sc.ts_col ? sc.act_col : sc.ts_col);
    const bool vec = (reinterpret_cast<uintptr_t>(text) & 15) == 0;
    for (int64_t r0 = (int64_t)blockIdx.x * 256; r0 < rows; r0 += (int64_t)gridDim.x * 256) {
        if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
        const int64_t rl = (r0 + 255 < rows ? r0 + 255 : rows - 1);
        const int64_t li0 = r0 + hdr, lil = rl + hdr;
        const int64_t lo = (li0 == 0 ? 0 : w.line_end[li0 - 1] + 1) & ~(int64_t)15;
        const int64_t hi = w.line_end[lil];   // bytes [lo, hi) hold the rows
        const bool staged = hi - lo <= kStage;   // block-uniform
        if (staged) {
            for (int64_t off = (int64_t)threadIdx.x * 16; off < hi - lo; off += 256 * 16) {
                const int64_t p = lo + off;
                if (vec && p + 16 <= n_bytes) {
                    stage4[off >> 4] = *reinterpret_cast<const uint4*>(text + p);
                } else {
                    for (int k = 0; k < 16; ++k) stage[off + k] = p + k < n_bytes ? text[p + k] : 0;
                }
            }
        }
        __syncthreads();
        const int64_t r = r0 + threadIdx.x;
        bool claimed[2] = {false, false};
        if (r < rows) {
            const int64_t li = r + hdr;
            const int64_t a = li == 0 ? 0 : w.line_end[li - 1] + 1;
            const int64_t e = w.line_end[li];
            if (staged) {
                StagedBytes SB{stage, lo};
                parse_row(SB, r, a, e, w, sc, need, seed, mask, ts_out, claimed);
            } else {
                Bytes B(text, n_bytes);
                parse_row(B, r, a, e, w, sc, need, seed, mask, ts_out, claimed);
            }
        }
        // list the claimed slots: one global reservation per table and block pass
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (claimed[k]) s_new[k][atomicAdd(&s_cnt[k], 1u)] = w.slot[2 * r + k];
        __syncthreads();
        if (threadIdx.x < 2)
            s_base[threadIdx.x] = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(&w.scal[10 + threadIdx.x]),
                                                     (unsigned long long)s_cnt[threadIdx.x]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; ++k)
            for (uint32_t j = threadIdx.x; j < s_cnt[k]; j += 256) w.dlist[k * w.max_rows + s_base[k] + j] = s_new[k][j];
        __syncthreads();
    }
}

// Every row's value against its slot's first row, byte by byte: equal values,
// or a hash collision (scal[4]: the call is repeated with another seed).  A
// thread takes two rows per step, and the four (row, field) items go through
// each stage together (slot, first row, field ranges, first 16 bytes) so that
// their loads are in flight at once; longer or unequal fields take the
// general comparison.
__global__ __launch_bounds__(256) void k_csv_verify(const uint8_t* __restrict__ text, int64_t n_bytes, CsvWs w) {
    const int64_t rows = w.scal[2];
    if (w.scal[3] != INT64_MAX) return;   // a parse error ends the call
    const bool aligned = (reinterpret_cast<uintptr_t>(text) & 7) == 0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    constexpr int kJ = 4;   // two rows x two fields
    for (int64_t r0 = (int64_t)blockIdx.x * 256 + threadIdx.x; r0 < rows; r0 += 2 * stride) {
        int64_t row[kJ];
        uint32_t sl[kJ], first[kJ];
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            row[j] = r0 + (j >> 1) * stride;
            sl[j] = row[j] < rows ? w.slot[2 * row[j] + (j & 1)] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kJ; ++j)
            first[j] = row[j] < rows ? w.table[(j & 1) * w.tsize + sl[j]].first : (uint32_t)row[j];
        bool need[kJ];
        int64_t b1[kJ], b2[kJ];
        int32_t l1[kJ], l2[kJ];
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            need[j] = row[j] < rows && first[j] != (uint32_t)row[j];
            const int64_t r = need[j] ? row[j] : 0, f = need[j] ? (int64_t)first[j] : 0;
            b1[j] = w.foff[2 * r + (j & 1)];
            l1[j] = w.flen[2 * r + (j & 1)];
            b2[j] = w.foff[2 * f + (j & 1)];
            l2[j] = w.flen[2 * f + (j & 1)];
        }
        // fields of at most 16 bytes whose aligned words lie inside the text
        bool quick[kJ];
        uint64_t x0[kJ], x1[kJ], y0[kJ], y1[kJ];
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            quick[j] = need[j] && aligned && l1[j] == l2[j] && l1[j] <= 16 && b1[j] + 24 <= n_bytes &&
                       b2[j] + 24 <= n_bytes;
            x0[j] = x1[j] = y0[j] = y1[j] = 0;
            if (quick[j]) {
                x0[j] = word_at(text, b1[j]);
                x1[j] = word_at(text, b1[j] + 8);
                y0[j] = word_at(text, b2[j]);
                y1[j] = word_at(text, b2[j] + 8);
            }
        }
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            if (!need[j]) continue;
            if (quick[j]) {
                const int L = l1[j];
                const uint64_t m0 = L >= 8 ? ~0ull : ((1ull << (8 * L)) - 1);
                const uint64_t m1 = L >= 16 ? ~0ull : (L <= 8 ? 0ull : ((1ull << (8 * (L - 8))) - 1));
                if (((x0[j] ^ y0[j]) & m0) == 0 && ((x1[j] ^ y1[j]) & m1) == 0) continue;
            } else if (l1[j] == l2[j] && raw_equal(text, n_bytes, b1[j], b2[j], l1[j], aligned)) {
                continue;
            }
            Bytes B1(text, n_bytes), B2(text, n_bytes);
            if (!same_value(B1, b1[j], b1[j] + l1[j], B2, b2[j], b2[j] + l2[j])) w.scal[4] = 1;
        }
    }
}

// The slots listed for table k with their first rows, to sort; their number
// goes to scal[5] (none after a capacity or parse error or a collision).
__global__ __launch_bounds__(256) void k_csv_gather(CsvWs w, int k) {
    const bool failed = w.scal[6] != 0 || w.scal[3] != INT64_MAX || w.scal[4] != 0;
    const int64_t D = failed ? 0 : w.scal[10 + k];
    if (blockIdx.x == 0 && threadIdx.x == 0) w.scal[5] = D;
    const uint32_t* dl = w.dlist + k * w.max_rows;
    const CsvSlot* tab = w.table + k * w.tsize;
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < D; d += (int64_t)gridDim.x * 256) {
        const uint32_t i = dl[d];
        w.k0[d] = tab[i].first;
        w.v0[d] = i;
    }
}

// Sorted by first row: the code of a slot is its rank.
__global__ __launch_bounds__(256) void k_csv_codes(CsvWs w, int k, const uint32_t* __restrict__ key,
                                                   const uint32_t* __restrict__ val, int64_t* __restrict__ dict_off,
                                                   int32_t* __restrict__ dict_len, int64_t* n_dict) {
    CsvSlot* tab = w.table + k * w.tsize;
    const int64_t D = w.scal[5];
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < D; d += (int64_t)gridDim.x * 256) {
        tab[val[d]].code = (uint32_t)d;
        const int64_t r = key[d];
        dict_off[d] = w.foff[2 * r + k];
        dict_len[d] = w.flen[2 * r + k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_dict = D;
}

__global__ __launch_bounds__(256) void k_csv_emit(CsvWs w, int32_t* __restrict__ case_code,
                                                  int32_t* __restrict__ act_code) {
    if (w.scal[6] != 0 || w.scal[3] != INT64_MAX || w.scal[4] != 0) return;
    const int64_t rows = w.scal[2];
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < rows; r += (int64_t)gridDim.x * 256) {
        case_code[r] = (int32_t)w.table[w.slot[2 * r]].code;
        act_code[r] = (int32_t)w.table[w.tsize + w.slot[2 * r + 1]].code;
    }
}

__global__ void k_csv_finish(CsvWs w, int64_t* n_rows, int32_t* status, int64_t* bad_row) {
    const bool over = w.scal[6] != 0, bad = w.scal[3] != INT64_MAX;
    *n_rows = (over || bad) ? 0 : w.scal[2];
    *bad_row = bad ? w.scal[3] : -1;
    *status = over ? PM4G_E_CAPACITY : (bad ? PM4G_E_PARSE : 0);
}

unsigned grid_rows(int64_t rows) {
    const int64_t g = (rows + 255) / 256;
    return (unsigned)(g < 2048 ? (g < 1 ? 1 : g) : 2048);
}

}  // namespace

hipError_t launch_csv_lines(const uint8_t* text, int64_t n_bytes, int has_header, int64_t max_rows, CsvWs w,
                            hipStream_t s) {
    const int64_t tiles = (n_bytes + kCT - 1) / kCT;
    const unsigned gt = (unsigned)(tiles < 2048 ? (tiles < 1 ? 1 : tiles) : 2048);
    k_csv_init<<<1, 1, 0, s>>>(w, n_bytes, max_rows + 1);
    k_csv_scan_text<<<gt, kCTB, 0, s>>>(text, n_bytes, w);
    dev::excl_scan<uint32_t>(w.qpar, &w.scal[0], w.qpre, w.part32, reinterpret_cast<uint32_t*>(&w.scal[7]), s);
    k_csv_pick<<<(unsigned)((tiles + 255) / 256 < 1024 ? ((tiles + 255) / 256 < 1 ? 1 : (tiles + 255) / 256) : 1024),
                 256, 0, s>>>(w);
    dev::excl_scan<int64_t>(w.lcnt, &w.scal[0], w.loff, w.part64, &w.scal[1], s);
    k_csv_lines<<<gt, kCTB, 0, s>>>(w);
    k_csv_close<<<1, 1, 0, s>>>(text, n_bytes, w, has_header, max_rows);
    return hipGetLastError();
}

hipError_t launch_csv_parse(const uint8_t* text, int64_t n_bytes, const pm4g_csv_schema& sc, uint64_t seed,
                            int hash_bits, int64_t max_rows, CsvWs w, const pm4g_csv_out& o, hipStream_t s) {
    const uint64_t mask = (hash_bits <= 0 || hash_bits >= 64) ? ~0ull : ((1ull << hash_bits) - 1);
    const unsigned gr = grid_rows(max_rows);
    k_csv_clear<<<2048, 256, 0, s>>>(w);
    k_csv_parse<<<gr, 256, 0, s>>>(text, n_bytes, w, sc, seed, mask, o.ts);
    k_csv_verify<<<gr, 256, 0, s>>>(text, n_bytes, w);
    return hipGetLastError();
}

hipError_t launch_csv_codes(CsvWs w, int64_t max_rows, const pm4g_csv_out& o, hipStream_t s) {
    int bits = 8;   // first rows are below max_rows: sort on that many bits
    while (bits < 32 && (int64_t(1) << bits) < max_rows) bits += 8;
    for (int k = 0; k < 2; ++k) {
        k_csv_gather<<<grid_rows(max_rows), 256, 0, s>>>(w, k);
        const bool flip = dev::sort_pairs<uint32_t>(w.k0, w.v0, w.k1, w.v1, &w.scal[5], max_rows, bits, w.hist,
                                                    w.rowsum, s);
        const uint32_t* key = flip ? w.k1 : w.k0;
        const uint32_t* val = flip ? w.v1 : w.v0;
        k_csv_codes<<<grid_rows(max_rows), 256, 0, s>>>(w, k, key, val, k == 0 ? o.case_dict_off : o.act_dict_off,
                                                        k == 0 ? o.case_dict_len : o.act_dict_len,
                                                        k == 0 ? o.n_cases : o.n_acts);
    }
    k_csv_emit<<<grid_rows(max_rows), 256, 0, s>>>(w, o.case_code, o.act_code);
    return hipGetLastError();
}

hipError_t launch_csv_finish(CsvWs w, const pm4g_csv_out& o, hipStream_t s) {
    k_csv_finish<<<1, 1, 0, s>>>(w, o.n_rows, o.status, o.bad_row);
    return hipGetLastError();
}

}  // namespace pm4g
