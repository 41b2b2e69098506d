// Parquet ingestion into the columns of an event log (Sec. 2.2: the log may
// be held as a columnar Parquet file, which the GPU dataframe library reads
// without going through rows).
//
// The file format is Apache Parquet's published specification: the file ends
// with its metadata (a Thrift compact-protocol struct), a 4-byte
// little-endian length and "PAR1"; every column of every row group is a
// chunk of pages, each a Thrift page header followed by the page's bytes.
// Covered: uncompressed chunks, flat schemas, data pages v1 and v2, PLAIN and
// dictionary-coded values (dictionary pages PLAIN), definition levels of
// optional columns (a null in a used column is an error at its row); INT32,
// INT64 and BYTE_ARRAY case and activity columns, INT32 and INT64 timestamps.
//
// Work:
//   host            reads the footer (one small copy), parses the metadata,
//                   lists the three columns' chunks with their first row
//   k_pq_decode     one block per chunk walks its pages in order: thread 0
//                   reads each page header (and the run headers of its RLE /
//                   bit-packed hybrid streams); the block decodes the values
//                   of the page in parallel: dictionaries into a per-chunk
//                   table, data values into per-row arrays (an integer, or the
//                   byte range of a byte array in the file)
//   k_pq_match      per row and column: a 64-bit hash of the value into an
//                   open-addressing table keyed by hash, each slot keeping the
//                   smallest row holding it; every row is then compared with
//                   its slot's first row (a hash collision repeats the
//                   matching with another seed)
//   codes           used slots sorted by first row: the code is the rank
//                   (first-appearance order), as for CSV ingestion
#include <string.h>

#include <vector>

#include "common.hpp"
#include "devsort.hpp"
#include "internal.hpp"
#include "prof.hpp"
#include "../../include/pm4g.h"

namespace pm4g {

// ---- host: the footer -------------------------------------------------------

namespace {

// Thrift compact protocol over host bytes.
class CompactIn {
  public:
    CompactIn(const uint8_t* b, int64_t n) : b_(b), n_(n) {}
    bool bad() const { return bad_; }
    uint8_t byte() {
        if (p_ >= n_) {
            bad_ = true;
            return 0;
        }
        return b_[p_++];
    }
    uint64_t uvar() {
        uint64_t v = 0;
        for (int s = 0; s < 64; s += 7) {
            const uint8_t c = byte();
            if (bad_) return 0;
            v |= (uint64_t)(c & 0x7f) << s;
            if ((c & 0x80) == 0) return v;
        }
        bad_ = true;
        return 0;
    }
    int64_t svar() {
        const uint64_t u = uvar();
        return (int64_t)(u >> 1) ^ -(int64_t)(u & 1);
    }
    // next field of the current struct: its compact type (0 at the end)
    int field(int& id) {
        const uint8_t h = byte();
        const int t = h & 15;
        if (t == 0 || bad_) return 0;
        const int delta = h >> 4;
        id = delta ? last_.back() + delta : (int)svar();
        last_.back() = id;
        return t;
    }
    void enter() { last_.push_back(0); }
    void leave() { last_.pop_back(); }
    // a list or set header: element count, element type
    int64_t list(int& et) {
        const uint8_t h = byte();
        uint64_t n = h >> 4;
        if (n == 15) n = uvar();
        et = h & 15;
        if (n > (uint64_t)n_) bad_ = true;
        return bad_ ? 0 : (int64_t)n;
    }
    void skip(int t, bool element = false, int depth = 0) {
        if (depth > 64) {
            bad_ = true;
            return;
        }
        switch (t) {
            case 1:
            case 2:
                if (element) byte();
                break;
            case 3: byte(); break;
            case 4:
            case 5:
            case 6: uvar(); break;
            case 7: p_ += 8; break;
            case 8: {
                const uint64_t len = uvar();
                if (len > (uint64_t)(n_ - p_)) bad_ = true;
                else p_ += (int64_t)len;
                break;
            }
            case 9:
            case 10: {
                int et;
                const int64_t cnt = list(et);
                for (int64_t k = 0; k < cnt && !bad_; ++k) skip(et, true, depth + 1);
                break;
            }
            case 11: {
                const uint64_t cnt = uvar();
                if (cnt) {
                    const uint8_t kv = byte();
                    for (uint64_t k = 0; k < cnt && !bad_; ++k) {
                        skip(kv >> 4, true, depth + 1);
                        skip(kv & 15, true, depth + 1);
                    }
                }
                break;
            }
            case 12: {
                enter();
                int id, ft;
                while ((ft = field(id)) != 0 && !bad_) skip(ft, false, depth + 1);
                leave();
                break;
            }
            default: bad_ = true;
        }
        if (p_ > n_) bad_ = true;
    }

  private:
    const uint8_t* b_;
    int64_t n_, p_ = 0;
    bool bad_ = false;
    std::vector<int> last_{0};
};

struct LeafCol {
    int32_t type = -1, repetition = 0;
    bool nested = false;
};

struct ChunkMeta {
    int32_t type = -1, codec = -1;
    int64_t num_values = -1, size = -1, data_off = -1, dict_off = -1;
    bool external = false;
};

}  // namespace

int pq_parse_footer(const uint8_t* meta, int64_t len, int64_t file_bytes, const int32_t cols[3],
                    std::vector<PqChunk>* chunks, int64_t* rows, char* msg, size_t msg_len) {
    CompactIn in(meta, len);
    std::vector<LeafCol> leaves;
    std::vector<int64_t> rg_rows;
    std::vector<ChunkMeta> picked;   // [row group][3]
    int64_t num_rows = -1;
    bool nested = false, external = false;
    int id, ft;
    while ((ft = in.field(id)) != 0 && !in.bad()) {
        if (id == 2 && ft == 9) {   // schema: the root, then the leaves of a flat schema
            int et;
            const int64_t n = in.list(et);
            for (int64_t e = 0; e < n && !in.bad(); ++e) {
                LeafCol c;
                in.enter();
                int i2, t2;
                while ((t2 = in.field(i2)) != 0 && !in.bad()) {
                    if (i2 == 1 && t2 == 5) c.type = (int32_t)in.svar();
                    else if (i2 == 3 && t2 == 5) c.repetition = (int32_t)in.svar();
                    else if (i2 == 5 && t2 == 5) c.nested = in.svar() > 0;
                    else in.skip(t2);
                }
                in.leave();
                if (e == 0) continue;
                nested |= c.nested;
                leaves.push_back(c);
            }
        } else if (id == 3 && ft == 6) {
            num_rows = in.svar();
        } else if (id == 4 && ft == 9) {   // row groups
            int et;
            const int64_t n = in.list(et);
            for (int64_t g = 0; g < n && !in.bad(); ++g) {
                int64_t r = -1;
                ChunkMeta mine[3];
                in.enter();
                int i2, t2;
                while ((t2 = in.field(i2)) != 0 && !in.bad()) {
                    if (i2 == 3 && t2 == 6) {
                        r = in.svar();
                    } else if (i2 == 1 && t2 == 9) {   // column chunks
                        int ct;
                        const int64_t nc = in.list(ct);
                        for (int64_t c = 0; c < nc && !in.bad(); ++c) {
                            ChunkMeta cm;
                            in.enter();
                            int i3, t3;
                            while ((t3 = in.field(i3)) != 0 && !in.bad()) {
                                if (i3 == 1 && t3 == 8) {
                                    cm.external = true;
                                    in.skip(t3);
                                } else if (i3 == 3 && t3 == 12) {   // column metadata
                                    in.enter();
                                    int i4, t4;
                                    while ((t4 = in.field(i4)) != 0 && !in.bad()) {
                                        if (i4 == 1 && t4 == 5) cm.type = (int32_t)in.svar();
                                        else if (i4 == 4 && t4 == 5) cm.codec = (int32_t)in.svar();
                                        else if (i4 == 5 && t4 == 6) cm.num_values = in.svar();
                                        else if (i4 == 7 && t4 == 6) cm.size = in.svar();
                                        else if (i4 == 9 && t4 == 6) cm.data_off = in.svar();
                                        else if (i4 == 11 && t4 == 6) cm.dict_off = in.svar();
                                        else in.skip(t4);
                                    }
                                    in.leave();
                                } else {
                                    in.skip(t3);
                                }
                            }
                            in.leave();
                            for (int k = 0; k < 3; ++k)
                                if (c == cols[k]) mine[k] = cm;
                        }
                    } else {
                        in.skip(t2);
                    }
                }
                in.leave();
                rg_rows.push_back(r);
                for (int k = 0; k < 3; ++k) {
                    picked.push_back(mine[k]);
                    external |= mine[k].external;
                }
            }
        } else {
            in.skip(ft);
        }
    }
    if (in.bad() || num_rows < 0 || leaves.empty()) {
        snprintf(msg, msg_len, "malformed Parquet metadata");
        return PM4G_E_PARSE;
    }
    *rows = num_rows;   // the file's row count, whatever the columns asked for
    if (nested || external) {
        snprintf(msg, msg_len, "%s", nested ? "nested Parquet schemas are not read" : "column chunks in other files");
        return PM4G_E_UNSUPPORTED;
    }
    for (int k = 0; k < 3; ++k) {
        if (cols[k] >= (int32_t)leaves.size()) {
            snprintf(msg, msg_len, "column %d: the file has %zu columns", cols[k], leaves.size());
            return PM4G_E_INVALID;
        }
        const LeafCol& c = leaves[cols[k]];
        const bool ok_type = k < 2 ? (c.type == 1 || c.type == 2 || c.type == 6) : (c.type == 1 || c.type == 2);
        if (!ok_type || c.repetition == 2) {
            snprintf(msg, msg_len, "column %d: physical type %d%s is not read", cols[k], c.type,
                     c.repetition == 2 ? " (repeated)" : "");
            return PM4G_E_UNSUPPORTED;
        }
    }
    int64_t total = 0, dict_base = 0;
    chunks->clear();
    for (size_t g = 0; g < rg_rows.size(); ++g) {
        if (rg_rows[g] < 0) {
            snprintf(msg, msg_len, "malformed Parquet metadata");
            return PM4G_E_PARSE;
        }
        for (int k = 0; k < 3; ++k) {
            const ChunkMeta& cm = picked[g * 3 + k];
            const LeafCol& c = leaves[cols[k]];
            if (cm.type < 0 || cm.type != c.type || cm.num_values < 0 || cm.size < 0) {
                snprintf(msg, msg_len, "malformed Parquet column chunk");
                return PM4G_E_PARSE;
            }
            if (cm.codec != 0) {
                snprintf(msg, msg_len, "compressed column chunks (codec %d) are not read", cm.codec);
                return PM4G_E_UNSUPPORTED;
            }
            if (cm.num_values != rg_rows[g]) {
                snprintf(msg, msg_len, "a column chunk's values differ from its rows");
                return PM4G_E_UNSUPPORTED;
            }
            if (cm.num_values == 0) continue;
            PqChunk ch{};
            ch.start = (cm.dict_off > 0 && (cm.dict_off < cm.data_off || cm.data_off <= 0)) ? cm.dict_off : cm.data_off;
            ch.end = ch.start + cm.size;
            if (ch.start < 4 || cm.size > file_bytes - 8 - ch.start) {
                snprintf(msg, msg_len, "a column chunk lies outside the file");
                return PM4G_E_PARSE;
            }
            ch.num_values = cm.num_values;
            ch.row0 = total;
            ch.dict_base = dict_base;
            ch.type = cm.type;
            ch.optional = c.repetition == 1;
            ch.col = k;
            dict_base += cm.num_values;
            chunks->push_back(ch);
        }
        total += rg_rows[g];
    }
    if (total != num_rows) {
        snprintf(msg, msg_len, "row groups hold %lld rows, the file %lld", (long long)total, (long long)num_rows);
        return PM4G_E_PARSE;
    }
    *rows = total;
    return PM4G_OK;
}

PqWs pq_ws_layout(Bump& b, int64_t max_rows) {
    PqWs w{};
    const size_t rows = (size_t)(max_rows > 0 ? max_rows : 1);
    int64_t t = 1024;
    while (t < 2 * (int64_t)rows) t <<= 1;
    w.tsize = t;
    w.scal = b.take<int64_t>(16);
    w.chunks = b.take<PqChunk>((size_t)kPqMaxChunks);
    w.dict_a = b.take<int64_t>(3 * rows);
    w.dict_b = b.take<int32_t>(3 * rows);
    w.val_a = b.take<int64_t>(2 * rows);
    w.val_b = b.take<int32_t>(2 * rows);
    w.slot = b.take<uint32_t>(2 * rows);
    w.table = b.take<CsvSlot>((size_t)(2 * w.tsize));
    w.used = b.take<uint32_t>((size_t)w.tsize);
    w.pos = b.take<uint32_t>((size_t)w.tsize);
    w.k0 = b.take<uint32_t>(rows);
    w.v0 = b.take<uint32_t>(rows);
    w.k1 = b.take<uint32_t>(rows);
    w.v1 = b.take<uint32_t>(rows);
    w.hist = b.take<uint32_t>((size_t)256 * (size_t)dev::tiles((int64_t)rows));
    w.rowsum = b.take<uint32_t>(256);
    w.part32 = b.take<uint32_t>(dev::kScanGrid);
    return w;
}

// ---- device --------------------------------------------------------------------

namespace {

constexpr int kPB = 256;        // threads per decode block
constexpr int kRuns = 256;      // hybrid runs read ahead per round

__device__ __forceinline__ int64_t le_int(const uint8_t* p, int bytes) {
    uint64_t v = 0;
    for (int i = 0; i < bytes; ++i) v |= (uint64_t)p[i] << (8 * i);
    return bytes == 4 ? (int64_t)(int32_t)(uint32_t)v : (int64_t)v;
}

__device__ __forceinline__ void pq_fail(const PqWs& w, int32_t code) {
    atomicCAS(reinterpret_cast<unsigned long long*>(&w.scal[0]), 0ull, (unsigned long long)(int64_t)code);
}

__device__ __forceinline__ void pq_null_at(const PqWs& w, int64_t row) {
    atomicMin(reinterpret_cast<unsigned long long*>(&w.scal[1]), (unsigned long long)row);
}

// Thrift compact reader of one page header (device, one thread).
struct HdrIn {
    const uint8_t* b;
    int64_t p, end;
    bool bad;
    __device__ uint8_t byte() {
        if (p >= end) {
            bad = true;
            return 0;
        }
        return b[p++];
    }
    __device__ uint64_t uvar() {
        uint64_t v = 0;
        for (int s = 0; s < 64; s += 7) {
            const uint8_t c = byte();
            if (bad) return 0;
            v |= (uint64_t)(c & 0x7f) << s;
            if ((c & 0x80) == 0) return v;
        }
        bad = true;
        return 0;
    }
    __device__ int64_t svar() {
        const uint64_t u = uvar();
        return (int64_t)(u >> 1) ^ -(int64_t)(u & 1);
    }
    __device__ int field(int& last) {
        const uint8_t h = byte();
        const int t = h & 15;
        if (t == 0 || bad) return 0;
        const int d = h >> 4;
        last = d ? last + d : (int)svar();
        return t;
    }
    // a scalar, binary, or list / set of them (page statistics and friends)
    __device__ void skip_flat(int t, bool element) {
        switch (t) {
            case 1:
            case 2:
                if (element) byte();
                break;
            case 3: byte(); break;
            case 4:
            case 5:
            case 6: uvar(); break;
            case 7: p += 8; break;
            case 8: {
                const uint64_t len = uvar();
                if (len > (uint64_t)(end - p)) bad = true;
                else p += (int64_t)len;
                break;
            }
            case 9:
            case 10: {
                const uint8_t h = byte();
                uint64_t n = h >> 4;
                if (n == 15) n = uvar();
                if (n > (uint64_t)(end - p)) bad = true;
                for (uint64_t k = 0; k < n && !bad; ++k) skip_flat(h & 15, true);
                break;
            }
            default: bad = true;   // maps and deeper nesting do not occur in page headers
        }
        if (p > end) bad = true;
    }
    // a struct whose fields are flat values or structs of flat values
    __device__ void skip_struct(int depth) {
        int last = 0, t;
        while ((t = field(last)) != 0 && !bad) {
            if (t == 12) {
                if (depth <= 0) bad = true;
                else skip_struct(depth - 1);
            } else {
                skip_flat(t, false);
            }
        }
    }
};

struct PageHdr {
    int32_t type, csize, nv, enc, dlen, rlen, v2, ok;
    int64_t data;   // file offset of the page's bytes
};

// Reads the page header at file offset `at` (chunk ends at `end`).
__device__ PageHdr read_page_header(const uint8_t* f, int64_t at, int64_t end) {
    PageHdr h{-1, -1, -1, -1, -1, -1, 0, 0, 0};
    HdrIn r{f, at, end, false};
    int last = 0, t;
    while ((t = r.field(last)) != 0 && !r.bad) {
        if (last == 1 && t == 5) h.type = (int32_t)r.svar();
        else if (last == 3 && t == 5) h.csize = (int32_t)r.svar();
        else if ((last == 5 || last == 7 || last == 8) && t == 12) {
            const int which = last;
            h.v2 = which == 8;
            int l2 = 0, t2;
            while ((t2 = r.field(l2)) != 0 && !r.bad) {
                if (l2 == 1 && t2 == 5) h.nv = (int32_t)r.svar();
                else if (((which != 8 && l2 == 2) || (which == 8 && l2 == 4)) && t2 == 5) h.enc = (int32_t)r.svar();
                else if (which == 8 && l2 == 5 && t2 == 5) h.dlen = (int32_t)r.svar();
                else if (which == 8 && l2 == 6 && t2 == 5) h.rlen = (int32_t)r.svar();
                else if (t2 == 12) r.skip_struct(1);
                else r.skip_flat(t2, false);
            }
        } else if (t == 12) {
            r.skip_struct(1);
        } else {
            r.skip_flat(t, false);
        }
    }
    h.data = r.p;
    h.ok = !r.bad && h.type >= 0 && h.csize >= 0 && h.csize <= end - r.p;
    return h;
}

// One run of an RLE / bit-packing hybrid stream.
struct Run {
    int64_t first;   // index of its first value in the stream
    int64_t count;
    int64_t pos;     // bit-packed: file offset of its bytes; RLE: unused
    uint32_t value;  // RLE: the repeated value
    int32_t packed;
};

// Thread 0 reads up to kRuns run headers from *at (< end), covering values
// [*done, total); returns the number read (-1 on a malformed stream).
__device__ int read_runs(const uint8_t* f, int64_t* at, int64_t end, int bw, int64_t* done, int64_t total,
                         Run* runs) {
    int n = 0;
    const int vb = (bw + 7) / 8;
    HdrIn r{f, *at, end, false};
    while (*done < total && n < kRuns) {
        const uint64_t h = r.uvar();
        if (r.bad) return -1;
        Run u{*done, 0, 0, 0, 0};
        if (h & 1) {
            const uint64_t groups = h >> 1;
            if (groups > (uint64_t)(end - r.p) || (int64_t)groups * bw > end - r.p) return -1;
            u.packed = 1;
            u.pos = r.p;
            u.count = (int64_t)groups * 8;
            r.p += (int64_t)groups * bw;
        } else {
            if (vb > end - r.p) return -1;
            uint32_t v = 0;
            for (int i = 0; i < vb; ++i) v |= (uint32_t)f[r.p + i] << (8 * i);
            r.p += vb;
            u.value = v;
            u.count = (int64_t)(h >> 1);
        }
        if (u.count > total - *done) u.count = total - *done;
        *done += u.count;
        runs[n++] = u;
    }
    *at = r.p;
    return n;
}

// Value j of a bit-packed run of width bw (least significant bit first).
__device__ __forceinline__ uint32_t unpack(const uint8_t* f, int64_t pos, int64_t j, int bw) {
    if (bw == 0) return 0;
    const int64_t bit = j * bw;
    const uint8_t* p = f + pos + (bit >> 3);
    const int nb = (int)(((bit & 7) + bw + 7) >> 3);   // bytes spanned, at most 5
    uint64_t v = 0;
    for (int i = 0; i < nb; ++i) v |= (uint64_t)p[i] << (8 * i);
    return (uint32_t)((v >> (bit & 7)) & ((bw == 32) ? 0xFFFFFFFFull : ((1ull << bw) - 1)));
}

// Where a decoded value goes: the per-row arrays (case, activity: integer or
// byte range; timestamps: the output) or the chunk's dictionary.
struct Sink {
    int64_t* a;
    int32_t* b;   // NULL for timestamps
};

__device__ __forceinline__ void put(Sink s, int64_t i, int64_t a, int32_t b) {
    s.a[i] = a;
    if (s.b) s.b[i] = b;
}

__global__ __launch_bounds__(kPB) void k_pq_decode(const uint8_t* __restrict__ f, PqWs w, int64_t* __restrict__ ts) {
    __shared__ PageHdr sh;
    __shared__ Run runs[kRuns];
    __shared__ int s_nruns, s_null, s_stop;
    __shared__ int64_t s_at, s_done;
    const PqChunk ch = w.chunks[blockIdx.x];
    const int tid = threadIdx.x;
    const int w_int = ch.type == 1 ? 4 : 8;
    const Sink rows = ch.col == 2 ? Sink{ts, nullptr} : Sink{w.val_a + ch.col * w.max_rows, w.val_b + ch.col * w.max_rows};
    const Sink dict{w.dict_a + ch.dict_base, w.dict_b + ch.dict_base};
    int64_t pos = ch.start, done = 0, dict_n = -1;
    while (done < ch.num_values) {
        __syncthreads();   // every thread has read the previous page's header
        if (tid == 0) {
            sh = read_page_header(f, pos, ch.end);
            s_stop = 0;
            if (!sh.ok) {
                pq_fail(w, PM4G_E_PARSE);
                s_stop = 1;
            }
        }
        __syncthreads();
        const PageHdr h = sh;
        if (s_stop) return;
        pos = h.data + h.csize;
        const int64_t pend = h.data + h.csize;
        if (h.type == 2) {   // dictionary page: PLAIN values
            bool bad = h.nv < 0 || dict_n >= 0 || h.nv > ch.num_values || (h.enc != 0 && h.enc != 2);
            if (bad) {
                if (tid == 0) pq_fail(w, (h.enc != 0 && h.enc != 2) ? PM4G_E_UNSUPPORTED : PM4G_E_PARSE);
                return;
            }
            dict_n = h.nv;
            if (ch.type != 6) {
                if ((int64_t)h.nv * w_int > h.csize) {
                    if (tid == 0) pq_fail(w, PM4G_E_PARSE);
                    return;
                }
                for (int64_t k = tid; k < dict_n; k += kPB) put(dict, k, le_int(f + h.data + k * w_int, w_int), -1);
            } else if (tid == 0) {   // length-prefixed byte arrays: a sequential walk
                int64_t p = h.data;
                for (int64_t k = 0; k < dict_n; ++k) {
                    if (4 > pend - p) { pq_fail(w, PM4G_E_PARSE); break; }
                    const int64_t L = le_int(f + p, 4) & 0xffffffffll;
                    if (L > pend - p - 4) { pq_fail(w, PM4G_E_PARSE); break; }
                    put(dict, k, p + 4, (int32_t)L);
                    p += 4 + L;
                }
            }
            __syncthreads();
            continue;
        }
        if (h.type != 0 && h.type != 3) continue;   // index pages hold no values
        if (h.nv < 0 || h.nv > ch.num_values - done || (h.v2 && (h.dlen < 0 || h.rlen < 0 || h.dlen > h.csize))) {
            if (tid == 0) pq_fail(w, PM4G_E_PARSE);
            return;
        }
        if (h.v2 && h.rlen != 0) {   // repetition levels belong to nested schemas
            if (tid == 0) pq_fail(w, PM4G_E_UNSUPPORTED);
            return;
        }
        const int64_t row_base = ch.row0 + done;
        int64_t p = h.data;
        // definition levels (width 1): a 0 is a null, the page's first one is reported
        if (tid == 0) {
            s_null = 0;
            s_at = p;
            if (ch.optional) {
                int64_t lb = h.dlen, q = p;
                if (!h.v2) {
                    lb = h.csize >= 4 ? (le_int(f + p, 4) & 0xffffffffll) : -1;
                    q = p + 4;
                }
                if (lb < 0 || lb > pend - q) {
                    pq_fail(w, PM4G_E_PARSE);
                    s_null = 2;
                } else {
                    // the level runs one at a time (no null: usually a single RLE run)
                    HdrIn r{f, q, q + lb, false};
                    int64_t k = 0;
                    while (k < h.nv && !r.bad && s_null == 0) {
                        const uint64_t hh = r.uvar();
                        if (r.bad) break;
                        if (hh & 1) {
                            const int64_t cnt = (int64_t)(hh >> 1) * 8, bytes = (int64_t)(hh >> 1);
                            if (bytes > q + lb - r.p) { r.bad = true; break; }
                            for (int64_t j = 0; j < cnt && k + j < h.nv; ++j)
                                if (((f[r.p + (j >> 3)] >> (j & 7)) & 1) == 0) {
                                    pq_null_at(w, row_base + k + j);
                                    s_null = 1;
                                    break;
                                }
                            r.p += bytes;
                            k += cnt;
                        } else {
                            if (1 > q + lb - r.p) { r.bad = true; break; }
                            const uint8_t v = f[r.p++];
                            if ((v & 1) == 0 && (hh >> 1) > 0) {
                                pq_null_at(w, row_base + k);
                                s_null = 1;
                            }
                            k += (int64_t)(hh >> 1);
                        }
                    }
                    if (r.bad || (s_null == 0 && k < h.nv)) {
                        pq_fail(w, PM4G_E_PARSE);
                        s_null = 2;
                    }
                    s_at = q + lb;
                }
            } else if (h.v2 && h.dlen != 0) {
                pq_fail(w, PM4G_E_PARSE);
                s_null = 2;
            }
        }
        __syncthreads();
        if (s_null == 2) return;
        if (s_null == 1) {   // this chunk's result is an error at its first null; later pages do not matter
            return;
        }
        p = s_at;
        if (h.enc == 0) {   // PLAIN
            if (ch.type != 6) {
                if ((int64_t)h.nv * w_int > pend - p) {
                    if (tid == 0) pq_fail(w, PM4G_E_PARSE);
                    return;
                }
                for (int64_t k = tid; k < h.nv; k += kPB) put(rows, row_base + k, le_int(f + p + k * w_int, w_int), -1);
            } else if (tid == 0) {
                for (int64_t k = 0; k < h.nv; ++k) {
                    if (4 > pend - p) { pq_fail(w, PM4G_E_PARSE); break; }
                    const int64_t L = le_int(f + p, 4) & 0xffffffffll;
                    if (L > pend - p - 4) { pq_fail(w, PM4G_E_PARSE); break; }
                    put(rows, row_base + k, p + 4, (int32_t)L);
                    p += 4 + L;
                }
            }
        } else if (h.enc == 2 || h.enc == 8) {   // dictionary indices: bit width, then the hybrid
            if (dict_n < 0 || p >= pend || f[p] > 32) {
                if (tid == 0) pq_fail(w, PM4G_E_PARSE);
                return;
            }
            const int bw = f[p];
            if (tid == 0) {
                s_at = p + 1;
                s_done = 0;
            }
            __syncthreads();
            for (;;) {
                if (tid == 0) {
                    int64_t at = s_at, d = s_done;
                    s_nruns = d < h.nv ? read_runs(f, &at, pend, bw, &d, h.nv, runs) : 0;
                    s_at = at;
                    s_done = d;
                    if (s_nruns < 0) pq_fail(w, PM4G_E_PARSE);
                }
                __syncthreads();
                const int nr = s_nruns;
                if (nr <= 0) break;
                for (int q = 0; q < nr; ++q) {
                    const Run u = runs[q];
                    for (int64_t j = tid; j < u.count; j += kPB) {
                        const uint32_t ix = u.packed ? unpack(f, u.pos, j, bw) : u.value;
                        if ((int64_t)ix >= dict_n) {
                            pq_fail(w, PM4G_E_PARSE);
                            continue;
                        }
                        put(rows, row_base + u.first + j, dict.a[ix], dict.b ? dict.b[ix] : -1);
                    }
                }
                __syncthreads();
            }
            if (s_nruns < 0) return;
        } else {
            if (tid == 0) pq_fail(w, PM4G_E_UNSUPPORTED);
            return;
        }
        done += h.nv;
        __syncthreads();
    }
}

constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull, kFnvPrime = 0x100000001b3ull;

// Slot of hash h (linear probing); the slot keeps the smallest row holding it.
__device__ __forceinline__ uint32_t pq_insert(CsvSlot* tab, int64_t tsize, uint64_t h, uint32_t r) {
    uint64_t i = h & (uint64_t)(tsize - 1);
    for (;;) {   // more slots than rows: an empty or equal slot exists
        unsigned long long cur = __hip_atomic_load(reinterpret_cast<unsigned long long*>(&tab[i].hash),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == 0)
            cur = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[i].hash), 0ull, (unsigned long long)h);
        if (cur == 0 || cur == h) {
            if (r < __hip_atomic_load(&tab[i].first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMin(&tab[i].first, r);
            return (uint32_t)i;
        }
        i = (i + 1) & (uint64_t)(tsize - 1);
    }
}

__global__ __launch_bounds__(256) void k_pq_clear(PqWs w) {
    if (blockIdx.x == 0 && threadIdx.x == 0) w.scal[2] = 0;   // no collision seen yet
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < 2 * w.tsize; i += (int64_t)gridDim.x * 256) {
        w.table[i].hash = 0;
        w.table[i].first = 0xFFFFFFFFu;
        w.table[i].code = 0;
    }
}

// Hash of row r's value in column k (0 case, 1 activity): integers by value,
// byte arrays by their bytes; never 0 (the empty slot).
__device__ __forceinline__ uint64_t value_hash(const uint8_t* f, const PqWs& w, int k, int64_t r, uint64_t seed,
                                               uint64_t mask) {
    const int64_t a = w.val_a[k * w.max_rows + r];
    const int32_t b = w.val_b[k * w.max_rows + r];
    uint64_t h;
    if (b < 0) {
        h = splitmix64(seed, (uint64_t)a);
    } else {
        h = kFnvBasis ^ seed;
        for (int32_t i = 0; i < b; ++i) h = (h ^ f[a + i]) * kFnvPrime;
        h = splitmix64(seed, h);
    }
    h &= mask;
    return h ? h : 1;
}

__global__ __launch_bounds__(256) void k_pq_insert(const uint8_t* __restrict__ f, PqWs w, uint64_t seed,
                                                   uint64_t mask) {
    const int64_t rows = w.scal[3];
    if (w.scal[0] != 0 || w.scal[1] != INT64_MAX) return;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < rows; r += (int64_t)gridDim.x * 256)
        for (int k = 0; k < 2; ++k)
            w.slot[k * w.max_rows + r] = pq_insert(w.table + k * w.tsize, w.tsize, value_hash(f, w, k, r, seed, mask),
                                                   (uint32_t)r);
}

// Every row against its slot's first row: equal values, or a hash collision.
__global__ __launch_bounds__(256) void k_pq_verify(const uint8_t* __restrict__ f, PqWs w) {
    const int64_t rows = w.scal[3];
    if (w.scal[0] != 0 || w.scal[1] != INT64_MAX) return;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < rows; r += (int64_t)gridDim.x * 256)
        for (int k = 0; k < 2; ++k) {
            const int64_t first = w.table[k * w.tsize + w.slot[k * w.max_rows + r]].first;
            if (first == r) continue;
            const int64_t a1 = w.val_a[k * w.max_rows + r], a2 = w.val_a[k * w.max_rows + first];
            const int32_t b1 = w.val_b[k * w.max_rows + r], b2 = w.val_b[k * w.max_rows + first];
            bool same = b1 == b2;
            if (same && b1 < 0) same = a1 == a2;
            for (int32_t i = 0; same && i < b1; ++i) same = f[a1 + i] == f[a2 + i];
            if (!same) w.scal[2] = 1;
        }
}

__global__ __launch_bounds__(256) void k_pq_used(PqWs w, int k) {
    const CsvSlot* tab = w.table + k * w.tsize;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < w.tsize; i += (int64_t)gridDim.x * 256)
        w.used[i] = tab[i].hash != 0 ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_pq_list(PqWs w, int k) {
    const CsvSlot* tab = w.table + k * w.tsize;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < w.tsize; i += (int64_t)gridDim.x * 256)
        if (w.used[i]) {
            w.k0[w.pos[i]] = tab[i].first;
            w.v0[w.pos[i]] = (uint32_t)i;
        }
}

// Sorted by first row: the code of a slot is its rank; the dictionary entry is
// the value at that first row.
__global__ __launch_bounds__(256) void k_pq_codes(PqWs w, int k, const uint32_t* __restrict__ key,
                                                  const uint32_t* __restrict__ val, int64_t* __restrict__ dict_off,
                                                  int32_t* __restrict__ dict_len, int64_t* n_dict) {
    CsvSlot* tab = w.table + k * w.tsize;
    const int64_t D = w.scal[5];
    for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < D; d += (int64_t)gridDim.x * 256) {
        tab[val[d]].code = (uint32_t)d;
        const int64_t r = key[d];
        dict_off[d] = w.val_a[k * w.max_rows + r];
        dict_len[d] = w.val_b[k * w.max_rows + r];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_dict = D;
}

__global__ __launch_bounds__(256) void k_pq_emit(PqWs w, int32_t* __restrict__ case_code,
                                                 int32_t* __restrict__ act_code) {
    const int64_t rows = w.scal[3];
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < rows; r += (int64_t)gridDim.x * 256) {
        case_code[r] = (int32_t)w.table[w.slot[r]].code;
        act_code[r] = (int32_t)w.table[w.tsize + w.slot[w.max_rows + r]].code;
    }
}

__global__ void k_pq_init(PqWs w, int64_t rows) {
    if (threadIdx.x < 16) w.scal[threadIdx.x] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        w.scal[1] = INT64_MAX;
        w.scal[3] = rows;
        w.scal[8] = w.tsize;
    }
}

__global__ void k_pq_finish(PqWs w, int64_t* n_rows, int32_t* status, int64_t* bad_row) {
    const int64_t err = w.scal[0];
    const bool null = w.scal[1] != INT64_MAX;
    *n_rows = (err || null) ? 0 : w.scal[3];
    *bad_row = (!err && null) ? w.scal[1] : -1;
    *status = err ? (int32_t)err : (null ? PM4G_E_PARSE : 0);
}

unsigned grid_of(int64_t rows) {
    const int64_t g = (rows + 255) / 256;
    return (unsigned)(g < 2048 ? (g < 1 ? 1 : g) : 2048);
}

}  // namespace

hipError_t launch_pq_decode(const uint8_t* file, PqWs w, int64_t n_chunks, int64_t rows, int64_t* ts_out,
                            hipStream_t s) {
    k_pq_init<<<1, 64, 0, s>>>(w, rows);
    if (n_chunks > 0) k_pq_decode<<<(unsigned)n_chunks, kPB, 0, s>>>(file, w, ts_out);
    return hipGetLastError();
}

hipError_t launch_pq_match(const uint8_t* file, PqWs w, int64_t rows, uint64_t seed, int hash_bits,
                           hipStream_t s) {
    const uint64_t mask = (hash_bits <= 0 || hash_bits >= 64) ? ~0ull : ((1ull << hash_bits) - 1);
    k_pq_clear<<<2048, 256, 0, s>>>(w);
    k_pq_insert<<<grid_of(rows), 256, 0, s>>>(file, w, seed, mask);
    k_pq_verify<<<grid_of(rows), 256, 0, s>>>(file, w);
    return hipGetLastError();
}

hipError_t launch_pq_codes(PqWs w, int64_t rows, const pm4g_csv_out& o, hipStream_t s) {
    const int64_t ts = w.tsize;
    const unsigned gs = (unsigned)((ts + 255) / 256 < 2048 ? (ts + 255) / 256 : 2048);
    for (int k = 0; k < 2; ++k) {
        k_pq_used<<<gs, 256, 0, s>>>(w, k);
        dev::excl_scan<uint32_t>(w.used, &w.scal[8], w.pos, w.part32, reinterpret_cast<uint32_t*>(&w.scal[5]), s);
        k_pq_list<<<gs, 256, 0, s>>>(w, k);
        const bool flip = dev::sort_pairs<uint32_t>(w.k0, w.v0, w.k1, w.v1, &w.scal[5], w.max_rows, 32, w.hist,
                                                    w.rowsum, s);
        k_pq_codes<<<grid_of(rows), 256, 0, s>>>(w, k, flip ? w.k1 : w.k0, flip ? w.v1 : w.v0,
                                                 k == 0 ? o.case_dict_off : o.act_dict_off,
                                                 k == 0 ? o.case_dict_len : o.act_dict_len,
                                                 k == 0 ? o.n_cases : o.n_acts);
    }
    k_pq_emit<<<grid_of(rows), 256, 0, s>>>(w, o.case_code, o.act_code);
    return hipGetLastError();
}

hipError_t launch_pq_finish(PqWs w, const pm4g_csv_out& o, hipStream_t s) {
    k_pq_finish<<<1, 1, 0, s>>>(w, o.n_rows, o.status, o.bad_row);
    return hipGetLastError();
}

}  // namespace pm4g
