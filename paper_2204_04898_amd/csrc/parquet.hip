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
    w.pt_size = pq_table_entries((int64_t)rows);
    w.pages = b.take<uint8_t>((size_t)w.pt_size * kPqPageBytes);
    w.pt_n = b.take<int64_t>((size_t)kPqMaxChunks);
    w.pt_dict = b.take<int64_t>((size_t)kPqMaxChunks);
    w.dict_a = b.take<int64_t>(3 * rows);
    w.dict_b = b.take<int32_t>(3 * rows);
    w.val_a = b.take<int64_t>(2 * rows);
    w.val_b = b.take<int32_t>(2 * rows);
    w.slot = b.take<uint32_t>(2 * rows);
    w.table = b.take<CsvSlot>((size_t)(2 * w.tsize));
    w.dlist = b.take<uint32_t>(2 * rows);
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

constexpr int kPB = 1024;       // threads per decode block
constexpr int kRuns = 256;      // hybrid runs read ahead per round
constexpr int kHdrStage = 512;  // page-header bytes staged in LDS for the parse
constexpr int kPageSplit = 64;  // blocks per column chunk, each decoding every 64th data page

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
    // a scalar or binary (an element of a list when `element`: booleans take a byte)
    __device__ __forceinline__ void skip_scalar(int t, bool element) {
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
            default: bad = true;
        }
        if (p > end) bad = true;
    }
    // a list / set header: element type and count
    __device__ __forceinline__ int list_head(uint64_t* n) {
        const uint8_t h = byte();
        *n = h >> 4;
        if (*n == 15) *n = uvar();
        if (*n > (uint64_t)(end - p)) bad = true;
        return h & 15;
    }
    // a scalar, binary, or list / set of them, or of lists of them (page
    // statistics and friends; maps and deeper nesting do not occur in page
    // headers).  Written without recursion: a recursive device function
    // keeps its frames in scratch memory.
    __device__ __noinline__ void skip_flat(int t, bool element) {
        if (t != 9 && t != 10) {
            skip_scalar(t, element);
            return;
        }
        uint64_t n;
        const int et = list_head(&n);
        for (uint64_t k = 0; k < n && !bad; ++k) {
            if (et == 9 || et == 10) {
                uint64_t m;
                const int it = list_head(&m);
                for (uint64_t i = 0; i < m && !bad; ++i) {
                    if (it == 9 || it == 10) bad = true;
                    else skip_scalar(it, true);
                }
            } else {
                skip_scalar(et, true);
            }
        }
        if (p > end) bad = true;
    }
    // a struct whose fields are flat values (depth 0) or also structs of flat
    // values (depth 1)
    __device__ __noinline__ void skip_struct0() {
        int last = 0, t;
        while ((t = field(last)) != 0 && !bad) {
            if (t == 12) bad = true;
            else skip_flat(t, false);
        }
    }
    __device__ __noinline__ void skip_struct(int depth) {
        int last = 0, t;
        while ((t = field(last)) != 0 && !bad) {
            if (t == 12) {
                if (depth <= 0) bad = true;
                else skip_struct0();
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
__device__ PageHdr read_page_header(const uint8_t* f, int64_t at, int64_t end, int64_t data_end) {
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
    h.ok = !r.bad && h.type >= 0 && h.csize >= 0 && h.csize <= data_end - r.p;
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

// ---- PLAIN byte arrays: the chain of lengths, walked in parallel ----
//
// A PLAIN BYTE_ARRAY page is a chain: each value is a 4-byte length and its
// bytes, so where value k + 1 starts is known only once value k is read.  A
// single lane or wave following the chain spends a few hundred cycles per
// value (each step is a dependent read), so the page is walked in rounds of
// kRound bytes staged in LDS, cut into kNSeg segments of kSeg bytes:
//   candidates  for every segment, the walks from each of its first kCand
//               byte offsets to the first position past the segment (their
//               exit), with the number of values met and whether a length
//               ran past the page: one thread per (segment, offset), all in
//               parallel;
//   stitch      one thread follows the true chain across the round's
//               segments through those tables (an entry beyond the first
//               kCand offsets, after a long value, is walked directly), which
//               gives each segment's entry and the index of its first value;
//   output      one thread per segment walks its part of the chain from its
//               entry and writes the values.
// The walks, errors and outputs are those of the sequential chain (a
// length running past the page end is an error only where the chain needs it).
constexpr int kSeg = 512;
constexpr int kCand = 64;
constexpr int kNSeg = 64;
constexpr int kRound = kSeg * kNSeg;            // 32 KiB of the page per round
constexpr int kStageQ = (kRound + 32) / 16;     // staged 16-byte groups (alignment, reads across the end)

struct ChainLds {
    uint32_t st[4 * kStageQ];         // bytes [rb, rb + 16 * kStageQ) of the file (zero past the page)
    uint64_t tab[kNSeg * kCand];      // candidate walk: exit - rb (low 32 bits), values (bits 32-45),
                                      // bit 46 (during the walks): it stopped at a later candidate,
                                      // bit 47: it met a length running past the page
    int32_t ent[kNSeg];               // entry of the chain into each segment - rb (-1: none)
    int64_t rk[kNSeg];                // index of the value starting there
    int64_t e, rank;                  // the chain's position and values done, after the round
    int32_t bad;
};
constexpr uint64_t kLink = 1ull << 46, kDead = 1ull << 47;

// Little-endian u32 at byte o of the stage (o + 4 <= the staged bytes).
__device__ __forceinline__ uint32_t st_u32(const uint32_t* st, uint32_t o) {
    const uint32_t w = o >> 2, sh = (o & 3) * 8;
    const uint32_t a = st[w];
    return sh ? (a >> sh) | (st[w + 1] << (32 - sh)) : a;
}

// The chain from q up to the first position >= s1: values met, exit, and
// whether a length ran past pend (the walk stops there).
__device__ __forceinline__ void chain_walk(const uint32_t* st, int64_t rb, int64_t pend, int64_t s1, int64_t* q,
                                           uint32_t* cnt, bool* dead) {
    uint32_t c = 0;
    int64_t x = *q;
    bool d = false;
    while (x < s1) {
        if (4 > pend - x) {
            d = true;
            break;
        }
        const uint32_t L = st_u32(st, (uint32_t)(x - rb));
        if ((int64_t)L > pend - x - 4) {
            d = true;
            break;
        }
        x += 4 + (int64_t)L;
        ++c;
    }
    *q = x;
    *cnt = c;
    *dead = d;
}

// The nv values of the chain starting at p (page data ends at pend), each
// written as (file offset of its bytes, length) to out[base ..].  All threads
// of the block call it; false (the same for every thread) when the chain
// needs a length that runs past pend.
__device__ bool walk_byte_arrays(const uint8_t* __restrict__ f, int64_t p, int64_t pend, int64_t nv, Sink out,
                                 int64_t base) {
    __shared__ ChainLds S;
    const int tid = threadIdx.x;
    const bool aligned = (reinterpret_cast<uintptr_t>(f) & 15) == 0;
    int64_t e = p, rank = 0;
    while (rank < nv) {   // block-uniform: e and rank come from LDS
        if (4 > pend - e) return false;
        const int64_t R = e, rb = R & ~(int64_t)15;
        // 1. stage [rb, rb + 16 * kStageQ), zero past pend
        for (int i = tid; i < kStageQ; i += kPB) {
            const int64_t q = rb + 16 * (int64_t)i;
            uint4 v;
            if (aligned && q + 16 <= pend) {
                v = *reinterpret_cast<const uint4*>(f + q);
            } else {
                uint32_t u[4] = {0, 0, 0, 0};
                for (int b = 0; b < 16; ++b)
                    if (q + b < pend) u[b >> 2] |= (uint32_t)f[q + b] << (8 * (b & 3));
                v = make_uint4(u[0], u[1], u[2], u[3]);
            }
            S.st[4 * i] = v.x;
            S.st[4 * i + 1] = v.y;
            S.st[4 * i + 2] = v.z;
            S.st[4 * i + 3] = v.w;
        }
        __syncthreads();
        // 2. candidate walks; reads stay below R + kRound + 4 <= rb + 16 * kStageQ.
        //    A walk that lands on a later candidate offset stops there with a
        //    link (kLink), so each segment's chain is walked once; a lane
        //    that finishes a walk starts its next candidate at once (no lane
        //    waits for the longest walk of its wave).
        {
            int i = tid;
            int j = i & (kNSeg - 1), c = i / kNSeg;
            int64_t s0 = R + (int64_t)j * kSeg, x = s0 + c;
            uint32_t n = 0;
            while (i < kNSeg * kCand) {
                uint32_t flag = 0;
                bool fin = true;
                if (x < s0 + kSeg) {   // (a start is always inside its segment)
                    if (4 > pend - x) {   // no length fits (a start at or past pend included)
                        flag = 0x8000u;   // kDead >> 32
                    } else {
                        const uint32_t L = st_u32(S.st, (uint32_t)(x - rb));
                        if ((int64_t)L > pend - x - 4) {
                            flag = 0x8000u;
                        } else {
                            x += 4 + (int64_t)L;
                            ++n;
                            if (x - s0 < kCand) flag = 0x4000u;   // kLink >> 32: to candidate x - s0
                            else fin = x >= s0 + kSeg;
                        }
                    }
                }
                if (fin) {
                    S.tab[j * kCand + c] = (uint64_t)(uint32_t)(x - rb) | ((uint64_t)(n | flag) << 32);
                    i += kPB;
                    j = i & (kNSeg - 1);
                    c = i / kNSeg;
                    s0 = R + (int64_t)j * kSeg;
                    x = s0 + c;
                    n = 0;
                }
            }
        }
        __syncthreads();
        // links resolved per segment, from the last candidate down (a link
        // points to a later offset, already resolved)
        if (tid < kNSeg) {
            const int64_t s0 = R + (int64_t)tid * kSeg;
            for (int c = kCand - 1; c >= 0; --c) {
                const int at = tid * kCand + c;
                const uint64_t v = S.tab[at];
                if (v & kLink) {
                    const uint64_t t = S.tab[tid * kCand + (int)(rb + (int64_t)(uint32_t)v - s0)];
                    // the target's exit and flags, the two counts added (both < 2^14)
                    S.tab[at] = (t & 0xFFFFFFFFull) | ((((v >> 32) & 0x3FFFull) + (t >> 32)) << 32);
                }
            }
        }
        __syncthreads();
        // 3. stitch (positions as 32-bit offsets from rb: a page is < 2^31 bytes)
        if (tid == 0) {
            const int32_t r0 = (int32_t)(R - rb);
            int32_t cur = r0;
            int64_t acc = rank;
            int32_t bad = 0;
            for (int j = 0; j < kNSeg; ++j) S.ent[j] = -1;
            for (int j = 0; j < kNSeg && acc < nv; ++j) {
                const int32_t s0 = r0 + j * kSeg, s1 = s0 + kSeg;
                if (cur >= s1) continue;   // a long value spans the segment
                const int32_t off = cur - s0;
                uint32_t n;
                bool dead;
                int32_t q;
                if (off < kCand) {
                    const uint64_t v = S.tab[j * kCand + off];
                    q = (int32_t)(uint32_t)v;
                    n = (uint32_t)(v >> 32) & 0x3FFFu;
                    dead = (v & kDead) != 0;
                } else {
                    int64_t x = rb + cur;
                    chain_walk(S.st, rb, pend, rb + s1, &x, &n, &dead);
                    q = (int32_t)(x - rb);
                }
                S.ent[j] = cur;
                S.rk[j] = acc;
                if (dead && acc + (int64_t)n < nv) {
                    bad = 1;
                    break;
                }
                acc += n;
                cur = q;
                if (dead) break;   // the values needed all came before
            }
            S.e = rb + cur;
            S.rank = acc < nv ? acc : nv;
            S.bad = bad;
        }
        __syncthreads();
        if (S.bad) return false;
        // 4. output: a thread per segment
        if (tid < kNSeg && S.ent[tid] >= 0) {
            int64_t q = rb + S.ent[tid], r = S.rk[tid];
            const int64_t s1 = R + (int64_t)tid * kSeg + kSeg;
            while (q < s1 && r < nv) {
                const uint32_t L = st_u32(S.st, (uint32_t)(q - rb));
                put(out, base + r, q + 4, (int32_t)L);
                q += 4 + (int64_t)L;
                ++r;
            }
        }
        e = S.e;
        rank = S.rank;
        __syncthreads();   // every thread has read the round's results
    }
    return true;
}

// One data page whose header was checked, its first row known; false when
// the block stops decoding the chunk (an error or a null was reported).
// Every thread of the block calls it.
__device__ bool decode_data_page(const uint8_t* __restrict__ f, const PqWs& w, const PqChunk& ch, const PageHdr& h,
                                 int64_t row_base, int64_t dict_n, Sink rows, Sink dict) {
    __shared__ Run runs[kRuns];
    __shared__ int s_nruns, s_null;
    __shared__ int64_t s_at, s_done;
    const int tid = threadIdx.x;
    const int w_int = ch.type == 1 ? 4 : 8;
    const int64_t pend = h.data + h.csize;
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
    if (s_null == 2) return false;
    if (s_null == 1) {   // this chunk's result is an error at its first null; later pages do not matter
        return false;
    }
    p = s_at;
    if (h.enc == 0) {   // PLAIN
        if (ch.type != 6) {
            if ((int64_t)h.nv * w_int > pend - p) {
                if (tid == 0) pq_fail(w, PM4G_E_PARSE);
                return false;
            }
            for (int64_t k = tid; k < h.nv; k += kPB) put(rows, row_base + k, le_int(f + p + k * w_int, w_int), -1);
        } else {   // the chain of lengths, walked by the block
            const bool ok = walk_byte_arrays(f, p, pend, h.nv, rows, row_base);
            if (!ok) {
                if (tid == 0) pq_fail(w, PM4G_E_PARSE);
                return false;
            }
        }
    } else if (h.enc == 2 || h.enc == 8) {   // dictionary indices: bit width, then the hybrid
        if (dict_n < 0 || p >= pend || f[p] > 32) {
            if (tid == 0) pq_fail(w, PM4G_E_PARSE);
            return false;
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
        if (s_nruns < 0) return false;
    } else {
        if (tid == 0) pq_fail(w, PM4G_E_UNSUPPORTED);
        return false;
    }
    return true;
}

// The chunk's pages in order (blockIdx.x: the chunk), shared by the two
// walks below: page headers staged in LDS and parsed by thread 0; false on
// a malformed header (reported).  Sets *h for every thread.
__device__ bool next_page_header(const uint8_t* __restrict__ f, const PqWs& w, const PqChunk& ch, int64_t pos,
                                 PageHdr* h) {
    __shared__ PageHdr sh;
    __shared__ uint8_t hstage[kHdrStage];
    __shared__ int s_stop;
    const int tid = threadIdx.x;
    __syncthreads();   // every thread has read the previous header
    // the header's first bytes staged with one coalesced load: its parse is a
    // chain of dependent byte reads
    const int64_t wlen = ch.end - pos < kHdrStage ? ch.end - pos : kHdrStage;
    for (int i = tid; i < kHdrStage; i += kPB) hstage[i] = i < wlen ? f[pos + i] : 0;
    __syncthreads();
    if (tid == 0) {
        sh = read_page_header(hstage, 0, wlen, ch.end - pos);   // offsets from pos
        if (sh.ok) sh.data += pos;
        else if (wlen < ch.end - pos) sh = read_page_header(f, pos, ch.end, ch.end);   // longer than the stage
        s_stop = 0;
        if (!sh.ok) {
            pq_fail(w, PM4G_E_PARSE);
            s_stop = 1;
        }
    }
    __syncthreads();
    *h = sh;
    return !s_stop;
}

// A data page's header checks, before its values: false (reported) when the
// block stops.
__device__ __forceinline__ bool check_data_page(const PqWs& w, const PqChunk& ch, const PageHdr& h, int64_t done) {
    if (h.nv < 0 || h.nv > ch.num_values - done || (h.v2 && (h.dlen < 0 || h.rlen < 0 || h.dlen > h.csize))) {
        if (threadIdx.x == 0) pq_fail(w, PM4G_E_PARSE);
        return false;
    }
    if (h.v2 && h.rlen != 0) {   // repetition levels belong to nested schemas
        if (threadIdx.x == 0) pq_fail(w, PM4G_E_UNSUPPORTED);
        return false;
    }
    return true;
}

struct PqPage {        // a page-table entry
    PageHdr h;
    int64_t row_base;  // the page's first row
};
static_assert(sizeof(PqPage) == kPqPageBytes, "page-table entry size");

// Column chunk blockIdx.x, two blocks working at once: blockIdx.y == 0
// decodes its dictionary page (the chunk's first page, when it has one);
// blockIdx.y == 1 walks its page headers in order and lists its data pages
// (header, first row) in its range of the page table (pt_n: their number;
// -1 when they exceed the range, -2 after an error; pt_dict: the
// dictionary's entries).  Both check the dictionary page's header.
__global__ __launch_bounds__(kPB) void k_pq_pages(const uint8_t* __restrict__ f, PqWs w) {
    const bool decode_dict = blockIdx.y == 0;
    const PqChunk ch = w.chunks[blockIdx.x];
    const int tid = threadIdx.x;
    const int w_int = ch.type == 1 ? 4 : 8;
    const Sink dict{w.dict_a + ch.dict_base, w.dict_b + ch.dict_base};
    PqPage* table = reinterpret_cast<PqPage*>(w.pages) + ch.pt_off;
    if (tid == 0 && !decode_dict) {
        w.pt_n[blockIdx.x] = -2;   // until the walk completes
        w.pt_dict[blockIdx.x] = -1;
    }
    int64_t pos = ch.start, done = 0, dict_n = -1, n = 0;
    while (done < ch.num_values) {
        PageHdr h;
        if (!next_page_header(f, w, ch, pos, &h)) return;
        if (decode_dict && h.type != 2) return;   // no dictionary page (it comes first)
        pos = h.data + h.csize;
        const int64_t pend = h.data + h.csize;
        if (h.type == 2) {   // dictionary page: PLAIN values
            const bool bad = h.nv < 0 || dict_n >= 0 || h.nv > ch.num_values || (h.enc != 0 && h.enc != 2);
            if (bad) {
                if (tid == 0) pq_fail(w, (h.enc != 0 && h.enc != 2) ? PM4G_E_UNSUPPORTED : PM4G_E_PARSE);
                return;
            }
            dict_n = h.nv;
            if (ch.type != 6 && (int64_t)h.nv * w_int > h.csize) {
                if (tid == 0) pq_fail(w, PM4G_E_PARSE);
                return;
            }
            if (!decode_dict) continue;
            if (ch.type != 6) {
                for (int64_t k = tid; k < dict_n; k += kPB) put(dict, k, le_int(f + h.data + k * w_int, w_int), -1);
            } else if (!walk_byte_arrays(f, h.data, pend, dict_n, dict, 0)) {   // the chain, walked by the block
                if (tid == 0) pq_fail(w, PM4G_E_PARSE);
            }
            return;
        }
        if (h.type != 0 && h.type != 3) continue;   // index pages hold no values
        if (!check_data_page(w, ch, h, done)) return;
        if (tid == 0 && n < ch.pt_cap) table[n] = PqPage{h, ch.row0 + done};
        ++n;
        done += h.nv;
    }
    if (tid == 0) {
        w.pt_n[blockIdx.x] = n <= ch.pt_cap ? n : -1;
        w.pt_dict[blockIdx.x] = dict_n;
    }
}

// Column chunk blockIdx.x, after k_pq_pages: its data pages whose index is
// blockIdx.y modulo gridDim.y, looked up in the page table (or, when the
// chunk's pages did not fit there, found by walking the headers again).
__global__ __launch_bounds__(kPB) void k_pq_decode(const uint8_t* __restrict__ f, PqWs w, int64_t* __restrict__ ts) {
    const PqChunk ch = w.chunks[blockIdx.x];
    const int64_t n = w.pt_n[blockIdx.x], dict_n = w.pt_dict[blockIdx.x];
    if (n == -2) return;   // an error was reported
    const Sink rows = ch.col == 2 ? Sink{ts, nullptr} : Sink{w.val_a + ch.col * w.max_rows, w.val_b + ch.col * w.max_rows};
    const Sink dict{w.dict_a + ch.dict_base, w.dict_b + ch.dict_base};
    if (n >= 0) {
        const PqPage* table = reinterpret_cast<const PqPage*>(w.pages) + ch.pt_off;
        for (int64_t k = blockIdx.y; k < n; k += gridDim.y) {
            const PqPage pg = table[k];
            if (!decode_data_page(f, w, ch, pg.h, pg.row_base, dict_n, rows, dict)) return;
        }
        return;
    }
    int64_t pos = ch.start, done = 0, page = 0;
    while (done < ch.num_values) {
        PageHdr h;
        if (!next_page_header(f, w, ch, pos, &h)) return;
        pos = h.data + h.csize;
        if (h.type != 0 && h.type != 3) continue;   // the dictionary page was decoded, index pages hold no values
        if (!check_data_page(w, ch, h, done)) return;
        if ((page++) % gridDim.y == blockIdx.y && !decode_data_page(f, w, ch, h, ch.row0 + done, dict_n, rows, dict))
            return;
        done += h.nv;
    }
}

constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull, kFnvPrime = 0x100000001b3ull;

__global__ __launch_bounds__(256) void k_pq_clear(PqWs w) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {   // empty slot lists
        w.scal[10] = 0;
        w.scal[11] = 0;
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < 2 * w.tsize; i += (int64_t)gridDim.x * 256) {
        w.table[i].hash = 0;
        w.table[i].first = 0xFFFFFFFFu;
        w.table[i].code = 0;
    }
}

// Word k of byte array [a, a + b) of the file: its bytes a + 8k .. a + 8k + 7,
// those past the value zero.  Only aligned words holding value bytes are
// read (a value ends at least 8 bytes before the end of a Parquet file, its
// footer length and magic, and f is 8-byte aligned).
__device__ __forceinline__ uint64_t value_word(const uint8_t* __restrict__ f, int64_t a, int32_t b, int32_t k) {
    const int64_t p = a + 8 * (int64_t)k;
    const int rem = b - 8 * k < 8 ? b - 8 * k : 8;
    const int64_t al = p & ~(int64_t)7;
    const int sh = (int)(p & 7) * 8;
    uint64_t v = *reinterpret_cast<const uint64_t*>(f + al) >> sh;
    if (sh && al + 8 < p + rem) v |= *reinterpret_cast<const uint64_t*>(f + al + 8) << (64 - sh);
    return rem < 8 ? v & ((1ull << (8 * rem)) - 1) : v;
}

// Hash of a value: integers by value, byte arrays by their bytes eight at a
// time (a byte at a time if f is not 8-byte aligned); never 0 (the empty slot).
__device__ __forceinline__ uint64_t value_hash(const uint8_t* __restrict__ f, bool aligned, int64_t a, int32_t b,
                                               uint64_t seed, uint64_t mask) {
    uint64_t h;
    if (b < 0) {
        h = splitmix64(seed, (uint64_t)a);
    } else {
        h = kFnvBasis ^ seed;
        if (aligned) {
            for (int32_t k = 0; 8 * k < b; ++k) h = (h ^ value_word(f, a, b, k)) * kFnvPrime;
            h ^= (uint64_t)b;
        } else {
            for (int32_t i = 0; i < b; ++i) h = (h ^ f[a + i]) * kFnvPrime;
        }
        h = splitmix64(seed, h);
    }
    h &= mask;
    return h ? h : 1;
}

// Two values (decoded by earlier launches): equal integers, or byte arrays of
// equal bytes.
__device__ __forceinline__ bool same_pq_value(const uint8_t* __restrict__ f, bool aligned, int64_t a1, int32_t b1,
                                              int64_t a2, int32_t b2) {
    if (b1 != b2) return false;
    if (b1 < 0) return a1 == a2;
    if (aligned) {
        for (int32_t k = 0; 8 * k < b1; ++k)
            if (value_word(f, a1, b1, k) != value_word(f, a2, b2, k)) return false;
        return true;
    }
    for (int32_t i = 0; i < b1; ++i)
        if (f[a1 + i] != f[a2 + i]) return false;
    return true;
}
// Slot of row r's value in column k (hash h).  A slot's hash word is (the
// hash's upper 32 bits | 1) << 32 | the row that claimed it: one
// compare-and-swap claims an empty slot and names its owner.  Probing from h,
// an empty slot is claimed; at a slot with the same upper hash bits the
// owner's value is compared with this row's: equal values share the slot,
// which keeps the smallest row (read first, so hot values take no atomic);
// different values with one hash probe on.  Sets *claimed for a new slot.
__device__ __forceinline__ uint32_t pq_insert(const uint8_t* __restrict__ f, bool aligned, const PqWs& w, int k,
                                              uint64_t h, uint32_t r, int64_t a, int32_t b, bool* claimed) {
    CsvSlot* tab = w.table + k * w.tsize;
    const uint64_t m = (uint64_t)(w.tsize - 1);
    const uint32_t tag = (uint32_t)(h >> 32) | 1u;
    const unsigned long long mine = ((unsigned long long)tag << 32) | r;
    uint64_t i = h & m;
    for (;;) {   // more slots than rows: an empty or equal slot exists
        unsigned long long* hw = reinterpret_cast<unsigned long long*>(&tab[i].hash);
        unsigned long long cur = __hip_atomic_load(hw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == 0) {
            cur = atomicCAS(hw, 0ull, mine);
            if (cur == 0) {
                atomicMin(&tab[i].first, r);
                *claimed = true;
                return (uint32_t)i;
            }
        }
        const int64_t r2 = (int64_t)(uint32_t)cur;
        if ((uint32_t)(cur >> 32) == tag &&
            same_pq_value(f, aligned, a, b, w.val_a[k * w.max_rows + r2], w.val_b[k * w.max_rows + r2])) {
            if (r < __hip_atomic_load(&tab[i].first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMin(&tab[i].first, r);
            return (uint32_t)i;
        }
        i = (i + 1) & m;
    }
}

// Every row's case and activity values into their tables; the slots claimed
// are listed per table (one global reservation per table and block pass).
__global__ __launch_bounds__(256) void k_pq_insert(const uint8_t* __restrict__ f, PqWs w, uint64_t seed,
                                                   uint64_t mask) {
    __shared__ uint32_t s_new[2][256];
    __shared__ uint32_t s_cnt[2];
    __shared__ int64_t s_base[2];
    const int64_t rows = w.scal[3];
    if (w.scal[0] != 0 || w.scal[1] != INT64_MAX) return;
    const bool aligned = (reinterpret_cast<uintptr_t>(f) & 7) == 0;
    for (int64_t r0 = (int64_t)blockIdx.x * 256; r0 < rows; r0 += (int64_t)gridDim.x * 256) {
        if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
        __syncthreads();
        const int64_t r = r0 + threadIdx.x;
        if (r < rows) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                bool claimed = false;
                const int64_t a = w.val_a[k * w.max_rows + r];
                const int32_t b = w.val_b[k * w.max_rows + r];
                const uint32_t slot =
                    pq_insert(f, aligned, w, k, value_hash(f, aligned, a, b, seed, mask), (uint32_t)r, a, b, &claimed);
                w.slot[k * w.max_rows + r] = slot;
                if (claimed) s_new[k][atomicAdd(&s_cnt[k], 1u)] = slot;
            }
        }
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

// The slots listed for table k with their first rows, to sort; their number
// goes to scal[5] (none after a decode error or a null).
__global__ __launch_bounds__(256) void k_pq_gather(PqWs w, int k) {
    const bool failed = w.scal[0] != 0 || w.scal[1] != INT64_MAX;
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
    if (w.scal[0] != 0 || w.scal[1] != INT64_MAX) return;
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
    if (n_chunks > 0) {
        k_pq_pages<<<dim3((unsigned)n_chunks, 2), kPB, 0, s>>>(file, w);
        k_pq_decode<<<dim3((unsigned)n_chunks, kPageSplit), kPB, 0, s>>>(file, w, ts_out);
    }
    return hipGetLastError();
}

hipError_t launch_pq_match(const uint8_t* file, PqWs w, int64_t rows, uint64_t seed, int hash_bits,
                           hipStream_t s) {
    const uint64_t mask = (hash_bits <= 0 || hash_bits >= 64) ? ~0ull : ((1ull << hash_bits) - 1);
    k_pq_clear<<<2048, 256, 0, s>>>(w);
    k_pq_insert<<<grid_of(rows), 256, 0, s>>>(file, w, seed, mask);
    return hipGetLastError();
}

hipError_t launch_pq_codes(PqWs w, int64_t rows, const pm4g_csv_out& o, hipStream_t s) {
    int bits = 8;   // first rows are below max_rows: sort on that many bits
    while (bits < 32 && (int64_t(1) << bits) < w.max_rows) bits += 8;
    for (int k = 0; k < 2; ++k) {
        k_pq_gather<<<grid_of(rows), 256, 0, s>>>(w, k);
        const bool flip = dev::sort_pairs<uint32_t>(w.k0, w.v0, w.k1, w.v1, &w.scal[5], w.max_rows, bits, w.hist,
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
