// Internal interface between the C-ABI layer (api.hip) and the kernel files.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pm4g.h"

namespace pm4g {

// Device header written by the range scan and read back by the host.
struct RangeInfo {
    int32_t case_min;
    int32_t case_max;
    int32_t status;     // first data-dependent error (PM4G_E_*), 0 if none
    int32_t long_case;  // the case-segment sort met a case beyond its LDS window
    int64_t ts_min;
    int64_t ts_max;
    int64_t reserved[4];
};

// Per-block partial of the range scan.
struct RangePart {
    int32_t cmin, cmax;
    int32_t bad, unsorted;
    int64_t tmin, tmax;
};
constexpr int kRangeParts = 2048;   // blocks of the grid-stride range scan
constexpr int kRangeTileThreads = 512;

// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures (used by pm4g_workspace_bytes), so the layout has one definition.
struct Bump {
    char* base;
    size_t off = 0;
    explicit Bump(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// ---- range scan (range.hip) ----
// hist_raw (may be NULL): [256][radix tiles] histograms of the raw case id's
// low byte, for the first radix pass (raw logs only; the partials then need
// one entry per radix tile).
hipError_t launch_range_scan(const int32_t* case_id, const int32_t* act, const int64_t* ts, int64_t n,
                             int32_t A, bool presorted, bool want_ts, RangeInfo* info, RangePart* part,
                             uint32_t* hist_raw, hipStream_t s);
hipError_t launch_ts_range(const int64_t* ts, int64_t n, RangeInfo* info, hipStream_t s);

// ---- LSD radix passes over (case key u32, ts i64, act u32) elements (radix.hip) ----
struct SortBufs {
    uint32_t* key;
    int64_t* ts;
    uint32_t* act;
    uint32_t* row;   // original row of each element; NULL when the row order is not carried
};

// Workspace of the formatting step (api.hip): range-scan header and partials,
// the two radix buffers, digit histograms, case-table and window counts.
struct PrepWs {
    RangeInfo* info;
    RangePart* rpart;
    SortBufs a, b;
    uint32_t* hist;
    uint32_t* hist_raw;
    uint32_t* rowsum;
    uint32_t* caseblk;
    uint32_t* wincnt;
};
// with_rows: room for the original row of each element in both sort buffers.
PrepWs prep_ws_layout(Bump& bp, int64_t n, bool with_rows);

constexpr int kRadixTile = 4096;
inline int64_t radix_blocks(int64_t n) { return (n + kRadixTile - 1) / kRadixTile; }
// One stable pass on an 8-bit digit.  digit_src 0: ((key & case bits) >> shift) & 255;
// digit_src 1: ((ts - ts_min) >> shift) & 255.  With `first`, the input is
// the raw log (in.key is the int32 case id, biased by case_min on the fly).
// act_shift > 0 selects the packed layout: key = case | act << act_shift and
// no activity column (act_shift = number of case bits, case bits + activity
// bits <= 32); act_shift = 0: separate activity column.
// hist_raw (may be NULL; first case pass only): the range scan's raw-byte
// histograms, used instead of a histogram kernel.
hipError_t launch_radix_pass(SortBufs in, SortBufs out, int64_t n, int digit_src, int shift,
                             bool first, const RangeInfo* info, uint32_t* hist, uint32_t* rowsum,
                             int act_shift, const uint32_t* hist_raw, hipStream_t s);

// ---- per-case ordering of a case-grouped sequence (segsort.hip) ----
constexpr int kSegWindow = 1024;
constexpr int kSegCap = 3072;   // window + the longest case kept on the fast path (2049) - 1
inline int64_t segsort_blocks(int64_t n) { return (n + kSegWindow - 1) / kSegWindow; }
// wincnt: [segsort_blocks(n)] cases starting in each window (valid unless long_case).
// row_s (may be NULL): the original row of each position, from in.row.
hipError_t launch_segsort(SortBufs in, int64_t n, RangeInfo* info, int32_t* case_s, int32_t* act_s,
                          int64_t* ts_s, int act_shift, uint32_t* wincnt, int32_t* row_s, hipStream_t s);
// Copies fully sorted buffers (fallback path) into the prepared arrays.
hipError_t launch_unbias_copy(SortBufs in, int64_t n, const RangeInfo* info, int32_t* case_s,
                              int32_t* act_s, int64_t* ts_s, int act_shift, int32_t* row_s, hipStream_t s);
// Copies a presorted raw log into the prepared arrays (row_s, if given: the identity).
hipError_t launch_copy_log(const int32_t* c, const int32_t* a, const int64_t* t, int64_t n,
                           int32_t* case_s, int32_t* act_s, int64_t* ts_s, int32_t* row_s, hipStream_t s);

// ---- case table (cases.hip) ----
constexpr int kCaseTile = 4096;
inline int64_t case_blocks(int64_t n) { return (n + kCaseTile - 1) / kCaseTile; }
// wincnt (may be NULL): cases starting in each kSegWindow window, from k_segsort.
hipError_t launch_case_table(const int32_t* case_s, int64_t n, uint32_t* blockcnt, int64_t* case_off,
                             int32_t* case_code, int64_t* n_cases, const uint32_t* wincnt, hipStream_t s);

// ---- DFG aggregation (dfg.hip) ----
constexpr int kCellsPerTable = 4096;     // one LDS table of cells
constexpr int kDfgLdsMaxA = 64;          // A*A <= 4096: one privatised table per block
constexpr int kDfgLdsBlocks = 256;
constexpr int kDfgTile = 4096;
constexpr int kDfgPartBlocks = 1024;
constexpr int kDfgAggTarget = 512;

struct DfgWs {
    // partial tables, slot-major [slot][kCellsPerTable]
    uint32_t* pcount;
    uint64_t* psum;
    int64_t* pmin;
    int64_t* pmax;
    // per-block activity partials [block][A] and span partials [block]
    uint32_t* pfreq;
    uint32_t* pstart;
    uint32_t* pend;
    uint64_t* pspan;
    // bucketed path: edges in bucket-major order, each bucket cut by chunks
    uint16_t* ecell;    // [edges] cell within the bucket
    uint64_t* egap;     // [edges] timestamp gap
    uint32_t* ecnt;     // [bucket][chunk] edge counts
    uint32_t* escan;    // [bucket][chunk] exclusive scan = first edge index
    uint32_t* bbase;    // [bucket] first edge index
    uint32_t* btotal;   // [bucket] edges
    uint32_t* bfirst;   // [bucket] first aggregation slot
    uint32_t* bslots;   // [bucket] slots
    int4* plan;         // [slot] (bucket, first, end) edge range within the bucket
    uint32_t* nplan;
    uint32_t* part32;   // scan partials
    int64_t* scal;      // [0] bucket x chunk entries, [1] edges (u32 total at utotal)
    uint32_t* utotal;
    int32_t n_act_blocks;
    int32_t n_slots_max;
};
DfgWs dfg_ws_layout(Bump& b, int64_t n, int32_t A);
struct DfgOutDev {
    int64_t* count;
    int64_t* dt_sum;
    int64_t* dt_min;
    int64_t* dt_max;
    double* dt_mean;
    int64_t* start_count;
    int64_t* end_count;
    int64_t* act_count;
    int64_t* n_cases;
    int32_t* overflow;
    int32_t* status;
};
// n_cases is the number of case starts seen; status_in (may be NULL) is the
// producing prepare's status word, propagated to out.status.
hipError_t launch_dfg(const int32_t* case_s, const int32_t* act_s, const int64_t* ts_s, int64_t n,
                      int32_t A, const int32_t* status_in, DfgWs ws, DfgOutDev out, hipStream_t s);

// ---- variants (variants.hip) ----
struct VarWs {
    uint64_t* hash;      // [C] sequence hash per case, then sorted (ping-pong with hash2)
    uint64_t* hash2;
    uint32_t* idx;       // [C] case index carried through the hash sort (ping-pong with idx2)
    uint32_t* idx2;
    uint32_t* hist;      // radix histograms
    uint32_t* rowsum;    // [256]
    uint32_t* flag;      // [C] group start flags in hash order
    uint32_t* sid;       // [C] exclusive count of group starts
    uint32_t* sstart;    // [V+1] group start positions
    uint32_t* repflag;   // [C] 1 for representative cases
    uint32_t* rrank;     // [C] representative-order index of representative cases
    uint2* vcr;          // [V] (cases, representative case index), representative order
    uint32_t* cvar;      // [C] representative-order variant of each case
    uint32_t* vkey;      // [V] ordering keys (ping-pong with vkey2)
    uint32_t* vkey2;
    uint32_t* vidx;      // [V] representative-order ids (ping-pong with vidx2)
    uint32_t* vidx2;
    uint32_t* fid;       // [V] final id of each representative-order variant
    uint32_t* lens;      // [V] sequence lengths in final order
    uint32_t* part32;    // scan partials
    int64_t* part64;
    int64_t* scal;       // [0] C, [1] V, [2] total sequence length
    uint32_t* u32scal;   // [0] collision flag, [1] V
};
VarWs var_ws_layout(Bump& b, int64_t n);
struct VarOutDev {
    int64_t* n_variants;
    int64_t* var_count;
    int32_t* var_len;
    int32_t* var_rep;
    int64_t* var_off;
    int32_t* var_acts;
    int32_t* case_variant;
    int32_t* status;
};
hipError_t launch_variants(const int32_t* act_s, const int64_t* case_off, const int32_t* case_code,
                           const int64_t* n_cases, const int32_t* status_in, int64_t n, VarWs ws,
                           VarOutDev out, uint32_t debug_hash_bits, hipStream_t s);

// ---- batched views (views.hip) ----
constexpr int kViewMaxBlocks = 1024;   // blocks of the persistent launch, at most
struct ViewWs {
    int32_t tile;
    int32_t n_buckets;
    int64_t n_tiles;
    int64_t pair_cap, rec_cap, cell_cap;
    int64_t* p0;            // [V] event slice of each view
    int64_t* p1;
    uint32_t* tcount;       // [tiles + 2] overlapping views per tile
    uint32_t* toff;         // [tiles + 2]
    uint32_t* tcursor;      // [tiles + 2]
    uint32_t* list;         // [pair_cap] views of each tile
    int64_t* scal;          // cursors and totals
    uint32_t* part32;
    int64_t* part64;
    int64_t* part64b;       // a second scan's partial sums (the persistent launch scans two at once)
    uint64_t* bar;          // [kViewMaxBlocks + 1] grid barrier words of the persistent launch
    uint16_t* rec_cell;     // [rec_cap] records: cell within its bucket (logs with a case of
    uint64_t* rec_gap;      //   2^52 time units or more), gap; else cell << 52 | gap in rec_gap
    uint4* pair_carry;      // [pair_cap] per (tile, view) pair: the walk's initial carry and
                            //   whether it keeps an event
    uint32_t* pair_rel;     // [pair_cap * n_buckets] place of the pair's run of records
                            //   inside each (view, bucket) segment (non-empty runs only)
    int64_t n_vb;           // V * n_buckets (view, bucket) pairs
    uint32_t* vb_cnt;       // [n_vb] records of each (view, bucket)
    int64_t* vb_base;       // [n_vb] its segment's first record (exclusive scan)
    uint32_t* vb_flag;      // [n_vb] non-empty
    uint32_t* vb_seg;       // [n_vb] segment index of a non-empty pair
    uint32_t* seg_key;      // [segments] view * n_buckets + bucket, increasing
    int64_t* seg_rec;       // [segments + 1] first record of each segment
    uint32_t* seg_cells;    // non-empty pair cells per segment
    int64_t* seg_tmp;       // their place in the temporary cell arrays
    int64_t* seg_out;       // their place in the output lists
    uint32_t* view_cells;   // [V] non-empty pair cells per view
    uint32_t* t_cell;       // [rec_cap] temporary aggregated cells
    uint32_t* t_count;
    uint64_t* t_sum;
    int64_t* t_min;
    int64_t* t_max;
};
int64_t view_buckets(int32_t A);
ViewWs view_ws_layout(Bump& b, int64_t n, int32_t A, int32_t V, int32_t tile, int64_t pair_cap,
                      int64_t rec_cap, int64_t cell_cap);
struct BatchedOutDev {
    int64_t* edge_off;
    int32_t* src;
    int32_t* dst;
    int64_t* count;
    int64_t* dt_sum;
    int64_t* dt_min;
    int64_t* dt_max;
    double* dt_mean;
    int64_t* start_count;
    int64_t* end_count;
    int64_t* act_count;
    int64_t* n_events;
    int64_t* n_cases;
    int64_t cap_edges;
    int64_t* required;
    int32_t* status;
};
// ---- one view as a prepared log (filter.hip) ----
constexpr int kFilterTile = 4096;
struct FilterWs {
    int64_t* scal;
    uint32_t* tile_cnt;
    int64_t* tile_off;
    int64_t* part64;
    uint32_t* caseblk;
};
FilterWs filter_ws_layout(Bump& b, int64_t n);
hipError_t launch_filter_view(const pm4g_prepared* p, const pm4g_view* view, const uint64_t* mask,
                              const pm4g_prepared* out, FilterWs w, hipStream_t s);
hipError_t launch_filter_df_events(const pm4g_prepared* p, const uint64_t* pairs, int32_t side, int32_t keep,
                                   const pm4g_prepared* out, FilterWs w, hipStream_t s);

// Cases dataframe and case-level filters (casefilter.hip).
struct CaseFilterWs {
    uint32_t* flags;   // [cases] containment bits
    uint32_t* cnt;     // [cases] kept events
    uint32_t* kept;    // [cases] kept flag
    int64_t* eoff;     // [cases] first output event
    uint32_t* koff;    // [cases] output case-table row
    uint32_t* part32;
    int64_t* part64;
    int64_t* scal;
    uint32_t* uscal;
};
CaseFilterWs case_filter_ws_layout(Bump& b, int64_t n);
hipError_t launch_cases_df(const pm4g_prepared* p, int64_t* n_events, int64_t* thr, hipStream_t s);
hipError_t launch_filter_cases(const pm4g_prepared* p, const pm4g_case_filter* f, const pm4g_prepared* out,
                               CaseFilterWs w, hipStream_t s);

hipError_t launch_views_plan(const pm4g_prepared* p, const pm4g_view* views, int32_t V, ViewWs w,
                             BatchedOutDev out, hipStream_t s);
// Count walk: per (tile, view) pair its records per bucket; each non-empty
// run's place inside its (view, bucket) segment.
hipError_t launch_views_count(const pm4g_prepared* p, const pm4g_view* views, const uint64_t* masks,
                              ViewWs w, int grid, hipStream_t s);
// After the segments are placed: write walk into the runs.
hipError_t launch_views_write(const pm4g_prepared* p, const pm4g_view* views, const uint64_t* masks,
                              ViewWs w, int grid, hipStream_t s);
hipError_t launch_views_reduce(const pm4g_prepared* p, const pm4g_view* views, const uint64_t* masks, int32_t V,
                               ViewWs w, BatchedOutDev out, int emit_grid, int agg_grid, hipStream_t s);
// The whole call as one persistent cooperative launch (the same phases, grid
// barriers in between).
hipError_t launch_views_fused(const pm4g_prepared* p, const pm4g_view* views, const uint64_t* masks, int32_t V,
                              ViewWs w, BatchedOutDev out, hipStream_t s);


// ---- eventually-follows graph and temporal profile (efg.hip) ----
struct EfgEntry {
    int64_t q0, q1;     // pair range [q0, q1) of the flattened list
    int64_t klo, khi;   // its bucket's list range
    int32_t b, pad;     // bucket
};
struct EfgWs {
    uint32_t* tail;     // [n] later events of the event's case
    int64_t* poff;      // [list + 1] pair offsets
    uint32_t* list;     // [n] bucketed source events (bucketed only)
    uint32_t* tl;       // [n] their tails
    uint32_t* bcnt;     // [buckets * chunks]
    int64_t* boff;      // [buckets * chunks]
    int64_t* part64;
    int64_t* scal;
    int64_t* bfirst;    // [buckets] first plan entry
    int64_t* bnum;      // [buckets] plan entries
    EfgEntry* plan;     // [plan blocks + buckets]
    uint64_t* part;     // [plan blocks + buckets][5][4096] partial tables
};
struct EfgOutDev {
    int64_t* count;
    uint64_t* sum_lo;
    uint64_t* sum_hi;
    uint64_t* sq_lo;
    uint64_t* sq_hi;
    double* mean;
    double* std;
    int64_t* n_pairs;
    int32_t* status;
};
constexpr int kEfgCells = 4096;          // cells of one LDS table
constexpr int kEfgChunk = 4096;          // events per block pass when bucketing
constexpr int kEfgPlanBlocks = 1024;     // plan entries spread over the pairs
constexpr int kSlotWords = 5 * kEfgCells;   // partial table words: cnt, sum lo, sum hi, sq lo, sq hi
int efg_rows(int32_t A);
int64_t efg_buckets(int32_t A);
EfgWs efg_ws_layout(Bump& b, int64_t n, int32_t A);
// pass_pairs: pairs per LDS pass (0: the full 2^31; smaller values are a test hook)
hipError_t launch_efg(const pm4g_prepared* p, EfgWs w, const EfgOutDev& o, int64_t pass_pairs, hipStream_t s);


// ---- sampling (sample.hip; the kept units' materialisation in filter.hip and
// casefilter.hip) ----
// Radix select of the k-th smallest SplitMix64 key over the units (events by
// position, or cases by id): after the passes, a unit is kept iff none == 0
// and (all != 0 or its key <= T).
struct SelState {
    uint64_t prefix;
    int64_t krem;
    uint64_t T;
    int32_t none;
    int32_t all;
    uint32_t hist[256];
};
hipError_t launch_sample_select(const pm4g_prepared* p, int64_t k, uint64_t seed, bool by_events, SelState* sel,
                                hipStream_t s);
hipError_t launch_sample_events(const pm4g_prepared* p, uint64_t seed, const SelState* sel,
                                const pm4g_prepared* out, FilterWs w, hipStream_t s);
hipError_t launch_sample_cases(const pm4g_prepared* p, uint64_t seed, const SelState* sel,
                               const pm4g_prepared* out, CaseFilterWs w, hipStream_t s);


// ---- CSV ingestion (csv.hip) ----
struct CsvSlot {
    uint64_t hash;    // 0: empty; CSV: the value's 64-bit hash; Parquet: (upper 32 hash bits | 1) << 32 | claiming row
    uint32_t first;   // first row holding the value
    uint32_t code;
};
struct CsvWs {
    int64_t tsize;        // slots per table (power of two, at least twice the rows)
    uint32_t* qpar;       // [tiles] quote parity
    uint32_t* qpre;       // [tiles] parity before the tile
    uint32_t* lcnt;       // [tiles] line ends (for the tile's starting quote parity once picked)
    uint32_t* lcnt1;      // [tiles] line ends if the tile starts inside quotes
    uint32_t* emask;      // [tiles][256] per-thread line-end masks: bits 0-15 starting outside quotes, 16-31 inside
    int64_t* loff;        // [tiles]
    int64_t* line_end;    // [rows + 2]
    int64_t* foff;        // [rows][2] raw field start (case, activity)
    int32_t* flen;        // [rows][2] raw field length
    uint32_t* slot;       // [rows][2] table slot
    CsvSlot* table;       // [2][tsize] case table, activity table
    int64_t max_rows;
    uint32_t* dlist;      // [2][max_rows] slots claimed in each table (the distinct values)
    uint32_t *k0, *v0, *k1, *v1;   // [rows] (first row, slot) pairs to sort
    uint32_t* hist;
    uint32_t* rowsum;
    uint32_t* part32;
    int64_t* part64;
    int64_t* scal;
};
CsvWs csv_ws_layout(Bump& b, int64_t n_bytes, int64_t max_rows);
hipError_t launch_csv_lines(const uint8_t* text, int64_t n_bytes, int has_header, int64_t max_rows, CsvWs w,
                            hipStream_t s);
// hash_bits: value hashes truncated to that many bits (0: all 64; a test hook)
hipError_t launch_csv_parse(const uint8_t* text, int64_t n_bytes, const pm4g_csv_schema& sc, uint64_t seed,
                            int hash_bits, int64_t max_rows, CsvWs w, const pm4g_csv_out& o, hipStream_t s);
hipError_t launch_csv_codes(CsvWs w, int64_t max_rows, const pm4g_csv_out& o, hipStream_t s);
hipError_t launch_csv_finish(CsvWs w, const pm4g_csv_out& o, hipStream_t s);


// ---- Parquet ingestion (parquet.hip) ----
constexpr int kPqPageBytes = 48;   // a page-table entry
// page-table entries for max_rows rows: a data page holds 32 values on average or more
inline int64_t pq_table_entries(int64_t max_rows) { return 3 * (max_rows / 32) + 4096; }
constexpr int64_t kPqMaxChunks = 3 * 65536;   // three columns of at most 65536 row groups
// One column chunk of the three read (case, activity, timestamp) in one row group.
struct PqChunk {
    int64_t start, end;    // file offsets of its pages
    int64_t num_values;    // = rows of the row group
    int64_t row0;          // its first row
    int64_t dict_base;     // its dictionary's entries in dict_a / dict_b
    int32_t type;          // 1 INT32, 2 INT64, 6 BYTE_ARRAY
    int32_t optional;      // definition levels present
    int32_t col;           // 0 case, 1 activity, 2 timestamp
    int32_t pt_cap;        // entries of the page table reserved for its data pages
    int64_t pt_off;        // the first of them
};
struct PqWs {
    int64_t tsize;         // slots per value table (power of two, at least twice the rows)
    int64_t max_rows;
    int64_t* scal;         // [0] error status, [1] first null row, [3] rows, [5] slots listed,
                           // [8] tsize, [10], [11] slots claimed in the case, activity tables
    PqChunk* chunks;
    int64_t pt_size;       // page-table entries (chunks get ranges of it on the host)
    uint8_t* pages;        // [pt_size] page table: kPqPageBytes per data page (header, first row)
    int64_t* pt_n;         // [chunks] data pages listed (-1: more than reserved, -2: a header error)
    int64_t* pt_dict;      // [chunks] dictionary entries (-1: none)
    int64_t* dict_a;       // [3 * rows] dictionary entries: integer, or byte offset in the file
    int32_t* dict_b;       //            -1, or byte length
    int64_t* val_a;        // [2][rows] case and activity values, the same way
    int32_t* val_b;
    uint32_t* slot;        // [2][rows] table slot of each value
    CsvSlot* table;        // [2][tsize]
    uint32_t* dlist;       // [2][max_rows] slots claimed in each table (the distinct values)
    uint32_t *k0, *v0, *k1, *v1;
    uint32_t* hist;
    uint32_t* rowsum;
    uint32_t* part32;
};
PqWs pq_ws_layout(Bump& b, int64_t max_rows);
// Parses the file's metadata (meta: its len bytes, copied to the host) and
// lists the chunks of columns cols[0..2]; PM4G_OK, or an error code with msg.
int pq_parse_footer(const uint8_t* meta, int64_t len, int64_t file_bytes, const int32_t cols[3],
                    std::vector<PqChunk>* chunks, int64_t* rows, char* msg, size_t msg_len);
hipError_t launch_pq_decode(const uint8_t* file, PqWs w, int64_t n_chunks, int64_t rows, int64_t* ts_out,
                            hipStream_t s);
hipError_t launch_pq_match(const uint8_t* file, PqWs w, int64_t rows, uint64_t seed, int hash_bits,
                           hipStream_t s);
hipError_t launch_pq_codes(PqWs w, int64_t rows, const pm4g_csv_out& o, hipStream_t s);
hipError_t launch_pq_finish(PqWs w, const pm4g_csv_out& o, hipStream_t s);

}  // namespace pm4g
