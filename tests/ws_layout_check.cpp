// Workspace layouts against the largest index their consumers use.
//
// Every entry point carves its caller-owned workspace into slices with one
// layout function (csrc/*.hip, `*_ws_layout`).  This program lays each one out
// over a fake base address (nothing is dereferenced) for a grid of sizes and
// checks, for every slice, that the room up to the next slice (or to the end
// of the workspace) holds what the kernels that read or write it index.  The
// needs below are restated from those kernels (their grids, loop bounds and
// index expressions), not from the layouts: a slice sized by the wrong count
// -- a table-sized scan written into a row-sized array, say -- fails here on
// the CPU instead of overwriting its neighbour on the GPU.
//
// Built and run by tests/test_ws_layout.py; prints one line per failure and
// exits with the number of failures (0: all layouts hold their consumers).
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "common.hpp"
#include "devsort.hpp"
#include "internal.hpp"

using namespace pm4g;

namespace {

struct Need {
    const char* name;
    const void* p;
    size_t bytes;   // 0: the slice is not used in this configuration
};

#define NEED(w, field, count) Need{#field, (const void*)(w).field, (size_t)(count) * sizeof(*(w).field)}

char* const kBase = reinterpret_cast<char*>(uintptr_t(1) << 40);
int g_fail = 0;
int g_checked = 0;

void check(const std::string& what, size_t total, std::vector<Need> v) {
    ++g_checked;
    std::vector<Need> live;
    for (const Need& x : v) {
        if (x.bytes == 0) continue;
        if (x.p == nullptr) {
            std::printf("FAIL %s: slice %s is needed (%zu B) but not laid out\n", what.c_str(), x.name, x.bytes);
            ++g_fail;
            continue;
        }
        live.push_back(x);
    }
    std::sort(live.begin(), live.end(), [](const Need& a, const Need& b) { return a.p < b.p; });
    for (size_t i = 0; i < live.size(); ++i) {
        const char* p = static_cast<const char*>(live[i].p);
        if (p < kBase || (size_t)(p - kBase) > total) {
            std::printf("FAIL %s: slice %s lies outside the workspace\n", what.c_str(), live[i].name);
            ++g_fail;
            continue;
        }
        const size_t end = i + 1 < live.size() ? (size_t)(static_cast<const char*>(live[i + 1].p) - kBase) : total;
        const size_t room = end - (size_t)(p - kBase);
        if (room < live[i].bytes) {
            std::printf("FAIL %s: slice %s has %zu B, its consumers index %zu B\n", what.c_str(), live[i].name, room,
                        live[i].bytes);
            ++g_fail;
        }
    }
}

std::string tag(const char* name, int64_t a, int64_t b = -1, int64_t c = -1) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s(%lld%s%s)", name, (long long)a,
                  b >= 0 ? (", " + std::to_string(b)).c_str() : "", c >= 0 ? (", " + std::to_string(c)).c_str() : "");
    return buf;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t at_least1(int64_t x) { return x > 0 ? x : 1; }

// pm4g_prepare and the raw-log entry points: range scan (partials per radix
// tile on the tile path, else one per grid block, at most kRangeParts), the
// radix passes (n elements per buffer, digit-major [256][tiles] histograms,
// 256 row totals), the case table (a count per case tile and its total), the
// per-case sort (a case count per window).
void prep(int64_t n, bool rows) {
    Bump b(kBase);
    const PrepWs w = prep_ws_layout(b, n, rows);
    const int64_t m = at_least1(n), nb = radix_blocks(n);
    const int64_t parts = std::max<int64_t>(nb, std::min<int64_t>(ceil_div(n, 256), kRangeParts));
    check(tag("prep", n, rows), b.off,
          {NEED(w, info, 1), NEED(w, rpart, std::max<int64_t>(parts, 1)), NEED(w, a.key, m), NEED(w, a.ts, m),
           NEED(w, a.act, m), NEED(w, b.key, m), NEED(w, b.ts, m), NEED(w, b.act, m),
           NEED(w, a.row, rows ? m : 0), NEED(w, b.row, rows ? m : 0), NEED(w, hist, 256 * at_least1(nb)),
           NEED(w, hist_raw, 256 * at_least1(nb)), NEED(w, rowsum, 256), NEED(w, caseblk, case_blocks(n) + 1),
           NEED(w, wincnt, at_least1(segsort_blocks(n)))});
}

// DFG.  A*A <= 4096: 256 LDS blocks each write one partial table and one row
// of activity partials.  Otherwise: count and scatter run n_act_blocks blocks
// over chunks of kDfgTile * ceil(buckets / 64) events (one chunk per block
// when there are fewer than kDfgPartBlocks); edges are at most n - 1; the
// plan cuts each bucket into ceil(edges / ceil(E / 512)) slots, at most
// 512 + buckets in all, one partial table each; scal[0] holds the counter count.
void dfg(int64_t n, int32_t A) {
    Bump b(kBase);
    const DfgWs w = dfg_ws_layout(b, n, A);
    const std::string t = tag("dfg", n, A);
    if (A <= kDfgLdsMaxA) {
        const int64_t cells = (int64_t)kDfgLdsBlocks * kCellsPerTable;
        check(t, b.off,
              {NEED(w, pcount, cells), NEED(w, psum, cells), NEED(w, pmin, cells), NEED(w, pmax, cells),
               NEED(w, pfreq, kDfgLdsBlocks * A), NEED(w, pstart, kDfgLdsBlocks * A),
               NEED(w, pend, kDfgLdsBlocks * A), NEED(w, pspan, kDfgLdsBlocks)});
        return;
    }
    const int64_t nbk = ceil_div((int64_t)A * A, kCellsPerTable);
    const int64_t chunk = (int64_t)kDfgTile * (nbk <= 64 ? 1 : ceil_div(nbk, 64));
    const int64_t nch = ceil_div(n, chunk);
    const int64_t g = std::min<int64_t>(at_least1(nch), kDfgPartBlocks);
    const int64_t slots = nbk + kDfgAggTarget;
    const int64_t edges = at_least1(n - 1);
    check(t, b.off,
          {NEED(w, pcount, slots * kCellsPerTable), NEED(w, psum, slots * kCellsPerTable),
           NEED(w, pmin, slots * kCellsPerTable), NEED(w, pmax, slots * kCellsPerTable), NEED(w, ecell, edges),
           NEED(w, egap, edges), NEED(w, ecnt, at_least1(nbk * nch)), NEED(w, escan, at_least1(nbk * nch)),
           NEED(w, bbase, nbk), NEED(w, btotal, nbk), NEED(w, bfirst, nbk), NEED(w, bslots, nbk),
           NEED(w, plan, slots), NEED(w, nplan, 1), NEED(w, part32, dev::kScanGrid), NEED(w, scal, 1),
           NEED(w, utotal, 1), NEED(w, pstart, g * A), NEED(w, pend, g * A), NEED(w, pspan, g)});
}

// Variants: C <= n cases hashed and sorted by (hash, index) with the device
// sort (histograms [256][tiles(n)]), V <= C groups with V + 1 starts, keys
// sorted again, lengths scanned into V offsets; scal[0..2], u32scal[0..1].
void variants(int64_t n) {
    Bump b(kBase);
    const VarWs w = var_ws_layout(b, n);
    const int64_t C = at_least1(n), V = C;
    check(tag("variants", n), b.off,
          {NEED(w, hash, C), NEED(w, hash2, C), NEED(w, idx, C), NEED(w, idx2, C),
           NEED(w, hist, 256 * dev::tiles(C)), NEED(w, rowsum, 256), NEED(w, flag, C), NEED(w, sid, C),
           NEED(w, sstart, V + 1), NEED(w, repflag, C), NEED(w, rrank, C), NEED(w, vcr, V), NEED(w, cvar, C),
           NEED(w, vkey, V), NEED(w, vkey2, V), NEED(w, vidx, V), NEED(w, vidx2, V), NEED(w, fid, V),
           NEED(w, lens, V), NEED(w, part32, dev::kScanGrid), NEED(w, part64, dev::kScanGrid), NEED(w, scal, 3),
           NEED(w, u32scal, 2)});
}

// Batched views: per tile a view count at p0 / tile and a decrement at
// (p1 - 1) / tile + 1 <= tiles, their scan with the total at [tiles]; tile
// lists and records bounded by their capacities (checked on the device before
// any write past them), a carry per pair and a run place per (pair,
// bucket); V * buckets (view, bucket) counters and segments with the segment
// total at [segments]; scal up to [12].
void views(int64_t n, int32_t A, int32_t V, int32_t tile, int64_t pair_cap, int64_t rec_cap, int64_t cell_cap) {
    Bump b(kBase);
    const ViewWs w = view_ws_layout(b, n, A, V, tile, pair_cap, rec_cap, cell_cap);
    const int64_t tiles = ceil_div(n, tile), nvb = at_least1((int64_t)V * view_buckets(A)), vm = at_least1(V);
    check(tag("views", n, A, V) + "/" + std::to_string(tile), b.off,
          {NEED(w, p0, vm), NEED(w, p1, vm), NEED(w, tcount, tiles + 2), NEED(w, toff, tiles + 1),
           NEED(w, tcursor, tiles + 1), NEED(w, list, at_least1(pair_cap)), NEED(w, scal, 13),
           NEED(w, part32, dev::kScanGrid), NEED(w, part64, dev::kScanGrid), NEED(w, part64b, dev::kScanGrid),
           NEED(w, bar, kViewMaxBlocks + 1), NEED(w, rec_cell, at_least1(rec_cap)),
           NEED(w, rec_gap, at_least1(rec_cap)), NEED(w, pair_carry, at_least1(pair_cap)),
           NEED(w, pair_rel, at_least1(pair_cap) * view_buckets(A)), NEED(w, vb_cnt, nvb), NEED(w, vb_base, nvb),
           NEED(w, vb_flag, nvb), NEED(w, vb_seg, nvb), NEED(w, seg_key, nvb), NEED(w, seg_rec, nvb + 1),
           NEED(w, seg_cells, nvb), NEED(w, seg_tmp, nvb), NEED(w, seg_out, nvb), NEED(w, view_cells, vm),
           NEED(w, t_cell, at_least1(cell_cap)), NEED(w, t_count, at_least1(cell_cap)),
           NEED(w, t_sum, at_least1(cell_cap)), NEED(w, t_min, at_least1(cell_cap)),
           NEED(w, t_max, at_least1(cell_cap))});
}

// Event filters: one count per kFilterTile tile of the scanned range, its scan
// (also reused for the case-block scan of the kept events: kCaseTile ==
// kFilterTile blocks), case-block counts with one extra entry, scal[0..7].
void filter(int64_t n) {
    Bump b(kBase);
    const FilterWs w = filter_ws_layout(b, n);
    const int64_t tiles = ceil_div(n, kFilterTile);
    check(tag("filter", n), b.off,
          {NEED(w, scal, 8), NEED(w, tile_cnt, at_least1(tiles)),
           NEED(w, tile_off, at_least1(std::max<int64_t>(tiles, case_blocks(n)))),
           NEED(w, part64, dev::kScanGrid), NEED(w, caseblk, case_blocks(n) + 1)});
}

// Case filters: per case (at most n) flags, counts, kept flags and their
// scans; scal[0..2], uscal[0].
void case_filter(int64_t n) {
    Bump b(kBase);
    const CaseFilterWs w = case_filter_ws_layout(b, n);
    const int64_t C = at_least1(n);
    check(tag("case_filter", n), b.off,
          {NEED(w, flags, C), NEED(w, cnt, C), NEED(w, kept, C), NEED(w, eoff, C), NEED(w, koff, C),
           NEED(w, part32, dev::kScanGrid), NEED(w, part64, dev::kScanGrid), NEED(w, scal, 3), NEED(w, uscal, 1)});
}

// Eventually-follows graph: a tail count per event and the pair offsets of the
// (bucketed) source list, with the pair total at [len] (len <= n); per
// (bucket, chunk of kEfgChunk events) counters and their scan; at most
// kEfgPlanBlocks + buckets plan entries, one partial table each; scal[0..4].
void efg(int64_t n, int32_t A) {
    Bump b(kBase);
    const EfgWs w = efg_ws_layout(b, n, A);
    const int64_t nbk = efg_buckets(A), nch = at_least1(ceil_div(n, kEfgChunk)), m = at_least1(n);
    const bool bk = nbk > 1;
    check(tag("efg", n, A), b.off,
          {NEED(w, tail, m), NEED(w, poff, m + 1), NEED(w, list, bk ? m : 0), NEED(w, tl, bk ? m : 0),
           NEED(w, bcnt, bk ? nbk * nch : 0), NEED(w, boff, bk ? nbk * nch : 0), NEED(w, part64, dev::kScanGrid),
           NEED(w, scal, 5), NEED(w, bfirst, nbk), NEED(w, bnum, nbk), NEED(w, plan, kEfgPlanBlocks + nbk),
           NEED(w, part, (kEfgPlanBlocks + nbk) * (int64_t)kSlotWords)});
}

// CSV: per 4096-byte tile quote parities, line counts (both starting
// parities) and their scans, 256 end masks per tile; line ends up to the line
// capacity max_rows + 1 (header) plus the unterminated last line; two fields
// per row; two hash tables of tsize slots; the slots claimed in each table
// (one per distinct value: at most the rows), sorted by first row; scal up
// to [11].
void csv(int64_t n_bytes, int64_t max_rows) {
    Bump b(kBase);
    const CsvWs w = csv_ws_layout(b, n_bytes, max_rows);
    const int64_t tiles = at_least1(ceil_div(n_bytes, 4096)), rows = at_least1(max_rows);
    check(tag("csv", n_bytes, max_rows), b.off,
          {NEED(w, qpar, tiles), NEED(w, qpre, tiles), NEED(w, lcnt, tiles), NEED(w, lcnt1, tiles),
           NEED(w, emask, tiles * 256), NEED(w, loff, tiles), NEED(w, line_end, rows + 2), NEED(w, foff, 2 * rows),
           NEED(w, flen, 2 * rows), NEED(w, slot, 2 * rows), NEED(w, table, 2 * w.tsize), NEED(w, dlist, 2 * rows),
           NEED(w, k0, rows), NEED(w, v0, rows), NEED(w, k1, rows), NEED(w, v1, rows),
           NEED(w, hist, 256 * dev::tiles(rows)), NEED(w, rowsum, 256), NEED(w, part32, dev::kScanGrid),
           NEED(w, part64, dev::kScanGrid), NEED(w, scal, 12)});
    if (w.tsize < 2 * rows) {
        std::printf("FAIL csv(%lld, %lld): %lld table slots for %lld rows\n", (long long)n_bytes, (long long)max_rows,
                    (long long)w.tsize, (long long)rows);
        ++g_fail;
    }
}

// Parquet: the chunk list (the host rejects more than kPqMaxChunks) and a
// page count and dictionary size per chunk; the page table (the host hands
// the chunks ranges of it, never past pt_size entries); each
// chunk's dictionary holds at most its values (checked per dictionary page),
// and the chunks of the three columns hold 3 * rows values; two value columns
// and two slot columns of max_rows; two tables; the slots claimed in each
// (at most the rows), sorted by first row; scal up to [11].
void parquet(int64_t max_rows) {
    Bump b(kBase);
    const PqWs w = pq_ws_layout(b, max_rows);
    const int64_t rows = at_least1(max_rows);
    check(tag("parquet", max_rows), b.off,
          {NEED(w, scal, 12), NEED(w, chunks, kPqMaxChunks), NEED(w, pages, w.pt_size * kPqPageBytes),
           NEED(w, pt_n, kPqMaxChunks), NEED(w, pt_dict, kPqMaxChunks), NEED(w, dict_a, 3 * rows), NEED(w, dict_b, 3 * rows),
           NEED(w, val_a, 2 * rows), NEED(w, val_b, 2 * rows), NEED(w, slot, 2 * rows), NEED(w, table, 2 * w.tsize),
           NEED(w, dlist, 2 * rows), NEED(w, k0, rows), NEED(w, v0, rows), NEED(w, k1, rows),
           NEED(w, v1, rows), NEED(w, hist, 256 * dev::tiles(rows)), NEED(w, rowsum, 256),
           NEED(w, part32, dev::kScanGrid)});
    if (w.tsize < 2 * rows) {
        std::printf("FAIL parquet(%lld): %lld table slots\n", (long long)max_rows, (long long)w.tsize);
        ++g_fail;
    }
}

}  // namespace

int main() {
    const int64_t ns[] = {0, 1, 2, 63, 4095, 4096, 4097, 100000, 1 << 20, 16777217, 98969504, (1ll << 31) - 1};
    const int32_t As[] = {1, 7, 64, 65, 100, 512, 1000, 4096};
    for (int64_t n : ns) {
        prep(n, false);
        prep(n, true);
        variants(n);
        filter(n);
        case_filter(n);
        for (int32_t A : As) {
            dfg(n, A);
            efg(n, A);
        }
        for (int32_t V : {0, 1, 100, 4096})
            for (int32_t tile : {256, 4096}) {
                const int64_t tiles = ceil_div(n, tile);
                const int64_t pair_cap = 4 * (tiles + V) + 1024, rec_cap = std::max<int64_t>(n, 4096);
                views(n, 512, V, tile, pair_cap, rec_cap, std::max<int64_t>(rec_cap / 2, 4096));
                views(n, 64, V, tile, 1, 1, 1);
            }
        parquet(n);
    }
    for (int64_t nb : {0ll, 1ll, 4095ll, 4096ll, 4097ll, 508795914ll, 1ll << 34})
        for (int64_t r : {0ll, 1ll, 2ll, 1000ll, 9976391ll, 1ll << 27}) csv(nb, r);
    std::printf("%d layouts checked, %d failures\n", g_checked, g_fail);
    return g_fail;
}
