/*
 * pm4g.h -- C ABI of the MI355X (gfx950) library for directly-follows graph
 * discovery over a columnar event log.
 *
 * The operations follow PM4Py-GPU (Berti, Phan Nghia, van der Aalst,
 * arXiv 2204.04898):
 *   - Sec. 3, formatting: the log is ordered by (case identifier, timestamp,
 *     absolute row index); each event is paired with the previous event of its
 *     case; a per-case table is built.                       -> pm4g_prepare
 *   - Sec. 3, directly-follows level: the frequency / performance
 *     directly-follows graph; start/end activities; occurrences per
 *     activity.                                               -> pm4g_dfg
 *   - Sec. 3, variant level: cases grouped by their activity sequence
 *     (an aggregation over the per-case aggregation).         -> pm4g_variants
 *   - Sec. 1 drill-down views combined with the Sec. 3 event-level timestamp
 *     filter and activity (attribute) filter, many views per launch
 *                                                             -> pm4g_dfg_batched
 *
 * Conventions shared by every entry point:
 *   - Every array argument is DEVICE memory allocated by the caller, unless the
 *     comment says "host".  The library never allocates or frees device memory;
 *     scratch space is the caller's workspace `ws` of at least
 *     pm4g_workspace_bytes(...) bytes (256-byte aligned).
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is the
 *     default stream).  Functions taking a raw (unsorted) log synchronise the
 *     stream once or twice to read a few bytes (key ranges, a long-case flag);
 *     functions taking a prepared log do not synchronise.
 *   - Host-detectable errors (NULL pointer, negative size, A outside
 *     [1, PM4G_MAX_ACTIVITIES], n_events >= 2^31, unknown flags, workspace too
 *     small) are returned before anything is enqueued.
 *   - Data-dependent errors (activity out of range, a false PM4G_PRESORTED
 *     claim, output capacity) are written to the caller's device `status`
 *     word; a call that synchronises anyway also returns them.  When a status
 *     is non-zero the other outputs are undefined.
 *   - Failures of HIP calls return PM4G_E_DEVICE; pm4g_last_error() (thread
 *     local) describes the last failure of the calling thread.
 *   - No C++ exception crosses this interface.  Calls on different streams with
 *     disjoint workspaces and outputs may run concurrently.
 */
#ifndef PM4G_H
#define PM4G_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PM4G_ABI_VERSION 2
#define PM4G_MAX_ACTIVITIES 4096
#define PM4G_BATCHED_MAX_ACTIVITIES 1024

/* Return and status codes. */
enum {
    PM4G_OK = 0,
    PM4G_E_INVALID = -1,     /* bad argument (host-detected) */
    PM4G_E_RANGE = -2,       /* an activity code outside [0, n_activities) */
    PM4G_E_NOT_SORTED = -3,  /* PM4G_PRESORTED given but rows are not in (case, ts, row) order */
    PM4G_E_CAPACITY = -4,    /* an output arena is too small; the required size is reported */
    PM4G_E_WORKSPACE = -5,   /* ws_bytes < pm4g_workspace_bytes(...) */
    PM4G_E_DEVICE = -6,      /* a HIP runtime call failed */
    PM4G_E_PARSE = -7,       /* CSV / Parquet ingestion: a data row could not be parsed */
    PM4G_E_UNSUPPORTED = -8  /* Parquet ingestion: a valid file outside the covered subset */
};

/* pm4g_log.flags */
enum {
    PM4G_PRESORTED = 1u      /* caller promises (case, ts, row) order; it is verified */
};

/* Operations, for pm4g_workspace_bytes. */
enum {
    PM4G_OP_PREPARE = 1,
    PM4G_OP_DFG = 2,             /* pm4g_dfg on a raw log */
    PM4G_OP_DFG_PREPARED = 3,
    PM4G_OP_VARIANTS = 4,        /* pm4g_variants on a raw log */
    PM4G_OP_VARIANTS_PREPARED = 5,
    PM4G_OP_DFG_BATCHED = 6
};

/*
 * A raw event log: row i is the event (case_id[i], activity[i], timestamp[i]).
 * Case ids are any int32 (ordered as signed); activities are codes in
 * [0, n_activities); timestamps are int64 in any unit (ordered as signed).
 * 0 <= n_events < 2^31.
 */
typedef struct {
    const int32_t *case_id;
    const int32_t *activity;
    const int64_t *timestamp;
    int64_t n_events;
    int32_t n_activities;
    uint32_t flags;
} pm4g_log;

/*
 * A prepared (formatted) log, Sec. 3: the events in (case, ts, row) order and
 * the per-case table.  Caller-owned device arrays, each with room for
 * n_events entries (case_off: n_events + 1).  pm4g_prepare fills them; the
 * *_prepared entry points and pm4g_dfg_batched only read them.
 *   case_s[k], act_s[k], ts_s[k]  the k-th event in order
 *   case_code[j]                  the j-th distinct case id, ascending
 *   case_off[j]..case_off[j+1]-1  positions of case j's events
 *   n_cases                       device scalar: number of distinct cases C
 *   status                        device status word of pm4g_prepare
 *   row                           optional (may be NULL): row[k] is the row, in
 *                                 the raw log given to pm4g_prepare, of the k-th
 *                                 event in order -- the permutation of the first
 *                                 formatting step, by which any other column of
 *                                 the caller's dataframe follows the formatted
 *                                 order (other_s[k] = other[row[k]]).  Only
 *                                 pm4g_prepare writes it, and only when it is not
 *                                 NULL (the sort then carries 4 more bytes per
 *                                 event); every other entry point ignores it.
 */
typedef struct {
    int32_t *case_s;
    int32_t *act_s;
    int64_t *ts_s;
    int64_t *case_off;
    int32_t *case_code;
    int64_t *n_cases;
    int32_t *status;
    int64_t n_events;
    int32_t n_activities;
    int32_t *row;
} pm4g_prepared;

/*
 * DFG outputs, Sec. 3 frequency / performance directly-follows graph.
 * Dense row-major tables of A*A cells, cell (x, y) at x*A + y, over all pairs
 * where an event with activity y directly follows one with activity x in the
 * same case:
 *   count     number of such pairs
 *   dt_sum    sum of gaps t_y - t_x, modulo 2^64, as int64
 *   dt_min    minimum gap (INT64_MAX for an empty cell)
 *   dt_max    maximum gap (INT64_MIN for an empty cell)
 *   dt_mean   (double)dt_sum / (double)count, NaN for an empty cell; may be NULL
 * Per-activity counts [A]: start_count (first event of a case), end_count
 * (last event of a case), act_count (all events).
 * Device scalars: n_cases; overflow = 1 iff the exact sum over cases of
 * (t_last - t_first) exceeds INT64_MAX (then some dt_sum may have wrapped);
 * status.
 */
typedef struct {
    int64_t *count;
    int64_t *dt_sum;
    int64_t *dt_min;
    int64_t *dt_max;
    double *dt_mean;
    int64_t *start_count;
    int64_t *end_count;
    int64_t *act_count;
    int64_t *n_cases;
    int32_t *overflow;
    int32_t *status;
} pm4g_dfg_out;

/*
 * Variant outputs, Sec. 3 variant level.  Cases are grouped by their exact
 * activity sequence; variant ids 0..V-1 are ordered by (number of cases
 * descending, representative ascending), the representative being the
 * smallest case id of the variant.  Arrays have room for n_events entries
 * (var_off: n_events + 1), which bounds V and the total sequence length, so
 * no capacity error can occur.
 *   n_variants         device scalar V
 *   var_count[v]       number of cases
 *   var_len[v]         sequence length
 *   var_rep[v]         representative case id
 *   var_off[v]..var_off[v+1]-1   the sequence, in var_acts
 *   case_variant[j]    variant of the j-th distinct case (ascending case id);
 *                      may be NULL
 */
typedef struct {
    int64_t *n_variants;
    int64_t *var_count;
    int32_t *var_len;
    int32_t *var_rep;
    int64_t *var_off;
    int32_t *var_acts;
    int32_t *case_variant;
    int32_t *status;
} pm4g_variants_out;

/*
 * A drill-down view (Sec. 1 drill-down: a filtered part of the log; Sec. 3 event-level
 * timestamp filter and activity-attribute filter).  Event i is kept iff
 * case_lo <= case_id_i < case_hi, t_lo <= timestamp_i <= t_hi and bit
 * activity_i of the view's mask is set; the view's DFG is re-discovered on
 * the kept events (a kept event is paired with the previous kept event of
 * its case).  24 bytes, naturally aligned.
 */
typedef struct {
    int32_t case_lo;
    int32_t case_hi;
    int64_t t_lo;
    int64_t t_hi;
} pm4g_view;

/*
 * Outputs of pm4g_dfg_batched for n_views views over A activities.
 *   edge_off[v]..edge_off[v+1]-1   view v's non-empty DFG cells, ordered by
 *                                  (src, dst): src, dst, count, dt_sum,
 *                                  dt_min, dt_max, dt_mean (mean may be NULL)
 *                                  in arrays of cap_edges entries
 *   start_count, end_count, act_count   [n_views * A], row v for view v
 *   n_events, n_cases                   [n_views] kept events and cases
 *   required   device int64[5]: output cells, internal records, internal run
 *              places ((tile, view) pairs x cell buckets), (tile, view) pairs
 *              and internal aggregated cells the call needed
 *   status     device status word (PM4G_E_CAPACITY if cap_edges was short)
 */
typedef struct {
    int64_t *edge_off;
    int32_t *src;
    int32_t *dst;
    int64_t *count;
    int64_t *dt_sum;
    int64_t *dt_min;
    int64_t *dt_max;
    double *dt_mean;
    int64_t *start_count;
    int64_t *end_count;
    int64_t *act_count;
    int64_t *n_events;
    int64_t *n_cases;
    int64_t cap_edges;
    int64_t *required;
    int32_t *status;
} pm4g_batched_out;

/*
 * Launch shape and internal capacities of pm4g_dfg_batched (NULL or zero
 * fields: defaults).  tile_events is 2048 or 4096 (events of the log staged
 * per block); launch is 0 (the whole call as one persistent cooperative
 * launch on a grid of resident blocks) or 1 (one launch per phase, on the
 * grids emit_blocks and agg_blocks for the walks and the aggregation); the
 * capacities size
 * the workspace: (tile, view) pairs, records (one per kept event) and
 * aggregated cells (before compaction into the output); each pair also holds
 * one run place per bucket of 4096 cells.  descriptor_capacity is ignored
 * (kept for the layout of the struct).
 */
typedef struct {
    int32_t tile_events;
    int32_t emit_blocks;
    int32_t agg_blocks;
    int32_t launch;
    int64_t pair_capacity;
    int64_t record_capacity;
    int64_t descriptor_capacity;
    int64_t cell_capacity;
} pm4g_batched_tuning;

/*
 * Bytes of workspace an operation needs for a log of n_events events and
 * n_activities activities (n_views for PM4G_OP_DFG_BATCHED, else ignored).
 * Returns 0 for invalid arguments.
 */
size_t pm4g_workspace_bytes(int op, int64_t n_events, int32_t n_activities, int32_t n_views);

/*
 * Formats a raw log (Sec. 3, first formatting step and the cases table):
 * writes `out`'s arrays and device scalars.  With PM4G_PRESORTED the order is
 * verified instead of computed (status PM4G_E_NOT_SORTED if it does not
 * hold).  Synchronises `stream` once (twice if a case has more than 2049
 * events).  out->n_events and out->n_activities must equal the log's.
 */
int pm4g_prepare(const pm4g_log *log, const pm4g_prepared *out, void *ws, size_t ws_bytes,
                 void *stream);

/* DFG of a raw log: pm4g_prepare into the workspace, then pm4g_dfg_prepared. */
int pm4g_dfg(const pm4g_log *log, const pm4g_dfg_out *out, void *ws, size_t ws_bytes,
             void *stream);

/* DFG of a prepared log.  Does not synchronise. */
int pm4g_dfg_prepared(const pm4g_prepared *log, const pm4g_dfg_out *out, void *ws,
                      size_t ws_bytes, void *stream);

/* Variants of a raw log: pm4g_prepare into the workspace, then pm4g_variants_prepared. */
int pm4g_variants(const pm4g_log *log, const pm4g_variants_out *out, void *ws, size_t ws_bytes,
                  void *stream);

/* Variants of a prepared log.  Does not synchronise. */
int pm4g_variants_prepared(const pm4g_prepared *log, const pm4g_variants_out *out, void *ws,
                           size_t ws_bytes, void *stream);

/*
 * pm4g_dfg_prepared for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and outputs, with the workspace taken from a
 * library-owned device array of PM4G_NOALLOC_SCRATCH_BYTES bytes instead of
 * a caller's buffer.  The library holds one such array per GPU it runs on
 * until the process ends; the call itself allocates nothing.
 *   - The array belongs to the current device; a non-NULL `stream` must
 *     belong to it too (else PM4G_E_INVALID).
 *   - When pm4g_workspace_bytes(PM4G_OP_DFG_PREPARED, n_events, n_activities,
 *     0) exceeds PM4G_NOALLOC_SCRATCH_BYTES, PM4G_E_WORKSPACE is returned
 *     before anything is enqueued (every n_events fits for n_activities <= 64;
 *     with 512 activities about 6.5 million events fit).
 *   - Every call on one GPU shares that GPU's array and leaves its contents
 *     behind (the kernels clear what must start at zero): calls that overlap
 *     in time on one GPU (other streams or threads) race and must be
 *     serialised by the caller.
 * Does not synchronise.
 */
#define PM4G_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int pm4g_dfg_prepared_noalloc(const pm4g_prepared *log, const pm4g_dfg_out *out, void *stream);

/*
 * DFGs of many drill-down views of one prepared log in one pass over the log
 * (views: device array of n_views records; act_masks: device array of
 * n_views * ceil(A/64) words, bit a of word a/64 of row v selects activity a
 * for view v).  Requires A <= PM4G_BATCHED_MAX_ACTIVITIES.  Does not
 * synchronise: every capacity is checked on the device.  When one is short
 * -- the pair, record or cell capacity of `tuning`, or cap_edges
 * -- out->status becomes PM4G_E_CAPACITY and out->required holds the sizes
 * known at that point (0 for those that are not: the output and cell counts
 * are known only once the records fit): call again with larger capacities
 * until the status is PM4G_OK.  More than 2^32 - 1 kept (event, view) pairs in
 * one call give status PM4G_E_INVALID (split the views).  n_views times the
 * number of 4096-cell buckets of the A*(A+1) cells, ceil(A*(A+1)/4096), must
 * stay below 2^32 (else PM4G_E_INVALID, returned, and a workspace size of 0).
 * With tuning->launch 0 (the default) the call is one cooperative launch of
 * one block per compute unit: its phases meet at grid barriers whose waits
 * are bounded, and a barrier that does not complete within seconds sets
 * out->status to PM4G_E_DEVICE (the outputs are then not valid) instead of
 * hanging; a failed cooperative launch returns PM4G_E_DEVICE.  With launch 1
 * each phase is a launch of its own.  Both give the same bytes.
 */
size_t pm4g_batched_workspace_bytes(int64_t n_events, int32_t n_activities, int32_t n_views,
                                    const pm4g_batched_tuning *tuning);
int pm4g_dfg_batched(const pm4g_prepared *log, const pm4g_view *views, const uint64_t *act_masks,
                     int32_t n_views, const pm4g_batched_out *out, const pm4g_batched_tuning *tuning,
                     void *ws, size_t ws_bytes, void *stream);

/*
 * One drill-down view (device record `view`, device mask of ceil(A/64)
 * words) of a prepared log, materialised as a prepared log of the kept
 * events, in their (case, timestamp, row) order, with its case table
 * (Sec. 3 event-level timestamp filter and activity filter on the formatted
 * log).  out->n_events is the capacity of out's arrays; if the view's case
 * range holds more events, nothing is kept and out->status is
 * PM4G_E_CAPACITY.  The kept count is out->case_off[*out->n_cases], on the
 * device.  The result can be
 * given to pm4g_variants_prepared (which only reads the case ranges).  Does
 * not synchronise.
 */
size_t pm4g_filter_workspace_bytes(int64_t n_events);
int pm4g_filter_view(const pm4g_prepared *log, const pm4g_view *view, const uint64_t *act_mask,
                     const pm4g_prepared *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Filter at the directly-follows level (Sec. 3: events kept or dropped on
 * their activity and that of the previous, or next, event of their case;
 * the paper's example keeps the Insert Fine Notification events whose
 * previous event is Send Fine).  In the log's (case, timestamp, row) order,
 * an event's partner is the previous event of its case (side = 0, pair
 * (partner, event)) or the next one (side = 1, pair (event, partner)); the
 * event matches iff it has a partner and bit src*A + dst of pair_mask
 * (device, ceil(A*A/64) words) is set.  keep = 1 keeps the matching events,
 * keep = 0 the others (events without a partner among them).  The kept
 * events form a prepared log in out (same order, a case table over the
 * cases that keep at least one event); the DFG of out pairs each kept event
 * with the previous kept event of its case.  out->n_events is the capacity:
 * if the kept events exceed it, nothing is written, the output log is empty
 * and out->status is PM4G_E_CAPACITY.  side and keep are 0 or 1, else
 * PM4G_E_INVALID.  Workspace: pm4g_filter_workspace_bytes(log->n_events).
 * Does not synchronise.
 */
int pm4g_filter_df_events(const pm4g_prepared *log, const uint64_t *pair_mask, int32_t side, int32_t keep,
                          const pm4g_prepared *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Cases dataframe (Sec. 3: one row per case with its number of events and its
 * throughput time, the cases-dataframe module).  For the j-th case of a
 * prepared log (its case-table order: ascending case id), n_events_out[j] is
 * its number of events and throughput_out[j] the timestamp of its last event
 * minus that of its first (computed modulo 2^64, read as int64).  Both device
 * arrays (either may be NULL) hold at least log->n_events entries (an upper
 * bound of the case count, which stays on the device).  No workspace; does
 * not synchronise.
 */
int pm4g_cases(const pm4g_prepared *log, int64_t *n_events_out, int64_t *throughput_out, void *stream);

/*
 * Case-level filter (Sec. 3: filtering at the case level on the number of
 * events and the throughput time; cases containing an activity; the DFG
 * module's paths filtering; timestamp filters on whole cases; start and end
 * activity filters; variant filtering).  With first/last the case's first
 * and last event in the (case, timestamp, row) order, a case is kept iff
 * every predicate holds (bounds inclusive):
 *   min_events <= its events <= max_events;
 *   min_throughput <= its throughput time <= max_throughput;
 *   contained in a window: ts(first) >= contain_lo and ts(last) <= contain_hi;
 *   intersecting a window: ts(first) <= meet_hi and ts(last) >= meet_lo
 *     (INT64_MIN / INT64_MAX leave a bound open);
 *   act_mask (device, ceil(A/64) words; NULL: no predicate): one of its
 *     events has an activity whose bit is set;
 *   path_mask (device, ceil(A*A/64) words, bit src*A + dst; NULL: no
 *     predicate): one of its directly-follows pairs has its bit set
 *     (path_keep = 1), or none has (path_keep = 0);
 *   start_mask / end_mask (device, ceil(A/64) words; NULL: no predicate): the
 *     activity of its first / last event has its bit set;
 *   variant_mask (device, ceil(n_variant_bits/64) words; NULL: no
 *     predicate): with v = case_variant[j] for the log's j-th case (device,
 *     as pm4g_variants writes it for the same prepared log), v <
 *     n_variant_bits and bit v is set (variant_keep = 1), or not
 *     (variant_keep = 0).  case_variant must be given with variant_mask.
 * path_keep and variant_keep are 0 or 1, else PM4G_E_INVALID.  The struct
 * itself is read on the host.
 */
typedef struct {
    int64_t min_events;
    int64_t max_events;
    int64_t min_throughput;
    int64_t max_throughput;
    const uint64_t *act_mask;
    const uint64_t *path_mask;
    int32_t path_keep;
    int32_t variant_keep;
    int64_t contain_lo;
    int64_t contain_hi;
    int64_t meet_lo;
    int64_t meet_hi;
    const uint64_t *start_mask;
    const uint64_t *end_mask;
    const int32_t *case_variant;
    const uint64_t *variant_mask;
    int64_t n_variant_bits;
} pm4g_case_filter;

/*
 * The events of the kept cases, as a prepared log of their own (order and
 * case table as in the input; whole cases).  out->n_events is the capacity
 * of out's arrays; if the kept events exceed it, nothing is written and
 * out->status is PM4G_E_CAPACITY.  The kept count is
 * out->case_off[*out->n_cases], on the device.  Does not synchronise.
 */
size_t pm4g_filter_cases_workspace_bytes(int64_t n_events);
int pm4g_filter_cases(const pm4g_prepared *log, const pm4g_case_filter *filter, const pm4g_prepared *out,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * Eventually-follows graph and temporal profile (Sec. 3: the EFG /
 * temporal-profile module, named there without a definition).  For every case
 * and every two of its events i, j with i before j in the (case, timestamp,
 * row) order, cell a_i*A + a_j of the [A*A] device arrays counts the pair and
 * accumulates its gap d = t_j - t_i (an exact unsigned 64-bit value, >= 0 in
 * that order):
 *   count                 number of pairs (the eventually-follows graph);
 *   sum_lo, sum_hi        the exact sum of the gaps, 128-bit (lo, hi words);
 *   sq_lo, sq_hi          the sum of the squared gaps modulo 2^128;
 *   mean (may be NULL)    S / n in FP64 with S converted as hi * 2^64 + lo,
 *                         NaN for an empty cell;
 *   std (may be NULL)     sample standard deviation sqrt(D / n / (n - 1)),
 *                         D = n*Q - S*S evaluated exactly in 256 bits and
 *                         converted to FP64 limb by limb, most significant
 *                         first (x = x * 2^64 + limb); 0 for one pair, NaN
 *                         for none (the temporal profile is (mean, std));
 *   n_pairs               device int64[1]: all pairs, sum of L(L-1)/2;
 *   status                device int32[1]: the input log's status, else 0.
 * mean and std are meaningful while the square sums stay below 2^128.
 * Requires n_activities <= PM4G_EFG_MAX_ACTIVITIES.  The work grows with the
 * number of pairs, not of events.  Does not synchronise.
 */
#define PM4G_EFG_MAX_ACTIVITIES 4096
typedef struct {
    int64_t *count;
    uint64_t *sum_lo;
    uint64_t *sum_hi;
    uint64_t *sq_lo;
    uint64_t *sq_hi;
    double *mean;
    double *std;
    int64_t *n_pairs;
    int32_t *status;
} pm4g_efg_out;

size_t pm4g_efg_workspace_bytes(int64_t n_events, int32_t n_activities);
int pm4g_efg(const pm4g_prepared *log, const pm4g_efg_out *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Sampling (Sec. 3: the sampling module, a sample of the log by a number of
 * cases or of events).  by_events = 0: the k cases (all when k >= their
 * number) whose key SplitMix64(seed, case id) is smallest, with all their
 * events; by_events = 1: the k events whose key SplitMix64(seed, position)
 * is smallest, the position being the event's index in the log's (case,
 * timestamp, row) order.  SplitMix64(seed, x) is the x-th output (x = 0, 1,
 * ...) of the SplitMix64 generator (Steele, Lea and Flood, 2014) started
 * from state seed, the case id taken as its 32-bit pattern; the keys of
 * distinct inputs differ, so the sample is unique and a smaller k gives a
 * subset of a larger one.  The kept events form a prepared log in out (same
 * order, a case table over the cases they belong to).  out->n_events is the
 * capacity: if the kept events exceed it, nothing is written, the output log
 * is empty and out->status is PM4G_E_CAPACITY.  k < 0 or by_events outside
 * {0, 1}: PM4G_E_INVALID.  Does not synchronise.
 */
size_t pm4g_sample_workspace_bytes(int64_t n_events);
int pm4g_sample(const pm4g_prepared *log, int64_t k, uint64_t seed, int32_t by_events, const pm4g_prepared *out,
                void *ws, size_t ws_bytes, void *stream);

/*
 * CSV ingestion (Sec. 2.2: a CSV text of a header row and data rows of values
 * separated by a separator character, parsed by many GPU threads at once into
 * columns).  text: device bytes of the whole file.  Lines end at newlines
 * outside quoted runs (quote characters '"' open and close runs wherever they
 * stand) or at the end of the text; a trailing carriage return is dropped;
 * empty lines are skipped; with has_header the first non-empty line is the
 * header.  Fields are split at `sep` outside quoted runs; a field's value
 * drops the delimiting quotes of its runs and reads a doubled quote inside a
 * run as one quote.  From every data row:
 *   case_code, act_code   the case and activity values (columns case_col,
 *                         act_col, 0-based) coded 0, 1, ... in order of first
 *                         appearance, byte-exact; per code, *_dict_off and
 *                         *_dict_len give the byte range of the raw field
 *                         (quotes included) where the value first appears;
 *   ts                    column ts_col: an integer (optional sign, within
 *                         int64) when ts_iso = 0, else an ISO-8601 date-time
 *                         YYYY-MM-DD[(T| )HH:MM[:SS[(.|,)F]]][Z|+-HH[[:]MM]]
 *                         (F: 1-9 digits; no offset: UTC) in units of
 *                         10^-ts_scale s since 1970-01-01T00:00Z, fraction
 *                         digits below the unit dropped.
 * The counts (n_rows, n_cases, n_acts) and status / bad_row are device
 * int64/int32 words.  A data row with fewer fields than the columns need or a
 * bad timestamp, or a quoted run still open at the end (reported at the last
 * row), returns PM4G_E_PARSE with *bad_row the first such data row (0-based);
 * more data rows than out->capacity returns PM4G_E_CAPACITY; nothing else is
 * valid then.  The case and activity arrays and dictionaries hold
 * out->capacity entries.  sep must not be '"', '\n' or '\r'.  Values are
 * matched through a 64-bit hash and then compared byte by byte; if two
 * different values share a hash, the call repeats with another hash seed.
 * Synchronises the stream (the counts decide the work).
 */
typedef struct {
    int32_t case_col;
    int32_t act_col;
    int32_t ts_col;
    int32_t has_header;
    int32_t ts_iso;
    int32_t ts_scale;
    char sep;
    char reserved[7];
} pm4g_csv_schema;

typedef struct {
    int32_t *case_code;
    int32_t *act_code;
    int64_t *ts;
    int64_t capacity;
    int64_t *n_rows;
    int64_t *case_dict_off;
    int32_t *case_dict_len;
    int64_t *n_cases;
    int64_t *act_dict_off;
    int32_t *act_dict_len;
    int64_t *n_acts;
    int32_t *status;
    int64_t *bad_row;
} pm4g_csv_out;

size_t pm4g_ingest_csv_workspace_bytes(int64_t n_bytes, int64_t capacity);
int pm4g_ingest_csv(const uint8_t *text, int64_t n_bytes, const pm4g_csv_schema *schema, const pm4g_csv_out *out,
                    void *ws, size_t ws_bytes, void *stream);

/*
 * Parquet ingestion (Sec. 2.2: the log as a columnar file the GPU reads
 * directly).  `file` holds a whole Apache Parquet file of n_bytes bytes in
 * device memory; case_col, act_col and ts_col are 0-based columns (leaves) of
 * its flat schema.  Read: uncompressed column chunks, data pages v1 and v2,
 * PLAIN and dictionary-coded values (PLAIN_DICTIONARY / RLE_DICTIONARY),
 * definition levels of optional columns; INT32, INT64 and BYTE_ARRAY case and
 * activity columns, INT32 and INT64 timestamp columns (timestamps are taken
 * as they are stored, in the column's unit).
 * Outputs as pm4g_ingest_csv: the rows' case and activity codes (0, 1, ... in
 * order of first appearance; integers compared by value, byte arrays byte by
 * byte), timestamps, and per code *_dict_off / *_dict_len: the byte range in
 * `file` of the value at the code's first row (integer columns: the value
 * itself in *_dict_off and -1 in *_dict_len).
 * Errors:
 *   - returned before anything runs on the device values: PM4G_E_INVALID
 *     (arguments, a column beyond the schema), PM4G_E_UNSUPPORTED (codec,
 *     physical type, nested or repeated columns, chunks in other files; also
 *     in out->status), PM4G_E_PARSE (a malformed footer), PM4G_E_CAPACITY (more
 *     rows than out->capacity; also in out->status, with *out->n_rows = 0);
 *   - found while decoding, in out->status and returned: PM4G_E_PARSE with
 *     *out->bad_row the smallest row holding a null in one of the three
 *     columns, or -1 for malformed pages; PM4G_E_UNSUPPORTED for other page
 *     encodings.
 * Synchronises the stream (the footer is read on the host; value hashes that
 * collide repeat the matching with another seed).  pm4g_debug_csv_hash_bits
 * applies to its value hashes too.
 */
typedef struct {
    int32_t case_col;
    int32_t act_col;
    int32_t ts_col;
    int32_t reserved;
} pm4g_parquet_schema;

/* Rows of a Parquet file in device memory, from its footer (host int64).
   Synchronises. */
int pm4g_parquet_rows(const uint8_t *file, int64_t n_bytes, int64_t *rows, void *stream);
size_t pm4g_ingest_parquet_workspace_bytes(int64_t n_bytes, int64_t capacity);
int pm4g_ingest_parquet(const uint8_t *file, int64_t n_bytes, const pm4g_parquet_schema *schema,
                        const pm4g_csv_out *out, void *ws, size_t ws_bytes, void *stream);

/* Text for a status code (static storage). */
const char *pm4g_status_string(int code);

/* Description of the calling thread's last failure (thread-local storage). */
const char *pm4g_last_error(void);

/*
 * Test hook for the variant grouping (Sec. 3, variant level): truncates the
 * sequence hash used by the calling thread's later variant calls to `bits`
 * bits (0 or >= 64: the full 64-bit hash), so that hash collisions, which the
 * exact regrouping must resolve, can be forced on small logs.  Results do not
 * depend on it.  Returns the previous setting.
 */
int pm4g_debug_variant_hash_bits(int bits);

/*
 * Test hook for the eventually-follows aggregation: the calling thread's later
 * pm4g_efg calls sum at most `pairs` pairs per pass of a block's LDS table
 * before adding the table into the block's partial slot (0: the full 2^31,
 * which keeps the table's 32-bit counters exact).  Small values exercise the
 * multi-pass accumulation on small logs; results do not depend on it.
 * Returns the previous setting.
 */
int64_t pm4g_debug_efg_pass_pairs(int64_t pairs);

/*
 * Test hook for CSV ingestion: the calling thread's later pm4g_ingest_csv
 * calls truncate the value hashes of their first matching attempt to `bits`
 * bits (0 or >= 64: all 64), so that hash collisions, which the byte-by-byte
 * check detects and a repeat with another seed resolves, can be forced on
 * small texts.  Results do not depend on it.  Returns the previous setting.
 */
int pm4g_debug_csv_hash_bits(int bits);

/*
 * Stage timing for measurement: while enabled (process-wide), every stage of
 * the library records a pair of HIP events on the stream it launches on.
 * pm4g_profile_read() waits for the recorded events, writes per-stage total
 * milliseconds and launch counts for stages 0..n_stages-1 (host arrays, may
 * be NULL) and clears the record.  Stage names: pm4g_profile_stage_name().
 * Timing adds event records between launches; it is off by default.
 */
int pm4g_profile_enable(int on);
int pm4g_profile_read(double *total_ms, int64_t *launches, int n_stages);
const char *pm4g_profile_stage_name(int stage);
int pm4g_profile_stage_count(void);

/* PM4G_ABI_VERSION of the loaded library. */
int pm4g_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PM4G_H */
