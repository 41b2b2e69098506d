/*
 * pm4g_oracle.c -- plain, slow, single-threaded CPU oracle for directly-follows
 * graph (DFG) discovery over a columnar event log (case id, activity, timestamp).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU path is compared
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with the
 * HIP library; it does not include pm4g.h.
 *
 * Every function writes out the plain definition of what the method computes
 * (PM4Py-GPU, Berti, Phan Nghia, van der Aalst, arXiv 2204.04898):
 *
 *   order      Sec. 3, first formatting step: events are ordered by case
 *              identifier, then timestamp, then absolute row index.
 *   shift      Sec. 3, second formatting step: each event sees the activity
 *              and timestamp of the previous event of its case.
 *   DFG        Sec. 3, aggregation at the directly-follows level: the frequency /
 *              performance directly-follows graph.  The paper names no
 *              performance aggregate; here it is the exact int64 count, sum,
 *              min and max of the time gaps, with the FP64 mean sum/count.
 *   endpoints  Sec. 3, start/end activities module, and the event-level
 *              count of each activity's events.
 *   variants   Sec. 3, variant-level aggregation (cases grouped by their
 *              activity sequence, an aggregation of the per-case one).
 *   views      Sec. 1 drill-down (filtered parts of the log), Sec. 3
 *              timestamp filter on events and attribute (activity) filter,
 *              composed as a conjunction; the DFG is re-discovered on the
 *              retained events.
 *   cases      Sec. 3 cases dataframe (events and throughput time per case)
 *              and the case-level filters on it, with paths filtering.
 *   df events  Sec. 3, filtering at the directly-follows level: events kept or
 *              dropped by the pair they form with the previous (or next)
 *              event of their case.
 *   EFG        Sec. 3, eventually-follows graph and temporal profile: every
 *              ordered pair of events of a case, with its gap statistics.
 *   sampling   Sec. 3, sampling module: a sample of k cases or k events.
 *   CSV        Sec. 2.2, ingestion of a CSV text into the columns of a log.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - the row tie-break is the 0-based row index in the caller's arrays;
 *   - a gap is t_next - t_prev computed modulo 2^64 and read as int64; sums
 *     wrap modulo 2^64; min/max compare as signed int64;
 *   - empty DFG cell: count 0, sum 0, min INT64_MAX, max INT64_MIN, mean NaN;
 *   - overflow flag: set iff the sum over cases of (t_last - t_first),
 *     evaluated exactly, exceeds INT64_MAX;
 *   - variants are exact sequence classes, numbered by (count desc,
 *     representative asc) where the representative is the smallest case code;
 *   - a view keeps event i iff case_lo <= c_i < case_hi, t_lo <= t_i <= t_hi
 *     and the activity bit of a_i is set in the mask;
 *   - throughput time = timestamp of the case's last event minus its first;
 *   - paths filtering keeps (or drops) the whole cases that contain a
 *     directly-follows pair of the given set; the case-level predicates
 *     combine as a conjunction, bounds inclusive;
 *   - a case is contained in a time window when its first and last events
 *     are inside it, and intersects it when its [first, last] span overlaps
 *     it; start/end filters look at the first/last event of the case;
 *   - the event-level directly-follows filter matches an event on the pair
 *     with its previous (or next) event in the (case, timestamp, row)
 *     order; the first (last) event of a case has no such pair and never
 *     matches;
 *   - the eventually-follows pairs of a case are all (i, j) with i before j
 *     in that order; the temporal profile of a pair of activities is the
 *     mean and the sample standard deviation of their gaps, from exact
 *     integer sums (see orc_efg);
 *   - a sample of k cases (events) keeps those with the k smallest SplitMix64
 *     keys of (seed, case id) ((seed, position in the formatted log)); the
 *     keys are distinct, so the sample is unique, and a smaller k gives a
 *     subset of a larger one.
 *
 * Status codes: 0 ok, -1 invalid argument, -2 activity out of [0, A),
 * -3 parse error (CSV ingestion).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_E_INVALID -1
#define ORC_E_RANGE -2

typedef struct {
    int32_t c;
    int64_t t;
    int64_t row;
} orc_event;

/* The total order of the first formatting step: (case, timestamp, row). */
static int cmp_event(const void *pa, const void *pb)
{
    const orc_event *a = (const orc_event *)pa, *b = (const orc_event *)pb;
    if (a->c != b->c) return a->c < b->c ? -1 : 1;
    if (a->t != b->t) return a->t < b->t ? -1 : 1;
    if (a->row != b->row) return a->row < b->row ? -1 : 1;
    return 0;
}

static int check_acts(int64_t n, const int32_t *act, int32_t A)
{
    for (int64_t i = 0; i < n; i++)
        if (act[i] < 0 || act[i] >= A) return ORC_E_RANGE;
    return ORC_OK;
}

/* Returns a malloc'ed array of the n events in (case, ts, row) order. */
static orc_event *sorted_events(int64_t n, const int32_t *case_id, const int64_t *ts)
{
    orc_event *e = (orc_event *)malloc((size_t)(n > 0 ? n : 1) * sizeof(orc_event));
    if (!e) return NULL;
    for (int64_t i = 0; i < n; i++) {
        e[i].c = case_id[i];
        e[i].t = ts[i];
        e[i].row = i;
    }
    qsort(e, (size_t)n, sizeof(orc_event), cmp_event);
    return e;
}

/*
 * orc_prepare: the formatted log.  Writes, for k = 0..n-1 in (case, ts, row)
 * order, the row, case, activity and timestamp of the k-th event, and the case
 * table: case_code[j] is the j-th distinct case (ascending), its events are
 * positions case_off[j] .. case_off[j+1]-1.  Any output pointer may be NULL.
 */
int orc_prepare(int64_t n, const int32_t *case_id, const int32_t *act, const int64_t *ts,
                int32_t A, int64_t *row_out, int32_t *case_s, int32_t *act_s, int64_t *ts_s,
                int64_t *case_off, int32_t *case_code, int64_t *n_cases)
{
    if (n < 0 || A < 1) return ORC_E_INVALID;
    if (check_acts(n, act, A)) return ORC_E_RANGE;
    orc_event *e = sorted_events(n, case_id, ts);
    if (!e) return ORC_E_INVALID;
    int64_t C = 0;
    for (int64_t k = 0; k < n; k++) {
        int64_t r = e[k].row;
        if (row_out) row_out[k] = r;
        if (case_s) case_s[k] = e[k].c;
        if (act_s) act_s[k] = act[r];
        if (ts_s) ts_s[k] = ts[r];
        if (k == 0 || e[k].c != e[k - 1].c) {
            if (case_off) case_off[C] = k;
            if (case_code) case_code[C] = e[k].c;
            C++;
        }
    }
    if (case_off) case_off[C] = n;
    if (n_cases) *n_cases = C;
    free(e);
    return ORC_OK;
}

/*
 * orc_dfg: frequency and performance DFG, start/end/activity counts.
 * count, dt_sum, dt_min, dt_max, dt_mean are [A*A] row-major (src*A + dst);
 * start_count, end_count, act_count are [A].  perm (optional, [n]) receives
 * the row of the k-th event in order.
 */
int orc_dfg(int64_t n, const int32_t *case_id, const int32_t *act, const int64_t *ts,
            int32_t A, int64_t *perm, int64_t *count, int64_t *dt_sum, int64_t *dt_min,
            int64_t *dt_max, double *dt_mean, int64_t *start_count, int64_t *end_count,
            int64_t *act_count, int64_t *n_cases, int32_t *overflow)
{
    if (n < 0 || A < 1) return ORC_E_INVALID;
    if (check_acts(n, act, A)) return ORC_E_RANGE;
    const int64_t cells = (int64_t)A * A;
    for (int64_t x = 0; x < cells; x++) {
        count[x] = 0;
        dt_sum[x] = 0;
        dt_min[x] = INT64_MAX;
        dt_max[x] = INT64_MIN;
    }
    for (int32_t a = 0; a < A; a++) start_count[a] = end_count[a] = act_count[a] = 0;

    orc_event *e = sorted_events(n, case_id, ts);
    if (!e) return ORC_E_INVALID;

    int64_t C = 0;
    unsigned __int128 total_span = 0;   /* exact sum over cases of t_last - t_first */
    int64_t case_first_t = 0;
    for (int64_t k = 0; k < n; k++) {
        int64_t r = e[k].row;
        int32_t a = act[r];
        if (perm) perm[k] = r;
        act_count[a] += 1;
        int new_case = (k == 0) || (e[k].c != e[k - 1].c);
        if (new_case) {
            if (k > 0) {
                /* close the previous case: its last event is k-1 */
                end_count[act[e[k - 1].row]] += 1;
                total_span += (unsigned __int128)((uint64_t)e[k - 1].t - (uint64_t)case_first_t);
            }
            start_count[a] += 1;
            case_first_t = e[k].t;
            C++;
        } else {
            /* event k directly follows event k-1 of the same case */
            int32_t x = act[e[k - 1].row];
            int64_t cell = (int64_t)x * A + a;
            uint64_t gap_u = (uint64_t)e[k].t - (uint64_t)e[k - 1].t;
            int64_t gap = (int64_t)gap_u;
            count[cell] += 1;
            dt_sum[cell] = (int64_t)((uint64_t)dt_sum[cell] + gap_u);
            if (gap < dt_min[cell]) dt_min[cell] = gap;
            if (gap > dt_max[cell]) dt_max[cell] = gap;
        }
    }
    if (n > 0) {
        end_count[act[e[n - 1].row]] += 1;
        total_span += (unsigned __int128)((uint64_t)e[n - 1].t - (uint64_t)case_first_t);
    }
    /* performance DFG mean: one int64 -> double conversion of each operand and
       one IEEE division; empty cells get NaN */
    for (int64_t x = 0; x < cells; x++)
        dt_mean[x] = count[x] > 0 ? (double)dt_sum[x] / (double)count[x] : NAN;
    *n_cases = C;
    *overflow = total_span > (unsigned __int128)INT64_MAX ? 1 : 0;
    free(e);
    return ORC_OK;
}

/* ---- variants -------------------------------------------------------- */

typedef struct {
    int32_t code;      /* case code */
    int64_t off, len;  /* its events in the ordered activity array */
} orc_case;

/* qsort has no context argument; one per thread, so that concurrent calls
   from several host threads do not share it */
static _Thread_local const int32_t *g_seq_acts;

/* Lexicographic order of activity sequences, a shorter prefix first. */
static int cmp_case_seq(const void *pa, const void *pb)
{
    const orc_case *a = (const orc_case *)pa, *b = (const orc_case *)pb;
    int64_t m = a->len < b->len ? a->len : b->len;
    for (int64_t k = 0; k < m; k++) {
        int32_t x = g_seq_acts[a->off + k], y = g_seq_acts[b->off + k];
        if (x != y) return x < y ? -1 : 1;
    }
    if (a->len != b->len) return a->len < b->len ? -1 : 1;
    return 0;
}

static int same_seq(const orc_case *a, const orc_case *b)
{
    if (a->len != b->len) return 0;
    return memcmp(g_seq_acts + a->off, g_seq_acts + b->off, (size_t)a->len * sizeof(int32_t)) == 0;
}

typedef struct {
    int64_t first, size;   /* index range in the sequence-sorted case array */
    int64_t n;             /* number of cases */
    int32_t rep;           /* smallest case code */
} orc_class;

static int cmp_class(const void *pa, const void *pb)
{
    const orc_class *a = (const orc_class *)pa, *b = (const orc_class *)pb;
    if (a->n != b->n) return a->n > b->n ? -1 : 1;     /* count descending */
    if (a->rep != b->rep) return a->rep < b->rep ? -1 : 1;   /* rep ascending */
    return 0;
}

static int cmp_case_code(const void *pa, const void *pb)
{
    const orc_case *a = (const orc_case *)pa, *b = (const orc_case *)pb;
    return a->code < b->code ? -1 : (a->code > b->code ? 1 : 0);
}

/*
 * orc_variants: exact trace variants.
 * Outputs (caller sizes them by n, which bounds both V and C):
 *   n_variants                     V
 *   var_count[V], var_len[V], var_rep[V]
 *   var_off[V+1], var_acts[sum of lengths]   CSR of the sequences
 *   case_code[C]                   distinct cases ascending
 *   case_variant[C]                variant id of case_code[j]
 *   n_cases                        C
 */
int orc_variants(int64_t n, const int32_t *case_id, const int32_t *act, const int64_t *ts,
                 int32_t A, int64_t *n_variants, int64_t *var_count, int32_t *var_len,
                 int32_t *var_rep, int64_t *var_off, int32_t *var_acts, int32_t *case_code,
                 int32_t *case_variant, int64_t *n_cases)
{
    if (n < 0 || A < 1) return ORC_E_INVALID;
    if (check_acts(n, act, A)) return ORC_E_RANGE;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *acts_sorted = (int32_t *)malloc(nn * sizeof(int32_t));
    int64_t *off = (int64_t *)malloc((nn + 1) * sizeof(int64_t));
    int32_t *codes = (int32_t *)malloc(nn * sizeof(int32_t));
    int64_t C = 0;
    int rc = orc_prepare(n, case_id, act, ts, A, NULL, NULL, acts_sorted, NULL, off, codes, &C);
    if (rc) { free(acts_sorted); free(off); free(codes); return rc; }

    orc_case *cs = (orc_case *)malloc((size_t)(C > 0 ? C : 1) * sizeof(orc_case));
    for (int64_t j = 0; j < C; j++) {
        cs[j].code = codes[j];
        cs[j].off = off[j];
        cs[j].len = off[j + 1] - off[j];
    }
    /* group: sort the cases by their sequence, equal sequences become adjacent */
    g_seq_acts = acts_sorted;
    qsort(cs, (size_t)C, sizeof(orc_case), cmp_case_seq);

    orc_class *cl = (orc_class *)malloc((size_t)(C > 0 ? C : 1) * sizeof(orc_class));
    int64_t V = 0;
    for (int64_t j = 0; j < C; j++) {
        if (j == 0 || !same_seq(&cs[j - 1], &cs[j])) {
            cl[V].first = j;
            cl[V].size = 0;
            cl[V].rep = cs[j].code;
            V++;
        }
        orc_class *k = &cl[V - 1];
        k->size += 1;
        if (cs[j].code < k->rep) k->rep = cs[j].code;
    }
    for (int64_t v = 0; v < V; v++) cl[v].n = cl[v].size;
    qsort(cl, (size_t)V, sizeof(orc_class), cmp_class);

    /* emit: CSR of sequences, and each case's variant id */
    int64_t pos = 0;
    for (int64_t v = 0; v < V; v++) {
        const orc_case *first = &cs[cl[v].first];
        var_count[v] = cl[v].n;
        var_len[v] = (int32_t)first->len;
        var_rep[v] = cl[v].rep;
        var_off[v] = pos;
        memcpy(var_acts + pos, acts_sorted + first->off, (size_t)first->len * sizeof(int32_t));
        pos += first->len;
    }
    var_off[V] = pos;
    /* case_variant in ascending case-code order */
    int32_t *vid_of_seqpos = (int32_t *)malloc((size_t)(C > 0 ? C : 1) * sizeof(int32_t));
    for (int64_t v = 0; v < V; v++)
        for (int64_t j = cl[v].first; j < cl[v].first + cl[v].size; j++) vid_of_seqpos[j] = (int32_t)v;
    /* carry the ids along (in the no longer needed len field) while putting
       the cases back in code order */
    for (int64_t j = 0; j < C; j++) cs[j].len = vid_of_seqpos[j];
    qsort(cs, (size_t)C, sizeof(orc_case), cmp_case_code);
    for (int64_t j = 0; j < C; j++) {
        case_code[j] = cs[j].code;
        case_variant[j] = (int32_t)cs[j].len;
    }
    *n_variants = V;
    *n_cases = C;
    free(vid_of_seqpos);
    free(cl);
    free(cs);
    free(acts_sorted);
    free(off);
    free(codes);
    return ORC_OK;
}

/* ---- views ---------------------------------------------------------- */

/*
 * orc_view: the DFG of a drill-down view.  The retained events are
 *   R = { i : case_lo <= c_i < case_hi, t_lo <= t_i <= t_hi, bit a_i of mask set },
 * kept in their original row order (so the row tie-break is unchanged); the
 * DFG, endpoints and case count are then those of R as a log of its own.
 * mask has ceil(A/64) words; bit a is (mask[a/64] >> (a%64)) & 1.
 * n_events receives |R|.
 */
int orc_view(int64_t n, const int32_t *case_id, const int32_t *act, const int64_t *ts,
             int32_t A, int32_t case_lo, int32_t case_hi, int64_t t_lo, int64_t t_hi,
             const uint64_t *mask, int64_t *count, int64_t *dt_sum, int64_t *dt_min,
             int64_t *dt_max, double *dt_mean, int64_t *start_count, int64_t *end_count,
             int64_t *act_count, int64_t *n_cases, int32_t *overflow, int64_t *n_events)
{
    if (n < 0 || A < 1) return ORC_E_INVALID;
    if (check_acts(n, act, A)) return ORC_E_RANGE;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *rc_ = (int32_t *)malloc(nn * sizeof(int32_t));
    int32_t *ra = (int32_t *)malloc(nn * sizeof(int32_t));
    int64_t *rt = (int64_t *)malloc(nn * sizeof(int64_t));
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t a = act[i];
        int keep = case_id[i] >= case_lo && case_id[i] < case_hi && ts[i] >= t_lo && ts[i] <= t_hi &&
                   ((mask[a / 64] >> (a % 64)) & 1u);
        if (keep) {
            rc_[m] = case_id[i];
            ra[m] = a;
            rt[m] = ts[i];
            m++;
        }
    }
    int r = orc_dfg(m, rc_, ra, rt, A, NULL, count, dt_sum, dt_min, dt_max, dt_mean, start_count,
                    end_count, act_count, n_cases, overflow);
    *n_events = m;
    free(rc_);
    free(ra);
    free(rt);
    return r;
}

/*
 * orc_view_formatted: the same view, answered from a log already in the
 * (case, timestamp, row) order (the output of orc_prepare: case_s, act_s, ts_s
 * of n events, and its case table case_code[C] ascending with case_off[C+1]).
 * Sec. 3: the log is formatted once and every later operation works on the
 * formatted log; removing events keeps the others in that order, so the
 * retained events of the cases in [case_lo, case_hi) are met in order by one
 * scan of those cases' positions.  Walking them, a retained event directly
 * follows the previous retained event of the same case.  Same outputs as
 * orc_view.
 */
int orc_view_formatted(int64_t n, const int32_t *case_s, const int32_t *act_s, const int64_t *ts_s,
                       int64_t C, const int64_t *case_off, const int32_t *case_code, int32_t A,
                       int32_t case_lo, int32_t case_hi, int64_t t_lo, int64_t t_hi,
                       const uint64_t *mask, int64_t *count, int64_t *dt_sum, int64_t *dt_min,
                       int64_t *dt_max, double *dt_mean, int64_t *start_count, int64_t *end_count,
                       int64_t *act_count, int64_t *n_cases, int32_t *overflow, int64_t *n_events)
{
    if (n < 0 || A < 1 || C < 0 || C > n || case_off[0] != 0 || case_off[C] != n) return ORC_E_INVALID;
    const int64_t cells = (int64_t)A * A;
    for (int64_t x = 0; x < cells; x++) {
        count[x] = 0;
        dt_sum[x] = 0;
        dt_min[x] = INT64_MAX;
        dt_max[x] = INT64_MIN;
    }
    for (int32_t a = 0; a < A; a++) start_count[a] = end_count[a] = act_count[a] = 0;

    /* first case with code >= case_lo, then the first with code >= case_hi
       (binary searches over the ascending case codes) */
    int64_t lo = 0, hi = C;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (case_code[mid] < case_lo) lo = mid + 1; else hi = mid;
    }
    int64_t j0 = lo;
    hi = C;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (case_code[mid] < case_hi) lo = mid + 1; else hi = mid;
    }
    int64_t j1 = case_lo < case_hi ? lo : j0;

    int64_t kept = 0, cases_seen = 0;
    unsigned __int128 total_span = 0;
    for (int64_t j = j0; j < j1; j++) {
        int64_t prev = -1, first = -1;      /* positions of retained events of this case */
        for (int64_t k = case_off[j]; k < case_off[j + 1]; k++) {
            int32_t a = act_s[k];
            if (case_s[k] != case_code[j]) return ORC_E_INVALID;   /* not the case table of this log */
            if (a < 0 || a >= A) return ORC_E_RANGE;     /* only the scanned slice is checked */
            if (ts_s[k] < t_lo || ts_s[k] > t_hi || !((mask[a / 64] >> (a % 64)) & 1u)) continue;
            kept++;
            act_count[a] += 1;
            if (prev < 0) {
                first = k;
                start_count[a] += 1;
            } else {
                int64_t cell = (int64_t)act_s[prev] * A + a;
                uint64_t gap_u = (uint64_t)ts_s[k] - (uint64_t)ts_s[prev];
                int64_t gap = (int64_t)gap_u;
                count[cell] += 1;
                dt_sum[cell] = (int64_t)((uint64_t)dt_sum[cell] + gap_u);
                if (gap < dt_min[cell]) dt_min[cell] = gap;
                if (gap > dt_max[cell]) dt_max[cell] = gap;
            }
            prev = k;
        }
        if (prev >= 0) {
            end_count[act_s[prev]] += 1;
            total_span += (unsigned __int128)((uint64_t)ts_s[prev] - (uint64_t)ts_s[first]);
            cases_seen++;
        }
    }
    for (int64_t x = 0; x < cells; x++)
        dt_mean[x] = count[x] > 0 ? (double)dt_sum[x] / (double)count[x] : NAN;
    *n_cases = cases_seen;
    *overflow = total_span > (unsigned __int128)INT64_MAX ? 1 : 0;
    *n_events = kept;
    return ORC_OK;
}

/* ---- cases dataframe and case-level filters -------------------------- */

/*
 * orc_cases: the cases dataframe (Sec. 3: third formatting step and the
 * cases-dataframe module).  For the j-th case in ascending case order: its
 * code, its number of events, and its throughput time, the timestamp of its
 * last event minus that of its first in the (case, timestamp, row) order
 * (computed modulo 2^64 and read as int64, like every gap here).  Any output
 * may be NULL.
 */
int orc_cases(int64_t n, const int32_t *case_id, const int32_t *act, const int64_t *ts, int32_t A,
              int32_t *case_code, int64_t *n_events, int64_t *throughput, int64_t *n_cases)
{
    if (n < 0 || A < 1) return ORC_E_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int64_t *ts_s = (int64_t *)malloc(nn * sizeof(int64_t));
    int64_t *off = (int64_t *)malloc((nn + 1) * sizeof(int64_t));
    int32_t *code = (int32_t *)malloc(nn * sizeof(int32_t));
    int64_t C = 0;
    int r = orc_prepare(n, case_id, act, ts, A, NULL, NULL, NULL, ts_s, off, code, &C);
    if (r == ORC_OK) {
        for (int64_t j = 0; j < C; j++) {
            int64_t first = off[j], last = off[j + 1] - 1;
            if (case_code) case_code[j] = code[j];
            if (n_events) n_events[j] = off[j + 1] - off[j];
            if (throughput) throughput[j] = (int64_t)((uint64_t)ts_s[last] - (uint64_t)ts_s[first]);
        }
        if (n_cases) *n_cases = C;
    }
    free(ts_s);
    free(off);
    free(code);
    return r;
}

/*
 * orc_filter_cases: case-level filtering (Sec. 3: aggregations / filtering at
 * the case level; the cases-dataframe module's filters on the number of
 * events and the throughput time; the DFG module's paths filtering; the
 * timestamp filters on whole cases; the start/end-activity and variant
 * filters).  bounds[8] = {min_events, max_events, min_thr, max_thr,
 * contain_lo, contain_hi, meet_lo, meet_hi}; with first/last = the case's
 * first and last event in the (case, timestamp, row) order, a case is kept
 * iff every predicate holds:
 *   min_events <= its number of events <= max_events;
 *   min_thr <= its throughput time <= max_thr;
 *   contained in the window: ts(first) >= contain_lo and ts(last) <= contain_hi;
 *   intersecting the window: ts(first) <= meet_hi and ts(last) >= meet_lo;
 *   act_mask (ceil(A/64) words, may be NULL): one of its events has an
 *     activity of the set;
 *   path_mask (ceil(A*A/64) words, bit src*A+dst, may be NULL): one of its
 *     directly-follows pairs is in the set (path_keep != 0), or none is
 *     (path_keep == 0);
 *   start_mask / end_mask (ceil(A/64) words, may be NULL): the activity of
 *     its first / last event is in the set;
 *   variant_mask (may be NULL; n_variant_bits bits over the variant ids of
 *     orc_variants): its variant is in the set (variant_keep != 0), or is not
 *     (variant_keep == 0).
 * The kept cases' events are written in (case, timestamp, row) order; n_out
 * receives their number and n_cases_out the number of kept cases.
 */
int orc_filter_cases(int64_t n, const int32_t *case_id, const int32_t *act, const int64_t *ts, int32_t A,
                     const int64_t *bounds, const uint64_t *act_mask, const uint64_t *path_mask,
                     int32_t path_keep, const uint64_t *start_mask, const uint64_t *end_mask,
                     const uint64_t *variant_mask, int64_t n_variant_bits, int32_t variant_keep,
                     int32_t *case_out, int32_t *act_out, int64_t *ts_out, int64_t *n_out,
                     int64_t *n_cases_out)
{
    if (n < 0 || A < 1 || !bounds) return ORC_E_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *case_s = (int32_t *)malloc(nn * sizeof(int32_t));
    int32_t *act_s = (int32_t *)malloc(nn * sizeof(int32_t));
    int64_t *ts_s = (int64_t *)malloc(nn * sizeof(int64_t));
    int64_t *off = (int64_t *)malloc((nn + 1) * sizeof(int64_t));
    int32_t *cvar = NULL;
    int64_t C = 0;
    int r = orc_prepare(n, case_id, act, ts, A, NULL, case_s, act_s, ts_s, off, NULL, &C);
    if (r == ORC_OK && variant_mask) {
        cvar = (int32_t *)malloc(nn * sizeof(int32_t));
        int64_t *vc = (int64_t *)malloc(nn * sizeof(int64_t));
        int32_t *vl = (int32_t *)malloc(nn * sizeof(int32_t));
        int32_t *vr = (int32_t *)malloc(nn * sizeof(int32_t));
        int64_t *vo = (int64_t *)malloc((nn + 1) * sizeof(int64_t));
        int32_t *va = (int32_t *)malloc(nn * sizeof(int32_t));
        int32_t *cc = (int32_t *)malloc(nn * sizeof(int32_t));
        int64_t V = 0, C2 = 0;
        r = orc_variants(n, case_id, act, ts, A, &V, vc, vl, vr, vo, va, cc, cvar, &C2);
        free(vc);
        free(vl);
        free(vr);
        free(vo);
        free(va);
        free(cc);
    }
    int64_t m = 0, kc = 0;
    if (r == ORC_OK) {
        for (int64_t j = 0; j < C; j++) {
            int64_t first = off[j], end = off[j + 1];
            int64_t events = end - first;
            int64_t t0 = ts_s[first], t1 = ts_s[end - 1];
            int64_t thr = (int64_t)((uint64_t)t1 - (uint64_t)t0);
            int keep = events >= bounds[0] && events <= bounds[1] && thr >= bounds[2] && thr <= bounds[3] &&
                       t0 >= bounds[4] && t1 <= bounds[5] && t0 <= bounds[7] && t1 >= bounds[6];
            if (keep && act_mask) {
                int has = 0;
                for (int64_t k = first; k < end; k++)
                    if ((act_mask[act_s[k] / 64] >> (act_s[k] % 64)) & 1u) has = 1;
                keep = has;
            }
            if (keep && path_mask) {
                int has = 0;
                for (int64_t k = first + 1; k < end; k++) {
                    int64_t cell = (int64_t)act_s[k - 1] * A + act_s[k];
                    if ((path_mask[cell / 64] >> (cell % 64)) & 1u) has = 1;
                }
                keep = path_keep ? has : !has;
            }
            if (keep && start_mask) keep = (start_mask[act_s[first] / 64] >> (act_s[first] % 64)) & 1u;
            if (keep && end_mask) keep = (end_mask[act_s[end - 1] / 64] >> (act_s[end - 1] % 64)) & 1u;
            if (keep && variant_mask) {
                int64_t v = cvar[j];
                int in = v < n_variant_bits && ((variant_mask[v / 64] >> (v % 64)) & 1u);
                keep = variant_keep ? in : !in;
            }
            if (!keep) continue;
            for (int64_t k = first; k < end; k++) {
                if (case_out) case_out[m] = case_s[k];
                if (act_out) act_out[m] = act_s[k];
                if (ts_out) ts_out[m] = ts_s[k];
                m++;
            }
            kc++;
        }
    }
    if (n_out) *n_out = m;
    if (n_cases_out) *n_cases_out = kc;
    free(case_s);
    free(act_s);
    free(ts_s);
    free(off);
    free(cvar);
    return r;
}

/*
 * orc_filter_df_events: filtering at the directly-follows level (Sec. 3: an
 * event is kept or dropped on its own activity together with that of the
 * previous, or the next, event of its case).  For each event in the (case,
 * timestamp, row) order, its partner is the previous event of its case
 * (side == 0, pair (partner, event)) or the next one (side == 1, pair
 * (event, partner)).  The event matches iff it has a partner and bit
 * src*A + dst of path_mask (ceil(A*A/64) words) is set for the pair.  keep
 * != 0 keeps the matching events, keep == 0 keeps the others (events with no
 * partner among them).  The kept events are written in that order; n_out
 * receives their number and n_cases_out the number of distinct cases among
 * them.
 */
int orc_filter_df_events(int64_t n, const int32_t *case_id, const int32_t *act, const int64_t *ts, int32_t A,
                         const uint64_t *path_mask, int32_t side, int32_t keep, int32_t *case_out,
                         int32_t *act_out, int64_t *ts_out, int64_t *n_out, int64_t *n_cases_out)
{
    if (n < 0 || A < 1 || !path_mask || (side != 0 && side != 1)) return ORC_E_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *case_s = (int32_t *)malloc(nn * sizeof(int32_t));
    int32_t *act_s = (int32_t *)malloc(nn * sizeof(int32_t));
    int64_t *ts_s = (int64_t *)malloc(nn * sizeof(int64_t));
    int64_t C = 0;
    int r = orc_prepare(n, case_id, act, ts, A, NULL, case_s, act_s, ts_s, NULL, NULL, &C);
    int64_t m = 0, kc = 0, last = -1;   /* last: sorted position of the previous kept event */
    if (r == ORC_OK) {
        for (int64_t k = 0; k < n; k++) {
            int match = 0;
            if (side == 0 && k > 0 && case_s[k - 1] == case_s[k]) {
                int64_t cell = (int64_t)act_s[k - 1] * A + act_s[k];
                match = (int)((path_mask[cell / 64] >> (cell % 64)) & 1u);
            }
            if (side == 1 && k + 1 < n && case_s[k + 1] == case_s[k]) {
                int64_t cell = (int64_t)act_s[k] * A + act_s[k + 1];
                match = (int)((path_mask[cell / 64] >> (cell % 64)) & 1u);
            }
            if (keep ? !match : match) continue;
            if (last < 0 || case_s[last] != case_s[k]) kc++;
            last = k;
            if (case_out) case_out[m] = case_s[k];
            if (act_out) act_out[m] = act_s[k];
            if (ts_out) ts_out[m] = ts_s[k];
            m++;
        }
    }
    if (n_out) *n_out = m;
    if (n_cases_out) *n_cases_out = kc;
    free(case_s);
    free(act_s);
    free(ts_s);
    return r;
}

/* ---- eventually-follows graph and temporal profile ----------------------- */

typedef unsigned __int128 orc_u128;

/* A 256-bit unsigned integer as four 64-bit limbs, least significant first. */
typedef struct {
    uint64_t w[4];
} orc_u256;

static orc_u256 u256_mul_128_128(orc_u128 a, orc_u128 b)
{
    /* schoolbook product of the two 64-bit halves */
    uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64), b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
    orc_u128 p00 = (orc_u128)a0 * b0, p01 = (orc_u128)a0 * b1, p10 = (orc_u128)a1 * b0, p11 = (orc_u128)a1 * b1;
    orc_u256 r;
    orc_u128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
    r.w[0] = (uint64_t)p00;
    r.w[1] = (uint64_t)mid;
    orc_u128 hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + (uint64_t)p11;
    r.w[2] = (uint64_t)hi;
    r.w[3] = (uint64_t)((hi >> 64) + (p11 >> 64));
    return r;
}

static orc_u256 u256_sub(orc_u256 a, orc_u256 b)
{
    orc_u256 r;
    uint64_t borrow = 0;
    for (int k = 0; k < 4; k++) {
        orc_u128 d = (orc_u128)a.w[k] - b.w[k] - borrow;
        r.w[k] = (uint64_t)d;
        borrow = (uint64_t)(d >> 64) ? 1 : 0;
    }
    return r;
}

/* Fixed rounding sequence: Horner over the limbs, most significant first. */
static double u256_to_double(orc_u256 a)
{
    const double two64 = 18446744073709551616.0;
    double x = (double)a.w[3];
    x = x * two64 + (double)a.w[2];
    x = x * two64 + (double)a.w[1];
    x = x * two64 + (double)a.w[0];
    return x;
}

static double u128_to_double(orc_u128 a)
{
    const double two64 = 18446744073709551616.0;
    return (double)(uint64_t)(a >> 64) * two64 + (double)(uint64_t)a;
}

/*
 * orc_efg: eventually-follows graph and temporal profile (Sec. 3, EFG /
 * temporal-profile module; the paper names them without a definition).  For
 * every case and every two of its events i, j with i before j in the (case,
 * timestamp, row) order, cell a_i*A + a_j counts the pair and accumulates the
 * gap d = t_j - t_i (>= 0 in that order, taken as an exact unsigned 64-bit
 * value).  Per cell:
 *   count             number of pairs;
 *   sum_lo, sum_hi    the exact sum of the gaps as a 128-bit integer;
 *   sq_lo, sq_hi      the sum of the squared gaps modulo 2^128 (exact below);
 *   mean              S / n in FP64, S converted as hi * 2^64 + lo; NaN when
 *                     the cell is empty;
 *   std               sample standard deviation sqrt(D / n / (n - 1)) with
 *                     D = n*Q - S*S evaluated exactly in 256 bits and
 *                     converted by the fixed sequence above; 0 for one pair,
 *                     NaN for none.
 * mean and std may be NULL.  n_pairs receives the total number of pairs.
 */
int orc_efg(int64_t n, const int32_t *case_id, const int32_t *act, const int64_t *ts, int32_t A,
            int64_t *count, uint64_t *sum_lo, uint64_t *sum_hi, uint64_t *sq_lo, uint64_t *sq_hi,
            double *mean, double *std_out, int64_t *n_pairs)
{
    if (n < 0 || A < 1 || !count || !sum_lo || !sum_hi || !sq_lo || !sq_hi) return ORC_E_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    size_t cells = (size_t)A * (size_t)A;
    int32_t *case_s = (int32_t *)malloc(nn * sizeof(int32_t));
    int32_t *act_s = (int32_t *)malloc(nn * sizeof(int32_t));
    int64_t *ts_s = (int64_t *)malloc(nn * sizeof(int64_t));
    int64_t *off = (int64_t *)malloc((nn + 1) * sizeof(int64_t));
    orc_u128 *S = (orc_u128 *)calloc(cells, sizeof(orc_u128));
    orc_u128 *Q = (orc_u128 *)calloc(cells, sizeof(orc_u128));
    int64_t C = 0, pairs = 0;
    int r = orc_prepare(n, case_id, act, ts, A, NULL, case_s, act_s, ts_s, off, NULL, &C);
    for (size_t k = 0; k < cells; k++) count[k] = 0;
    if (r == ORC_OK) {
        for (int64_t c = 0; c < C; c++) {
            for (int64_t i = off[c]; i < off[c + 1]; i++) {
                for (int64_t j = i + 1; j < off[c + 1]; j++) {
                    size_t cell = (size_t)act_s[i] * (size_t)A + (size_t)act_s[j];
                    uint64_t d = (uint64_t)ts_s[j] - (uint64_t)ts_s[i];
                    count[cell] += 1;
                    S[cell] += d;
                    Q[cell] += (orc_u128)d * d;
                    pairs++;
                }
            }
        }
    }
    for (size_t k = 0; k < cells; k++) {
        sum_lo[k] = (uint64_t)S[k];
        sum_hi[k] = (uint64_t)(S[k] >> 64);
        sq_lo[k] = (uint64_t)Q[k];
        sq_hi[k] = (uint64_t)(Q[k] >> 64);
        int64_t m = count[k];
        if (mean) mean[k] = m > 0 ? u128_to_double(S[k]) / (double)m : NAN;
        if (std_out) {
            if (m == 0) {
                std_out[k] = NAN;
            } else if (m == 1) {
                std_out[k] = 0.0;
            } else {
                orc_u256 nq = u256_mul_128_128((orc_u128)(uint64_t)m, Q[k]);
                orc_u256 ss = u256_mul_128_128(S[k], S[k]);
                double D = u256_to_double(u256_sub(nq, ss));
                std_out[k] = sqrt(D / (double)m / (double)(m - 1));
            }
        }
    }
    if (n_pairs) *n_pairs = pairs;
    free(case_s);
    free(act_s);
    free(ts_s);
    free(off);
    free(S);
    free(Q);
    return r;
}

/* ---- sampling -------------------------------------------------------------- */

/*
 * orc_splitmix: the x-th output (x = 0, 1, ...) of the SplitMix64 generator
 * (Steele, Lea and Flood, OOPSLA 2014) started from state `seed`: the state
 * advances by the odd constant 0x9E3779B97F4A7C15 per output and each output
 * is the state passed through the published variant-13 mixer.  Distinct x
 * give distinct outputs (every step is a bijection of 64-bit words).
 */
uint64_t orc_splitmix(uint64_t seed, uint64_t x)
{
    uint64_t z = seed + (x + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    uint64_t key;
    int64_t idx;
} orc_keyed;

static int cmp_keyed(const void *pa, const void *pb)
{
    const orc_keyed *a = (const orc_keyed *)pa, *b = (const orc_keyed *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/*
 * orc_sample: the sampling module (Sec. 3: a sample of the log by a number
 * of cases or of events).  by_events == 0: the k cases whose key
 * orc_splitmix(seed, case id as a 32-bit pattern) is smallest (all cases
 * when k >= their number), with all their events; by_events != 0: the k
 * events whose key orc_splitmix(seed, position) is smallest, the position
 * being the event's index in the (case, timestamp, row) order.  The kept
 * events are written in that order; n_out and n_cases_out receive their
 * number and the number of distinct cases among them.
 */
int orc_sample(int64_t n, const int32_t *case_id, const int32_t *act, const int64_t *ts, int32_t A, int64_t k,
               uint64_t seed, int32_t by_events, int32_t *case_out, int32_t *act_out, int64_t *ts_out,
               int64_t *n_out, int64_t *n_cases_out)
{
    if (n < 0 || A < 1 || k < 0) return ORC_E_INVALID;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *case_s = (int32_t *)malloc(nn * sizeof(int32_t));
    int32_t *act_s = (int32_t *)malloc(nn * sizeof(int32_t));
    int64_t *ts_s = (int64_t *)malloc(nn * sizeof(int64_t));
    int64_t *off = (int64_t *)malloc((nn + 1) * sizeof(int64_t));
    int32_t *code = (int32_t *)malloc(nn * sizeof(int32_t));
    orc_keyed *kv = (orc_keyed *)malloc(nn * sizeof(orc_keyed));
    unsigned char *keep = (unsigned char *)calloc(nn, 1);
    int64_t C = 0, m = 0, kc = 0;
    int r = orc_prepare(n, case_id, act, ts, A, NULL, case_s, act_s, ts_s, off, code, &C);
    if (r == ORC_OK) {
        int64_t units = by_events ? n : C;
        for (int64_t u = 0; u < units; u++) {
            uint64_t x = by_events ? (uint64_t)u : (uint64_t)(uint32_t)code[u];
            kv[u].key = orc_splitmix(seed, x);
            kv[u].idx = u;
        }
        qsort(kv, (size_t)units, sizeof(orc_keyed), cmp_keyed);
        for (int64_t u = 0; u < units && u < k; u++) keep[kv[u].idx] = 1;
        int64_t last_case = -1;
        for (int64_t c = 0; c < C; c++) {
            for (int64_t e = off[c]; e < off[c + 1]; e++) {
                if (!(by_events ? keep[e] : keep[c])) continue;
                if (last_case != c) {
                    kc++;
                    last_case = c;
                }
                if (case_out) case_out[m] = case_s[e];
                if (act_out) act_out[m] = act_s[e];
                if (ts_out) ts_out[m] = ts_s[e];
                m++;
            }
        }
    }
    if (n_out) *n_out = m;
    if (n_cases_out) *n_cases_out = kc;
    free(case_s);
    free(act_s);
    free(ts_s);
    free(off);
    free(code);
    free(kv);
    free(keep);
    return r;
}

/* ---- CSV ingestion ------------------------------------------------------------ */

#define ORC_E_PARSE -3

/* Days from 1970-01-01 to y-m-d in the proleptic Gregorian calendar, by
 * H. Hinnant's published days-from-civil algorithm ("chrono-Compatible
 * Low-Level Date Algorithms"): count the
 * days of whole 400-year eras since 0000-03-01, the years of the current era
 * (each from March, so the leap day ends a year) and the days of the current
 * year, then shift the origin. */
static int64_t civil_days(int64_t y, int64_t m, int64_t d)
{
    y -= m <= 2;
    int64_t era = (y >= 0 ? y : y - 399) / 400;
    int64_t yoe = y - era * 400;                              /* 0..399 */
    int64_t doy = (153 * (m + (m > 2 ? -3 : 9)) + 2) / 5 + d - 1; /* 0..365, from March 1 */
    int64_t doe = yoe * 365 + yoe / 4 - yoe / 100 + doy;       /* 0..146096 */
    return era * 146097 + doe - 719468;
}

static int days_in_month(int64_t y, int64_t m)
{
    static const int dm[12] = {31, 28, 31, 30, 31, 30, 31, 31, 30, 31, 30, 31};
    int leap = (y % 4 == 0 && y % 100 != 0) || y % 400 == 0;
    return m == 2 ? 28 + leap : dm[m - 1];
}

static int read_fixed(const char *s, int64_t n, int64_t *i, int width, int64_t *out)
{
    int64_t v = 0;
    for (int k = 0; k < width; k++) {
        if (*i >= n || s[*i] < '0' || s[*i] > '9') return 0;
        v = v * 10 + (s[*i] - '0');
        (*i)++;
    }
    *out = v;
    return 1;
}

/* ISO-8601 date-time: YYYY-MM-DD, optionally [T or space]HH:MM[:SS[(.|,)F]]
 * with 1-9 fraction digits, optionally Z or +-HH[[:]MM].  The value counts
 * units of 10^-scale s since 1970-01-01T00:00Z; fraction digits beyond the
 * unit are dropped.  Returns 1 and writes *out, or 0. */
static int parse_iso(const char *s, int64_t n, int scale, int64_t *out)
{
    int64_t i = 0, y, mo, d, h = 0, mi = 0, se = 0, frac = 0, tz = 0;
    int fdig = 0;
    if (!read_fixed(s, n, &i, 4, &y) || i >= n || s[i++] != '-' || !read_fixed(s, n, &i, 2, &mo) || i >= n ||
        s[i++] != '-' || !read_fixed(s, n, &i, 2, &d))
        return 0;
    if (mo < 1 || mo > 12 || d < 1 || d > days_in_month(y, mo)) return 0;
    if (i < n && (s[i] == 'T' || s[i] == ' ')) {
        i++;
        if (!read_fixed(s, n, &i, 2, &h) || i >= n || s[i++] != ':' || !read_fixed(s, n, &i, 2, &mi)) return 0;
        if (i < n && s[i] == ':') {
            i++;
            if (!read_fixed(s, n, &i, 2, &se)) return 0;
            if (i < n && (s[i] == '.' || s[i] == ',')) {
                i++;
                while (i < n && s[i] >= '0' && s[i] <= '9') {
                    if (fdig < 9) {
                        if (fdig < scale) frac = frac * 10 + (s[i] - '0');
                        fdig++;
                    } else {
                        return 0;
                    }
                    i++;
                }
                if (fdig == 0) return 0;
            }
        }
        if (h > 23 || mi > 59 || se > 59) return 0;
        if (i < n && s[i] == 'Z') {
            i++;
        } else if (i < n && (s[i] == '+' || s[i] == '-')) {
            int64_t sign = s[i] == '-' ? -1 : 1, th, tm = 0;
            i++;
            if (!read_fixed(s, n, &i, 2, &th)) return 0;
            if (i < n && s[i] == ':') i++;
            if (i < n && !read_fixed(s, n, &i, 2, &tm)) return 0;
            if (th > 23 || tm > 59) return 0;
            tz = sign * (th * 3600 + tm * 60);
        }
    }
    if (i != n) return 0;
    for (int k = fdig < scale ? fdig : scale; k < scale; k++) frac *= 10;
    __int128 secs = (__int128)civil_days(y, mo, d) * 86400 + h * 3600 + mi * 60 + se - tz;
    __int128 p10 = 1;
    for (int k = 0; k < scale; k++) p10 *= 10;
    __int128 v = secs * p10 + frac;
    if (v > (__int128)INT64_MAX || v < (__int128)INT64_MIN) return 0;
    *out = (int64_t)v;
    return 1;
}

/* Optional sign, then 1 or more decimal digits, within int64. */
static int parse_int(const char *s, int64_t n, int64_t *out)
{
    int64_t i = 0;
    int neg = 0;
    if (i < n && (s[i] == '+' || s[i] == '-')) neg = s[i++] == '-';
    if (i >= n) return 0;
    __int128 v = 0;
    for (; i < n; i++) {
        if (s[i] < '0' || s[i] > '9') return 0;
        v = v * 10 + (s[i] - '0');
        if (v > (__int128)INT64_MAX + 1) return 0;
    }
    if (neg) v = -v;
    if (v > (__int128)INT64_MAX || v < (__int128)INT64_MIN) return 0;
    *out = (int64_t)v;
    return 1;
}

/* Field value: quote characters open and close quoted runs wherever they
 * stand, a doubled quote inside a run is one literal quote, and the run's
 * delimiting quotes are dropped.  Writes the value into buf; returns its
 * length. */
static int64_t unquote(const char *s, int64_t n, char *buf)
{
    int64_t m = 0;
    int in = 0;
    for (int64_t i = 0; i < n; i++) {
        if (s[i] == '"') {
            if (in && i + 1 < n && s[i + 1] == '"') {
                buf[m++] = '"';
                i++;
            } else {
                in = !in;
            }
        } else {
            buf[m++] = s[i];
        }
    }
    return m;
}

typedef struct {
    const char *p;
    int64_t len;
    int64_t row;
} orc_str;

static int cmp_str_row(const void *pa, const void *pb)
{
    const orc_str *a = (const orc_str *)pa, *b = (const orc_str *)pb;
    int64_t m = a->len < b->len ? a->len : b->len;
    int c = memcmp(a->p, b->p, (size_t)m);
    if (c) return c;
    if (a->len != b->len) return a->len < b->len ? -1 : 1;
    return (a->row > b->row) - (a->row < b->row);
}

/* Codes in order of first appearance: sort (value, row), take each value's
 * first row, rank the values by it. */
static int64_t factorize(orc_str *v, int64_t rows, int32_t *code, int64_t *first_of_code)
{
    orc_str *srt = (orc_str *)malloc((size_t)(rows > 0 ? rows : 1) * sizeof(orc_str));
    int64_t *grp_first = (int64_t *)malloc((size_t)(rows > 0 ? rows : 1) * sizeof(int64_t));
    int64_t *grp_of_row = (int64_t *)malloc((size_t)(rows > 0 ? rows : 1) * sizeof(int64_t));
    memcpy(srt, v, (size_t)rows * sizeof(orc_str));
    qsort(srt, (size_t)rows, sizeof(orc_str), cmp_str_row);
    int64_t G = 0;
    for (int64_t k = 0; k < rows; k++) {
        if (k == 0 || srt[k].len != srt[k - 1].len || memcmp(srt[k].p, srt[k - 1].p, (size_t)srt[k].len) != 0)
            grp_first[G++] = srt[k].row;
        grp_of_row[srt[k].row] = G - 1;
    }
    /* the groups' first rows are distinct; the code of a group is the number of
       groups whose first row comes earlier */
    int64_t *mark = (int64_t *)malloc((size_t)(rows > 0 ? rows : 1) * sizeof(int64_t));
    for (int64_t r = 0; r < rows; r++) mark[r] = -1;
    for (int64_t g = 0; g < G; g++) mark[grp_first[g]] = g;
    int64_t *code_of_grp = (int64_t *)malloc((size_t)(G > 0 ? G : 1) * sizeof(int64_t));
    int64_t next = 0;
    for (int64_t r = 0; r < rows; r++)
        if (mark[r] >= 0) {
            code_of_grp[mark[r]] = next;
            first_of_code[next] = r;
            next++;
        }
    for (int64_t r = 0; r < rows; r++) code[r] = (int32_t)code_of_grp[grp_of_row[r]];
    free(srt);
    free(grp_first);
    free(grp_of_row);
    free(mark);
    free(code_of_grp);
    return G;
}

/*
 * orc_ingest_csv: a CSV text (Sec. 2.2: a header row and data rows of values
 * separated by a separator character) into the columns of an event log.
 *   lines     a line ends at a newline outside quoted runs (quote characters
 *             toggle the quoted state wherever they stand), or at the end of
 *             the text; a trailing carriage return is not part of the line;
 *             empty lines are skipped; with has_header the first non-empty
 *             line is the header.
 *   fields    split at separators outside quoted runs; values as in unquote.
 *   columns   case_col, act_col, ts_col (0-based); case and activity values
 *             are coded 0, 1, ... in order of first appearance (byte-exact
 *             comparison); timestamps are integers (ts_iso == 0) or ISO-8601
 *             date-times in units of 10^-ts_scale s (ts_iso != 0).
 * For each code, *_first_off / *_first_len give the byte range of the raw
 * field (quotes included) in the row of its first appearance.  A data row
 * with too few fields or a bad timestamp, or an open quoted run at the end of
 * the text (reported at the last row), is a parse error: the function
 * returns ORC_E_PARSE with *bad_row the first such data row (0-based).  More
 * data rows than max_rows: ORC_E_INVALID.
 */
int orc_ingest_csv(const char *text, int64_t n_bytes, int32_t case_col, int32_t act_col, int32_t ts_col,
                   char sep, int32_t has_header, int32_t ts_iso, int32_t ts_scale, int64_t max_rows,
                   int32_t *case_code, int32_t *act_code, int64_t *ts, int64_t *n_rows,
                   int64_t *case_first_off, int32_t *case_first_len, int64_t *n_cases,
                   int64_t *act_first_off, int32_t *act_first_len, int64_t *n_acts, int64_t *bad_row)
{
    if (n_bytes < 0 || case_col < 0 || act_col < 0 || ts_col < 0 || ts_scale < 0 || ts_scale > 9 || max_rows < 0)
        return ORC_E_INVALID;
    /* lines */
    int64_t cap_lines = n_bytes / 1 + 1;
    int64_t *ls = (int64_t *)malloc((size_t)cap_lines * sizeof(int64_t));
    int64_t *le = (int64_t *)malloc((size_t)cap_lines * sizeof(int64_t));
    int64_t L = 0, start = 0;
    int in = 0;
    for (int64_t i = 0; i <= n_bytes; i++) {
        int at_end = i == n_bytes;
        if (!at_end && text[i] == '"') in = !in;
        if (at_end || (text[i] == '\n' && !in)) {
            int64_t e = i;
            if (e > start && text[e - 1] == '\r') e--;
            if (e > start) {
                ls[L] = start;
                le[L] = e;
                L++;
            }
            start = i + 1;
        }
    }
    int open_at_end = in;
    int64_t first = (has_header && L > 0) ? 1 : 0;
    int64_t rows = L - first;
    int rc = ORC_OK;
    *bad_row = -1;
    if (rows > max_rows) {
        free(ls);
        free(le);
        return ORC_E_INVALID;
    }
    orc_str *cv = (orc_str *)malloc((size_t)(rows > 0 ? rows : 1) * sizeof(orc_str));
    orc_str *av = (orc_str *)malloc((size_t)(rows > 0 ? rows : 1) * sizeof(orc_str));
    int64_t *craw = (int64_t *)malloc((size_t)(rows > 0 ? rows : 1) * 2 * sizeof(int64_t));
    int64_t *araw = (int64_t *)malloc((size_t)(rows > 0 ? rows : 1) * 2 * sizeof(int64_t));
    char *store = (char *)malloc((size_t)(n_bytes > 0 ? n_bytes : 1) * 2 + 16);
    int64_t used = 0;
    int32_t need = case_col;
    if (act_col > need) need = act_col;
    if (ts_col > need) need = ts_col;
    for (int64_t r = 0; r < rows && rc == ORC_OK; r++) {
        int64_t a = ls[first + r], b = le[first + r];
        int64_t fb[3] = {-1, -1, -1}, fe[3] = {-1, -1, -1};
        int32_t f = 0;
        int q = 0;
        int64_t fs = a;
        for (int64_t i = a; i <= b; i++) {
            if (i < b && text[i] == '"') q = !q;
            if (i == b || (text[i] == sep && !q)) {
                if (f == case_col) { fb[0] = fs; fe[0] = i; }
                if (f == act_col) { fb[1] = fs; fe[1] = i; }
                if (f == ts_col) { fb[2] = fs; fe[2] = i; }
                f++;
                fs = i + 1;
            }
        }
        if (f <= need) {
            rc = ORC_E_PARSE;
            *bad_row = r;
            break;
        }
        int64_t k;
        k = unquote(text + fb[0], fe[0] - fb[0], store + used);
        cv[r].p = store + used; cv[r].len = k; cv[r].row = r; used += k;
        craw[2 * r] = fb[0]; craw[2 * r + 1] = fe[0] - fb[0];
        k = unquote(text + fb[1], fe[1] - fb[1], store + used);
        av[r].p = store + used; av[r].len = k; av[r].row = r; used += k;
        araw[2 * r] = fb[1]; araw[2 * r + 1] = fe[1] - fb[1];
        char tbuf[96];
        int64_t tl = fe[2] - fb[2];
        int ok = tl <= 64;
        if (ok) {
            k = unquote(text + fb[2], tl, tbuf);
            ok = ts_iso ? parse_iso(tbuf, k, ts_scale, &ts[r]) : parse_int(tbuf, k, &ts[r]);
        }
        if (!ok) {
            rc = ORC_E_PARSE;
            *bad_row = r;
        }
    }
    if (rc == ORC_OK && open_at_end && rows > 0) {
        rc = ORC_E_PARSE;
        *bad_row = rows - 1;
    }
    *n_rows = rows;
    *n_cases = 0;
    *n_acts = 0;
    if (rc == ORC_OK) {
        int64_t *firsts = (int64_t *)malloc((size_t)(rows > 0 ? rows : 1) * sizeof(int64_t));
        *n_cases = factorize(cv, rows, case_code, firsts);
        for (int64_t c = 0; c < *n_cases; c++) {
            case_first_off[c] = craw[2 * firsts[c]];
            case_first_len[c] = (int32_t)craw[2 * firsts[c] + 1];
        }
        *n_acts = factorize(av, rows, act_code, firsts);
        for (int64_t c = 0; c < *n_acts; c++) {
            act_first_off[c] = araw[2 * firsts[c]];
            act_first_len[c] = (int32_t)araw[2 * firsts[c] + 1];
        }
        free(firsts);
    }
    free(ls);
    free(le);
    free(cv);
    free(av);
    free(craw);
    free(araw);
    free(store);
    return rc;
}

/* ---- Parquet ingestion ------------------------------------------------ */

/*
 * Sec. 2.2: the event log may also come as a Parquet file, a columnar format
 * the GPU dataframe library reads directly.  The format is Apache Parquet's
 * published specification: the file ends with its metadata (a Thrift
 * compact-protocol struct), a 4-byte little-endian length and "PAR1"; each
 * column of each row group is a chunk of pages, each page a Thrift header and
 * its data.  Covered here: uncompressed chunks, flat schemas (required or
 * optional columns, no nesting), data pages of version 1 and 2, values PLAIN
 * or dictionary-coded (PLAIN_DICTIONARY / RLE_DICTIONARY, the dictionary page
 * PLAIN), definition levels in the RLE / bit-packing hybrid; INT32, INT64 and
 * BYTE_ARRAY case and activity columns, INT32 and INT64 timestamps.
 */
#define ORC_E_UNSUPPORTED -4

typedef struct {
    const uint8_t *b;
    int64_t n, p;
    int bad;
} orc_tr;   /* a reader of Thrift's compact protocol */

static uint64_t tr_varint(orc_tr *r)
{
    uint64_t v = 0;
    for (int sh = 0; sh < 64; sh += 7) {
        if (r->p >= r->n) break;
        uint8_t c = r->b[r->p++];
        v |= (uint64_t)(c & 0x7f) << sh;
        if (!(c & 0x80)) return v;
    }
    r->bad = 1;
    return 0;
}

static int64_t tr_zigzag(orc_tr *r)
{
    uint64_t u = tr_varint(r);
    return (int64_t)(u >> 1) ^ -(int64_t)(u & 1);
}

static uint8_t tr_byte(orc_tr *r)
{
    if (r->p >= r->n) {
        r->bad = 1;
        return 0;
    }
    return r->b[r->p++];
}

/* A field header inside a struct: returns its type (0 = end of struct) and the
   field id, whose delta from the previous id is in the high nibble (0: the id
   follows as a zigzag varint). */
static int tr_field(orc_tr *r, int *last_id, int *id)
{
    uint8_t h = tr_byte(r);
    int t = h & 0x0f;
    if (t == 0 || r->bad) return 0;
    int d = h >> 4;
    *id = d ? *last_id + d : (int)tr_zigzag(r);
    *last_id = *id;
    return t;
}

/* Skips one value of compact type t (in_list: booleans take a byte). */
static void tr_skip(orc_tr *r, int t, int in_list, int depth)
{
    if (depth > 64 || r->bad) {
        r->bad = 1;
        return;
    }
    switch (t) {
    case 1:
    case 2:
        if (in_list) r->p += 1;   /* in a field header the value is the type itself */
        break;
    case 3: r->p += 1; break;
    case 4:
    case 5:
    case 6: tr_varint(r); break;
    case 7: r->p += 8; break;
    case 8: {
        uint64_t len = tr_varint(r);
        if (len > (uint64_t)(r->n - r->p)) r->bad = 1;
        else r->p += (int64_t)len;
        break;
    }
    case 9:
    case 10: {
        uint8_t h = tr_byte(r);
        uint64_t sz = h >> 4;
        if (sz == 15) sz = tr_varint(r);
        for (uint64_t k = 0; k < sz && !r->bad; k++) tr_skip(r, h & 0x0f, 1, depth + 1);
        break;
    }
    case 11: {
        uint64_t sz = tr_varint(r);
        if (sz) {
            uint8_t kv = tr_byte(r);
            for (uint64_t k = 0; k < sz && !r->bad; k++) {
                tr_skip(r, kv >> 4, 1, depth + 1);
                tr_skip(r, kv & 0x0f, 1, depth + 1);
            }
        }
        break;
    }
    case 12: {
        int last = 0, id = 0, ft;
        while ((ft = tr_field(r, &last, &id)) != 0 && !r->bad) tr_skip(r, ft, 0, depth + 1);
        break;
    }
    default: r->bad = 1;
    }
    if (r->p > r->n) r->bad = 1;
}

/* A list header: element count; *etype the element type. */
static int64_t tr_list(orc_tr *r, int *etype)
{
    uint8_t h = tr_byte(r);
    uint64_t sz = h >> 4;
    if (sz == 15) sz = tr_varint(r);
    *etype = h & 0x0f;
    if (sz > (uint64_t)r->n) r->bad = 1;
    return (int64_t)sz;
}

typedef struct {
    int32_t type, rep, has_children;
} orc_pq_leaf;

typedef struct {
    int32_t type, codec;
    int64_t num_values, size, data_off, dict_off;
} orc_pq_chunk;

typedef struct {
    int32_t type;        /* 1 INT32, 2 INT64, 6 BYTE_ARRAY */
    int32_t optional;    /* repetition OPTIONAL: definition levels present */
    /* decoded values, one per row: integers, or byte ranges in the file */
    int64_t *ival;
    int64_t *off;
    int32_t *len;
} orc_pq_col;

/* Parquet's RLE / bit-packing hybrid: count values of bw bits from b[0..n). */
static int pq_hybrid(const uint8_t *b, int64_t n, int bw, int64_t count, uint32_t *out)
{
    orc_tr r = {b, n, 0, 0};
    int64_t k = 0;
    int vb = (bw + 7) / 8;
    while (k < count) {
        uint64_t h = tr_varint(&r);
        if (r.bad) return -1;
        if (h & 1) {   /* bit-packed: (h >> 1) groups of 8 values, least significant bit first */
            uint64_t groups = h >> 1;
            if (groups > (uint64_t)n || (int64_t)(groups * (uint64_t)bw) > n - r.p) return -1;
            for (int64_t j = 0; j < (int64_t)groups * 8 && k < count; j++) {
                uint32_t v = 0;
                for (int i = 0; i < bw; i++) {
                    int64_t q = j * bw + i;
                    v |= (uint32_t)((b[r.p + q / 8] >> (q % 8)) & 1u) << i;
                }
                out[k++] = v;
            }
            r.p += (int64_t)groups * bw;
        } else {       /* a run of one value in ceil(bw/8) little-endian bytes */
            uint64_t run = h >> 1;
            if (vb > n - r.p) return -1;
            uint32_t v = 0;
            for (int i = 0; i < vb; i++) v |= (uint32_t)b[r.p + i] << (8 * i);
            r.p += vb;
            for (uint64_t j = 0; j < run && k < count; j++) out[k++] = v;
        }
    }
    return 0;
}

static int64_t rd_le(const uint8_t *p, int bytes)
{
    uint64_t v = 0;
    for (int i = 0; i < bytes; i++) v |= (uint64_t)p[i] << (8 * i);
    if (bytes == 4) return (int64_t)(int32_t)(uint32_t)v;
    return (int64_t)v;
}

/* One PLAIN value at b[p] of n bytes: the integer or the byte range. */
static int pq_plain(const uint8_t *b, int64_t n, int64_t *p, int32_t type, int64_t base, int64_t *ival,
                    int64_t *off, int32_t *len)
{
    if (type == 1 || type == 2) {
        int w = type == 1 ? 4 : 8;
        if (w > n - *p) return -1;
        *ival = rd_le(b + *p, w);
        *p += w;
        return 0;
    }
    if (4 > n - *p) return -1;
    int64_t L = (int64_t)(uint32_t)rd_le(b + *p, 4) & 0xffffffffll;
    if (L > n - *p - 4) return -1;
    *off = base + *p + 4;
    *len = (int32_t)L;
    *p += 4 + L;
    return 0;
}

/* The values of one column chunk into col at rows row0 ..; returns 0, a
   negative status, or (parse error) sets *bad_row. */
static int pq_chunk(const uint8_t *f, int64_t fn, const orc_pq_chunk *ch, orc_pq_col *col, int64_t row0,
                    int64_t *bad_row)
{
    if (ch->codec != 0) return ORC_E_UNSUPPORTED;
    if (ch->type != col->type) return ORC_E_PARSE;
    if (ch->num_values == 0) return ORC_OK;   /* nothing to read (its pages, if any, hold no value) */
    int64_t pos = (ch->dict_off > 0 && (ch->dict_off < ch->data_off || ch->data_off <= 0)) ? ch->dict_off
                                                                                          : ch->data_off;
    if (pos < 4 || ch->size < 0 || ch->size > fn - pos) return ORC_E_PARSE;
    int64_t end = pos + ch->size;
    int64_t done = 0;
    int64_t dn = -1;   /* dictionary entries, -1 before a dictionary page */
    int64_t *d_ival = NULL, *d_off = NULL;
    int32_t *d_len = NULL;
    int rc = ORC_OK;
    while (done < ch->num_values && rc == ORC_OK) {
        orc_tr r = {f, end, pos, 0};
        int last = 0, id = 0, ft;
        int32_t ptype = -1, csize = -1, nv = -1, enc = -1, dlen = -1, rlen = -1, v2 = 0;
        while ((ft = tr_field(&r, &last, &id)) != 0 && !r.bad) {
            if (id == 1 && ft == 5) ptype = (int32_t)tr_zigzag(&r);
            else if (id == 3 && ft == 5) csize = (int32_t)tr_zigzag(&r);
            else if ((id == 5 || id == 7 || id == 8) && ft == 12) {
                v2 = id == 8;
                int l2 = 0, i2 = 0, t2;
                while ((t2 = tr_field(&r, &l2, &i2)) != 0 && !r.bad) {
                    if (i2 == 1 && t2 == 5) nv = (int32_t)tr_zigzag(&r);
                    else if (((id != 8 && i2 == 2) || (id == 8 && i2 == 4)) && t2 == 5) enc = (int32_t)tr_zigzag(&r);
                    else if (id == 8 && i2 == 5 && t2 == 5) dlen = (int32_t)tr_zigzag(&r);
                    else if (id == 8 && i2 == 6 && t2 == 5) rlen = (int32_t)tr_zigzag(&r);
                    else tr_skip(&r, t2, 0, 1);
                }
            } else tr_skip(&r, ft, 0, 0);
        }
        if (r.bad || ptype < 0 || csize < 0 || csize > end - r.p) { rc = ORC_E_PARSE; break; }
        const uint8_t *pg = f + r.p;
        int64_t pbase = r.p;
        pos = r.p + csize;
        if (ptype == 2) {   /* dictionary page: nv PLAIN values */
            if (nv < 0 || dn >= 0) { rc = ORC_E_PARSE; break; }
            if (enc != 0 && enc != 2) { rc = ORC_E_UNSUPPORTED; break; }
            dn = nv;
            d_ival = (int64_t *)malloc((size_t)(dn > 0 ? dn : 1) * sizeof(int64_t));
            d_off = (int64_t *)malloc((size_t)(dn > 0 ? dn : 1) * sizeof(int64_t));
            d_len = (int32_t *)malloc((size_t)(dn > 0 ? dn : 1) * sizeof(int32_t));
            int64_t p = 0;
            for (int64_t k = 0; k < dn; k++)
                if (pq_plain(pg, csize, &p, col->type, pbase, &d_ival[k], &d_off[k], &d_len[k])) {
                    rc = ORC_E_PARSE;
                    break;
                }
            continue;
        }
        if (ptype != 0 && ptype != 3) continue;   /* index pages carry no values */
        if (nv < 0 || nv > ch->num_values - done) { rc = ORC_E_PARSE; break; }
        if (v2 && (dlen < 0 || rlen != 0 || (int64_t)dlen > csize)) { rc = v2 && rlen > 0 ? ORC_E_UNSUPPORTED : ORC_E_PARSE; break; }
        int64_t p = 0;
        if (col->optional) {   /* definition levels (bit width 1): 0 is a null */
            int64_t lb;
            if (v2) lb = dlen;
            else {
                if (csize < 4) { rc = ORC_E_PARSE; break; }
                lb = (int64_t)(uint32_t)rd_le(pg, 4) & 0xffffffffll;
                p = 4;
            }
            if (lb > csize - p) { rc = ORC_E_PARSE; break; }
            uint32_t *lev = (uint32_t *)malloc((size_t)(nv > 0 ? nv : 1) * sizeof(uint32_t));
            if (pq_hybrid(pg + p, lb, 1, nv, lev)) rc = ORC_E_PARSE;
            for (int64_t k = 0; k < nv && rc == ORC_OK; k++)
                if (lev[k] == 0) {
                    rc = ORC_E_PARSE;
                    *bad_row = row0 + done + k;
                }
            free(lev);
            if (rc != ORC_OK) break;
            p += lb;
        } else if (v2 && dlen != 0) {
            rc = ORC_E_PARSE;
            break;
        }
        if (enc == 0) {
            for (int64_t k = 0; k < nv; k++) {
                int64_t row = row0 + done + k;
                if (pq_plain(pg, csize, &p, col->type, pbase, &col->ival[row], &col->off[row], &col->len[row])) {
                    rc = ORC_E_PARSE;
                    break;
                }
            }
        } else if (enc == 2 || enc == 8) {
            if (dn < 0 || p >= csize) { rc = ORC_E_PARSE; break; }
            int bw = pg[p++];
            if (bw > 32) { rc = ORC_E_PARSE; break; }
            uint32_t *idx = (uint32_t *)malloc((size_t)(nv > 0 ? nv : 1) * sizeof(uint32_t));
            if (pq_hybrid(pg + p, csize - p, bw, nv, idx)) rc = ORC_E_PARSE;
            for (int64_t k = 0; k < nv && rc == ORC_OK; k++) {
                if ((int64_t)idx[k] >= dn) {
                    rc = ORC_E_PARSE;
                    break;
                }
                int64_t row = row0 + done + k;
                col->ival[row] = d_ival[idx[k]];
                col->off[row] = d_off[idx[k]];
                col->len[row] = d_len[idx[k]];
            }
            free(idx);
        } else {
            rc = ORC_E_UNSUPPORTED;
        }
        done += nv;
    }
    free(d_ival);
    free(d_off);
    free(d_len);
    if (rc == ORC_OK && done != ch->num_values) rc = ORC_E_PARSE;
    return rc;
}

/*
 * orc_ingest_parquet: columns case_col, act_col, ts_col (0-based leaf
 * columns of a flat schema) of a Parquet file held in f[0..n) into the
 * columns of an event log.  Case and activity values are coded 0, 1, ... in
 * order of first appearance (integers by value, byte arrays byte-exact); for
 * each code, *_first_off / *_first_len give the byte range of the value at
 * its first row (for an integer column: the value itself, and -1).
 * Timestamps are the INT64 (or INT32) values.  A null in one of the three
 * columns is a parse error at its row (*bad_row); a malformed file is a parse
 * error with *bad_row = -1; a valid file outside what is covered (compression,
 * other encodings or types, nesting) returns ORC_E_UNSUPPORTED.  More rows than
 * max_rows: ORC_E_INVALID.
 */
int orc_ingest_parquet(const uint8_t *f, int64_t n, int32_t case_col, int32_t act_col, int32_t ts_col,
                       int64_t max_rows, int32_t *case_code, int32_t *act_code, int64_t *ts, int64_t *n_rows,
                       int64_t *case_first_off, int32_t *case_first_len, int64_t *n_cases,
                       int64_t *act_first_off, int32_t *act_first_len, int64_t *n_acts, int64_t *bad_row)
{
    *bad_row = -1;
    *n_rows = *n_cases = *n_acts = 0;
    if (n < 0 || case_col < 0 || act_col < 0 || ts_col < 0 || max_rows < 0) return ORC_E_INVALID;
    if (n < 12 || memcmp(f, "PAR1", 4) != 0 || memcmp(f + n - 4, "PAR1", 4) != 0) return ORC_E_PARSE;
    int64_t flen = (int64_t)(uint32_t)rd_le(f + n - 8, 4) & 0xffffffffll;
    if (flen > n - 12) return ORC_E_PARSE;
    orc_tr r = {f, n - 8, n - 8 - flen, 0};

    /* FileMetaData: 2 schema, 3 num_rows, 4 row_groups */
    orc_pq_leaf *leaf = NULL;
    int64_t n_leaf = 0, num_rows = -1, n_rg = 0;
    int64_t *rg_rows = NULL;
    orc_pq_chunk *chunks = NULL;   /* [row group][3] */
    int want[3] = {case_col, act_col, ts_col};
    int rc = ORC_OK;
    int last = 0, id = 0, ft;
    while ((ft = tr_field(&r, &last, &id)) != 0 && !r.bad && rc == ORC_OK) {
        if (id == 2 && ft == 9) {
            int et;
            int64_t ne = tr_list(&r, &et);
            if (et != 12 || ne < 1) { rc = ORC_E_PARSE; break; }
            leaf = (orc_pq_leaf *)calloc((size_t)ne, sizeof(orc_pq_leaf));
            for (int64_t e = 0; e < ne && !r.bad; e++) {
                orc_pq_leaf el = {-1, 0, 0};
                int l2 = 0, i2 = 0, t2;
                while ((t2 = tr_field(&r, &l2, &i2)) != 0 && !r.bad) {
                    if (i2 == 1 && t2 == 5) el.type = (int32_t)tr_zigzag(&r);
                    else if (i2 == 3 && t2 == 5) el.rep = (int32_t)tr_zigzag(&r);
                    else if (i2 == 5 && t2 == 5) el.has_children = tr_zigzag(&r) > 0;
                    else tr_skip(&r, t2, 0, 1);
                }
                if (e == 0) continue;   /* the root */
                if (el.has_children) rc = ORC_E_UNSUPPORTED;   /* nested schema */
                leaf[n_leaf++] = el;
            }
        } else if (id == 3 && ft == 6) {
            num_rows = tr_zigzag(&r);
        } else if (id == 4 && ft == 9) {
            int et;
            n_rg = tr_list(&r, &et);
            if (et != 12) { rc = ORC_E_PARSE; break; }
            rg_rows = (int64_t *)calloc((size_t)(n_rg > 0 ? n_rg : 1), sizeof(int64_t));
            chunks = (orc_pq_chunk *)calloc((size_t)(n_rg > 0 ? n_rg : 1) * 3, sizeof(orc_pq_chunk));
            for (int64_t g = 0; g < n_rg && !r.bad; g++) {
                int l2 = 0, i2 = 0, t2;
                rg_rows[g] = -1;
                while ((t2 = tr_field(&r, &l2, &i2)) != 0 && !r.bad) {
                    if (i2 == 3 && t2 == 6) rg_rows[g] = tr_zigzag(&r);
                    else if (i2 == 1 && t2 == 9) {
                        int ct;
                        int64_t nc = tr_list(&r, &ct);
                        if (ct != 12) { r.bad = 1; break; }
                        for (int64_t c = 0; c < nc && !r.bad; c++) {
                            orc_pq_chunk cm = {-1, -1, -1, -1, -1, -1};
                            int l3 = 0, i3 = 0, t3;
                            while ((t3 = tr_field(&r, &l3, &i3)) != 0 && !r.bad) {
                                if (i3 == 1 && t3 == 8) rc = rc ? rc : ORC_E_UNSUPPORTED;   /* chunk in another file */
                                if (i3 == 3 && t3 == 12) {
                                    int l4 = 0, i4 = 0, t4;
                                    while ((t4 = tr_field(&r, &l4, &i4)) != 0 && !r.bad) {
                                        if (i4 == 1 && t4 == 5) cm.type = (int32_t)tr_zigzag(&r);
                                        else if (i4 == 4 && t4 == 5) cm.codec = (int32_t)tr_zigzag(&r);
                                        else if (i4 == 5 && t4 == 6) cm.num_values = tr_zigzag(&r);
                                        else if (i4 == 7 && t4 == 6) cm.size = tr_zigzag(&r);
                                        else if (i4 == 9 && t4 == 6) cm.data_off = tr_zigzag(&r);
                                        else if (i4 == 11 && t4 == 6) cm.dict_off = tr_zigzag(&r);
                                        else tr_skip(&r, t4, 0, 2);
                                    }
                                } else tr_skip(&r, t3, 0, 1);
                            }
                            for (int k = 0; k < 3; k++)
                                if (c == want[k]) chunks[g * 3 + k] = cm;
                        }
                    } else tr_skip(&r, t2, 0, 1);
                }
            }
        } else {
            tr_skip(&r, ft, 0, 0);
        }
    }
    if (rc == ORC_OK && (r.bad || !leaf || num_rows < 0)) rc = ORC_E_PARSE;
    for (int k = 0; k < 3 && rc == ORC_OK; k++) {
        if (want[k] >= n_leaf) rc = ORC_E_INVALID;
        else if (leaf[want[k]].rep == 2) rc = ORC_E_UNSUPPORTED;
        else if (k < 2 && leaf[want[k]].type != 1 && leaf[want[k]].type != 2 && leaf[want[k]].type != 6) rc = ORC_E_UNSUPPORTED;
        else if (k == 2 && leaf[want[k]].type != 1 && leaf[want[k]].type != 2) rc = ORC_E_UNSUPPORTED;
    }
    int64_t total = 0;
    for (int64_t g = 0; g < n_rg && rc == ORC_OK; g++) {
        if (rg_rows[g] < 0) rc = ORC_E_PARSE;
        for (int k = 0; k < 3 && rc == ORC_OK; k++)
            if (chunks[g * 3 + k].num_values != rg_rows[g]) rc = chunks[g * 3 + k].type < 0 ? ORC_E_PARSE : ORC_E_UNSUPPORTED;
        total += rg_rows[g];
    }
    if (rc == ORC_OK && total != num_rows) rc = ORC_E_PARSE;
    if (rc == ORC_OK && total > max_rows) rc = ORC_E_INVALID;
    orc_pq_col col[3];
    size_t m = (size_t)(total > 0 ? total : 1);
    for (int k = 0; k < 3; k++) {
        col[k].type = (rc == ORC_OK) ? leaf[want[k]].type : 0;
        col[k].optional = (rc == ORC_OK) ? leaf[want[k]].rep == 1 : 0;
        col[k].ival = (int64_t *)calloc(m, sizeof(int64_t));
        col[k].off = (int64_t *)calloc(m, sizeof(int64_t));
        col[k].len = (int32_t *)calloc(m, sizeof(int32_t));
    }
    /* row groups in order; a structural error stops at once; nulls: the
       smallest row with a null in any of the three columns */
    int64_t row0 = 0;
    for (int64_t g = 0; g < n_rg && rc == ORC_OK; g++) {
        int64_t null_row = -1;
        for (int k = 0; k < 3 && rc == ORC_OK; k++) {
            int64_t b = -1;
            int c = pq_chunk(f, n - 8 - flen, &chunks[g * 3 + k], &col[k], row0, &b);
            if (c == ORC_E_PARSE && b >= 0) {
                if (null_row < 0 || b < null_row) null_row = b;
            } else if (c != ORC_OK) {
                rc = c;
            }
        }
        if (rc == ORC_OK && null_row >= 0) {
            rc = ORC_E_PARSE;
            *bad_row = null_row;
        }
        row0 += rg_rows[g];
    }
    if (rc == ORC_OK) {
        *n_rows = total;
        for (int64_t i = 0; i < total; i++) ts[i] = col[2].ival[i];
        int32_t *codes[2] = {case_code, act_code};
        int64_t *fo[2] = {case_first_off, act_first_off};
        int32_t *fl[2] = {case_first_len, act_first_len};
        int64_t *nc[2] = {n_cases, n_acts};
        orc_str *sv = (orc_str *)malloc(m * sizeof(orc_str));
        int64_t *firsts = (int64_t *)malloc(m * sizeof(int64_t));
        for (int k = 0; k < 2; k++) {
            int is_int = col[k].type != 6;
            for (int64_t i = 0; i < total; i++) {
                sv[i].p = is_int ? (const char *)&col[k].ival[i] : (const char *)f + col[k].off[i];
                sv[i].len = is_int ? 8 : col[k].len[i];
                sv[i].row = i;
            }
            *nc[k] = factorize(sv, total, codes[k], firsts);
            for (int64_t c = 0; c < *nc[k]; c++) {
                fo[k][c] = is_int ? col[k].ival[firsts[c]] : col[k].off[firsts[c]];
                fl[k][c] = is_int ? -1 : col[k].len[firsts[c]];
            }
        }
        free(sv);
        free(firsts);
    }
    for (int k = 0; k < 3; k++) {
        free(col[k].ival);
        free(col[k].off);
        free(col[k].len);
    }
    free(leaf);
    free(rg_rows);
    free(chunks);
    return rc;
}
