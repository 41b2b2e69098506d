/*
 * Test driver: every oracle function on varied inputs, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py.
 * The inputs come from a small linear congruential generator; the driver
 * checks return codes only (the values are pinned elsewhere), so what it
 * catches is out-of-bounds access, leaks and undefined behaviour.
 */
#include "../oracle/pm4g_oracle.c"

#include <stdio.h>

static uint64_t lcg_state = 88172645463325252ull;
static uint64_t next_u64(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return lcg_state;
}

static int64_t range(int64_t lo, int64_t hi)   /* uniform-ish in [lo, hi], unsigned arithmetic throughout */
{
    uint64_t span = (uint64_t)hi - (uint64_t)lo + 1u;
    return (int64_t)((uint64_t)lo + (span ? next_u64() % span : next_u64()));
}

static int fails = 0;
#define EXPECT(cond)                                                           \
    do {                                                                       \
        if (!(cond)) {                                                         \
            fprintf(stderr, "expectation failed at line %d: %s\n", __LINE__, #cond); \
            fails++;                                                           \
        }                                                                      \
    } while (0)

static void run_log(int64_t n, int32_t A, int ts_kind)
{
    size_t nn = (size_t)(n > 0 ? n : 1), cells = (size_t)A * (size_t)A;
    int32_t *c = malloc(nn * 4), *a = malloc(nn * 4);
    int64_t *t = malloc(nn * 8);
    int64_t ncases = n > 0 ? range(1, n) : 1;
    for (int64_t i = 0; i < n; i++) {
        c[i] = (int32_t)(range(0, ncases - 1) * 9973 - 1000000);
        a[i] = (int32_t)range(0, A - 1);
        t[i] = ts_kind == 0 ? range(-3, 3) : ts_kind == 1 ? range(0, 1000000000) : range(-(1ll << 62), 1ll << 62);
    }
    int32_t *i32a = malloc(nn * 4), *i32b = malloc(nn * 4), *i32c = malloc(nn * 4), *i32d = malloc(nn * 4);
    int64_t *i64a = malloc((nn + 1) * 8), *i64b = malloc((nn + 1) * 8), *i64c = malloc((nn + 1) * 8);
    int64_t *cl = malloc(cells * 8), *s = malloc(cells * 8), *mn = malloc(cells * 8), *mx = malloc(cells * 8);
    uint64_t *u1 = malloc(cells * 8), *u2 = malloc(cells * 8), *u3 = malloc(cells * 8), *u4 = malloc(cells * 8);
    double *d1 = malloc(cells * 8), *d2 = malloc(cells * 8);
    int64_t *st = malloc((size_t)A * 8), *en = malloc((size_t)A * 8), *ac = malloc((size_t)A * 8);
    int64_t C = 0, V = 0, m = 0, kc = 0, np = 0, ne = 0;
    int32_t ov = 0;
    size_t mw = ((size_t)A + 63) / 64, pw = (cells + 63) / 64;
    uint64_t *mask = calloc(mw, 8), *pmask = calloc(pw, 8), *vmask = calloc(nn / 64 + 1, 8);
    for (size_t w = 0; w < mw; w++) mask[w] = next_u64();
    for (size_t w = 0; w < pw; w++) pmask[w] = next_u64();
    for (size_t w = 0; w < nn / 64 + 1; w++) vmask[w] = next_u64();

    EXPECT(orc_prepare(n, c, a, t, A, i64a, i32a, i32b, i64b, i64c, i32c, &C) == ORC_OK);
    EXPECT(orc_dfg(n, c, a, t, A, i64a, cl, s, mn, mx, d1, st, en, ac, &C, &ov) == ORC_OK);
    EXPECT(orc_variants(n, c, a, t, A, &V, i64a, i32a, i32b, i64b, i32c, i32d, i32a, &C) == ORC_OK);
    EXPECT(orc_view(n, c, a, t, A, -500000, 500000, -100, 1000000, mask, cl, s, mn, mx, d1, st, en, ac, &C, &ov,
                    &ne) == ORC_OK);
    EXPECT(orc_cases(n, c, a, t, A, i32a, i64a, i64b, &C) == ORC_OK);
    int64_t bounds[8] = {1, 50, INT64_MIN, INT64_MAX, -5, INT64_MAX, INT64_MIN, 7};
    EXPECT(orc_filter_cases(n, c, a, t, A, bounds, mask, pmask, 1, mask, NULL, vmask, (int64_t)nn, 0, i32a, i32b,
                            i64a, &m, &kc) == ORC_OK);
    EXPECT(orc_filter_df_events(n, c, a, t, A, pmask, 1, 0, i32a, i32b, i64a, &m, &kc) == ORC_OK);
    EXPECT(orc_efg(n, c, a, t, A, cl, u1, u2, u3, u4, d1, d2, &np) == ORC_OK);
    EXPECT(orc_sample(n, c, a, t, A, n / 3, next_u64(), 0, i32a, i32b, i64a, &m, &kc) == ORC_OK);
    EXPECT(orc_sample(n, c, a, t, A, n / 3, next_u64(), 1, i32a, i32b, i64a, &m, &kc) == ORC_OK);
    EXPECT(m == n / 3);
    free(c); free(a); free(t); free(i32a); free(i32b); free(i32c); free(i32d); free(i64a); free(i64b);
    free(i64c); free(cl); free(s); free(mn); free(mx); free(u1); free(u2); free(u3); free(u4); free(d1);
    free(d2); free(st); free(en); free(ac); free(mask); free(pmask); free(vmask);
}

static void run_csv(const char *text, int64_t n, int ts_iso, int expect)
{
    int64_t cap = n + 1;
    int32_t *cc = malloc((size_t)cap * 4), *ac = malloc((size_t)cap * 4), *cl = malloc((size_t)cap * 4),
            *al = malloc((size_t)cap * 4);
    int64_t *ts = malloc((size_t)cap * 8), *co = malloc((size_t)cap * 8), *ao = malloc((size_t)cap * 8);
    int64_t nr = 0, nc = 0, na = 0, bad = 0;
    char *copy = malloc((size_t)(n > 0 ? n : 1));   /* exact length: reads past it are caught */
    memcpy(copy, text, (size_t)n);
    int rc = orc_ingest_csv(copy, n, 0, 1, 2, ',', 1, ts_iso, 6, cap, cc, ac, ts, &nr, co, cl, &nc, ao, al, &na, &bad);
    EXPECT(rc == expect);
    free(cc); free(ac); free(cl); free(al); free(ts); free(co); free(ao); free(copy);
}

int main(void)
{
    run_log(0, 1, 1);
    run_log(1, 1, 0);
    for (int r = 0; r < 30; r++) run_log(range(1, 400), (int32_t)range(1, 70), (int)range(0, 2));
    const char *ok[] = {
        "c,a,t\n1,x,5\n2,y,6\n",
        "c,a,t\r\n\"1,2\",\"a\"\"b\",7\r\n\r\n3,z,8",
        "c,a,t\n1,x,2006-07-24T10:00:00.123456789+01:00\n2,y,2006-07-24 00:00Z\n",
        "", "\n\n", "c,a,t", "c,a,t\n\"\",\"\",1\n"};
    const int ok_iso[] = {0, 0, 1, 0, 0, 0, 0};
    for (int k = 0; k < 7; k++) run_csv(ok[k], (int64_t)strlen(ok[k]), ok_iso[k], ORC_OK);
    const char *bad[] = {"c,a,t\n1,x\n", "c,a,t\n1,x,2006-02-30\n", "c,a,t\n1,x,\"5\n", "c,a,t\n1,x,99999999999999999999\n",
                         "c,a,t\n1,x,2006-01-01T10:00+01:00trailing\n"};
    const int bad_iso[] = {0, 1, 0, 0, 1};
    for (int k = 0; k < 5; k++) run_csv(bad[k], (int64_t)strlen(bad[k]), bad_iso[k], ORC_E_PARSE);
    /* random bytes: any return code, but no invalid access */
    for (int r = 0; r < 200; r++) {
        int64_t len = range(0, 300);
        char *buf = malloc((size_t)(len > 0 ? len : 1));
        const char alphabet[] = "ab,\"\r\n 0123456789-:TZ+.";
        for (int64_t i = 0; i < len; i++) buf[i] = alphabet[next_u64() % (sizeof(alphabet) - 1)];
        int64_t cap = len + 1;
        int32_t *cc = malloc((size_t)cap * 4), *ac = malloc((size_t)cap * 4), *cl = malloc((size_t)cap * 4),
                *al = malloc((size_t)cap * 4);
        int64_t *ts = malloc((size_t)cap * 8), *co = malloc((size_t)cap * 8), *ao = malloc((size_t)cap * 8);
        int64_t nr, nc, na, bd;
        (void)orc_ingest_csv(buf, len, 0, 1, 2, ',', (int)(r & 1), (int)((r >> 1) & 1), 3, cap, cc, ac, ts, &nr, co,
                             cl, &nc, ao, al, &na, &bd);
        free(buf); free(cc); free(ac); free(cl); free(al); free(ts); free(co); free(ao);
    }
    if (fails) return 1;
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
