"""Seeded synthetic event logs and drill-down views.

The paper measures on public event logs (road traffic fines, two BPI
challenge logs, replicated 2-20 times; Table 1).  Those logs are not used
here.  This module draws logs with the same kind of structure instead:
case lengths from a stated law, activity sequences from a seeded Markov
chain, integer timestamps with exponential gaps, and a row layout that is
either already in (case, time) order or shuffled.

This module is shared by the tests, the benchmark and the oracle checks.  It
holds none of the method's arithmetic: it never sorts by (case, time),
never forms directly-follows pairs and never aggregates.  It only draws
random numbers and lays rows out.
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_BASE = 220404898
DAY_MS = 86_400_000
DAY_NS = 86_400_000_000_000


@dataclasses.dataclass
class Log:
    """A columnar event log: row i is (case[i], act[i], ts[i])."""

    case: np.ndarray          # int32 [N]
    act: np.ndarray           # int32 [N]
    ts: np.ndarray            # int64 [N]
    n_activities: int
    presorted: bool           # rows are already in (case, ts, row) order
    lengths_by_code: np.ndarray | None = None   # int64 [C]; events of case code c
    name: str = ""

    @property
    def n_events(self) -> int:
        return int(self.case.shape[0])


def zipf_weights(A: int, s: float, rng: np.random.Generator) -> np.ndarray:
    """Zipf(s) over ranks 1..A, ranks assigned to activities by a permutation."""
    w = np.arange(1, A + 1, dtype=np.float64) ** (-s)
    w /= w.sum()
    pi = np.empty(A)
    pi[rng.permutation(A)] = w
    return pi


def markov_chain(A: int, law: str, rng: np.random.Generator):
    """Initial distribution pi0 and row-stochastic transition matrix P."""
    if law == "dirichlet":
        pi0 = rng.dirichlet(np.ones(A))
        P = rng.dirichlet(np.ones(A), size=A)
    elif law == "zipf":
        pi = zipf_weights(A, 1.1, rng)
        pi0 = pi
        P = 0.5 * pi[None, :] + 0.5 * rng.dirichlet(np.ones(A), size=A)
    else:
        raise ValueError(law)
    return pi0, P


def alias_table(p: np.ndarray):
    """Walker/Vose alias table of one distribution: (prob, alias)."""
    A = p.shape[0]
    scaled = p * A
    prob = np.ones(A)
    alias = np.arange(A)
    small = [i for i in range(A) if scaled[i] < 1.0]
    large = [i for i in range(A) if scaled[i] >= 1.0]
    while small and large:
        s_, l_ = small.pop(), large.pop()
        prob[s_] = scaled[s_]
        alias[s_] = l_
        scaled[l_] -= 1.0 - scaled[s_]
        (small if scaled[l_] < 1.0 else large).append(l_)
    return prob, alias


def _sample_alias(prob: np.ndarray, alias: np.ndarray, rows: np.ndarray, u: np.ndarray) -> np.ndarray:
    # one uniform: its integer part picks a column, its fraction accepts it or its alias
    A = prob.shape[1]
    x = u * A
    j = np.minimum(x.astype(np.int64), A - 1)
    keep = (x - j) < prob[rows, j]
    return np.where(keep, j, alias[rows, j]).astype(np.int32)


def markov_sequences(lengths: np.ndarray, pi0: np.ndarray, P: np.ndarray,
                     rng: np.random.Generator) -> np.ndarray:
    """Activities of every case, case-major: case k occupies off[k]..off[k]+L_k.

    The chain is advanced position by position over the cases still running
    (longest first), stored position-major so each step reads and writes one
    contiguous block; one gather then lays the sequences out case by case.
    """
    A = P.shape[0]
    C = lengths.shape[0]
    N = int(lengths.sum())
    if N == 0:
        return np.zeros(0, np.int32)
    order = np.argsort(-lengths, kind="stable")   # longest cases first
    rank = np.empty(C, np.int64)
    rank[order] = np.arange(C)
    sorted_len = lengths[order]
    max_len = int(sorted_len[0])
    # n_k = cases with L > k, for k = 0 .. max_len-1
    n_k = np.searchsorted(-sorted_len, -np.arange(max_len), side="left")
    block = np.zeros(max_len + 1, np.int64)
    np.cumsum(n_k, out=block[1:])
    tables = [alias_table(P[r]) for r in range(A)]
    prob = np.stack([t[0] for t in tables])
    alias = np.stack([t[1] for t in tables])
    p0, a0 = alias_table(pi0)
    pm = np.empty(N, np.int32)
    n0 = int(n_k[0])
    pm[:n0] = _sample_alias(p0[None, :], a0[None, :], np.zeros(n0, np.int64), rng.random(n0))
    for k in range(1, max_len):
        n = int(n_k[k])
        prev = pm[block[k - 1]:block[k - 1] + n]
        pm[block[k]:block[k] + n] = _sample_alias(prob, alias, prev, rng.random(n))
    off = np.zeros(C + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    within = np.arange(N, dtype=np.int64) - np.repeat(off[:-1], lengths)
    return pm[block[within] + np.repeat(rank, lengths)]


def make_log(*, n_cases: int, length_law: str, A: int, act_law: str, unit: str,
             gap_mean: float, dup_p: float, presorted: bool, seed: int,
             name: str = "") -> Log:
    """Draw one log.

    length_law: "geom10" (Geometric(p=0.1) on 1, 2, ...) or
                "lognorm12" (round(LogNormal(ln 12, 1)) clipped to [1, 2000]).
    act_law:    "dirichlet" (pi0 and rows of P ~ Dirichlet(1)) or
                "zipf" (Zipf(1.1) stationary mix, P = 0.5 pi + 0.5 Dirichlet(1)).
    unit:       "ms" or "ns"; case starts are uniform over one year.
    gap_mean:   mean of the exponential gap, in the unit.
    dup_p:      probability that a non-first event copies its predecessor's time.
    """
    rng = np.random.default_rng(seed)
    C = n_cases
    if length_law == "geom10":
        lengths = rng.geometric(0.1, size=C).astype(np.int64)
    elif length_law == "lognorm12":
        lengths = np.clip(np.rint(rng.lognormal(np.log(12.0), 1.0, size=C)), 1, 2000).astype(np.int64)
    else:
        raise ValueError(length_law)
    pi0, P = markov_chain(A, act_law, rng)
    acts = markov_sequences(lengths, pi0, P, rng)
    N = int(lengths.sum())

    if unit == "ms":
        t0, year = 1_600_000_000_000, 365 * DAY_MS
    elif unit == "ns":
        t0, year = 1_600_000_000_000_000_000, 365 * DAY_NS
    else:
        raise ValueError(unit)
    case_start = t0 + rng.integers(0, year, size=C, dtype=np.int64)
    gaps = np.floor(rng.exponential(gap_mean, size=N)).astype(np.int64)
    if dup_p > 0:
        gaps[rng.random(N) < dup_p] = 0
    off = np.zeros(C + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    gaps[off[:-1]] = 0
    cs = np.cumsum(gaps)
    within = cs - np.repeat(cs[off[:-1]], lengths)
    ts = np.repeat(case_start, lengths) + within

    codes = rng.permutation(C).astype(np.int32)    # generated case k gets code codes[k]
    case = np.repeat(codes, lengths)
    lengths_by_code = np.empty(C, dtype=np.int64)
    lengths_by_code[codes] = lengths

    if presorted:
        # cases laid out by ascending code, each case in generation (time) order
        rows = np.argsort(case, kind="stable")
    else:
        rows = rng.permutation(N)
    return Log(case=np.ascontiguousarray(case[rows]), act=np.ascontiguousarray(acts[rows]),
               ts=np.ascontiguousarray(ts[rows]), n_activities=A, presorted=presorted,
               lengths_by_code=lengths_by_code, name=name)


# The five workloads.  scale < 1 shrinks the case count (same laws), for tests.
def config_log(k: int, scale: float = 1.0) -> Log:
    seed = SEED_BASE + k
    if k == 1:
        return make_log(n_cases=max(1, int(10_000 * scale)), length_law="geom10", A=16,
                        act_law="dirichlet", unit="ms", gap_mean=3_600_000.0, dup_p=0.0,
                        presorted=True, seed=seed, name="plain-dfg-10k-cases-A16-presorted")
    if k == 2:
        return make_log(n_cases=max(1, int(1_000_000 * scale)), length_law="geom10", A=64,
                        act_law="zipf", unit="ms", gap_mean=3_600_000.0, dup_p=0.05,
                        presorted=False, seed=seed, name="dfg-perf-1M-cases-A64-zipf-shuffled")
    if k == 3:
        return make_log(n_cases=max(1, int(5_000_000 * scale)), length_law="lognorm12", A=512,
                        act_law="zipf", unit="ns", gap_mean=1e10, dup_p=0.0,
                        presorted=False, seed=seed, name="dfg-variants-5M-cases-A512-ns-shuffled")
    raise ValueError(k)


@dataclasses.dataclass
class Views:
    """Drill-down views: case-code range [lo, hi), closed time window, activity mask."""

    case_lo: np.ndarray   # int32 [V]
    case_hi: np.ndarray   # int32 [V]
    t_lo: np.ndarray      # int64 [V]
    t_hi: np.ndarray      # int64 [V]
    masks: np.ndarray     # uint64 [V, W], W = ceil(A / 64)

    @property
    def n_views(self) -> int:
        return int(self.case_lo.shape[0])

    def packed(self) -> np.ndarray:
        """[V] records of (int32 lo, int32 hi, int64 t_lo, int64 t_hi) = 24 bytes."""
        rec = np.zeros(self.n_views, dtype=np.dtype([("lo", "<i4"), ("hi", "<i4"),
                                                     ("t_lo", "<i8"), ("t_hi", "<i8")]))
        rec["lo"], rec["hi"], rec["t_lo"], rec["t_hi"] = self.case_lo, self.case_hi, self.t_lo, self.t_hi
        return rec


def make_views(log: Log, n_views: int, seed: int, min_events: float = 1e3,
               max_events: float = 2e7) -> Views:
    """Views over a log whose case codes are dense 0..C-1.

    Slice size S is log-uniform in [min_events, max_events] (capped at N); the
    case range starts at a uniform case code and grows until it holds at least
    S events.  The time window covers a fraction f ~ U(0.05, 1) of the log's
    time span at a uniform position; the activity subset has k ~ U{8..A}
    members drawn without replacement.
    """
    rng = np.random.default_rng(seed)
    A = log.n_activities
    W = (A + 63) // 64
    lengths = log.lengths_by_code
    C = lengths.shape[0]
    N = int(lengths.sum())
    cum = np.zeros(C + 1, dtype=np.int64)
    np.cumsum(lengths, out=cum[1:])
    t_min, t_max = int(log.ts.min()), int(log.ts.max())
    span = t_max - t_min
    lo = np.empty(n_views, np.int32)
    hi = np.empty(n_views, np.int32)
    tl = np.empty(n_views, np.int64)
    th = np.empty(n_views, np.int64)
    masks = np.zeros((n_views, W), np.uint64)
    hi_cap = min(max_events, N)
    lo_cap = min(min_events, hi_cap)
    for v in range(n_views):
        S = int(round(np.exp(rng.uniform(np.log(lo_cap), np.log(max(hi_cap, lo_cap))))))
        p = int(rng.integers(0, C))
        need = cum[p] + S
        h = int(np.searchsorted(cum, need, side="left"))
        h = min(max(h, p + 1), C)
        if cum[h] - cum[p] < S:   # ran off the end: extend downwards
            p = int(np.searchsorted(cum, cum[h] - S, side="right")) - 1
            p = max(p, 0)
        lo[v], hi[v] = p, h
        f = rng.uniform(0.05, 1.0)
        w = int(f * span)
        tl[v] = t_min + int(rng.integers(0, max(1, span - w + 1)))
        th[v] = tl[v] + w
        k = int(rng.integers(min(8, A), A + 1))
        sub = rng.choice(A, size=k, replace=False)
        for a in sub:
            masks[v, a // 64] |= np.uint64(1) << np.uint64(a % 64)
    return Views(case_lo=lo, case_hi=hi, t_lo=tl, t_hi=th, masks=masks)


def _digits(x: np.ndarray, width: int) -> np.ndarray:
    """[n, width] ASCII decimal digits of non-negative x, zero-padded."""
    out = np.empty((x.shape[0], width), dtype=np.uint8)
    v = x.astype(np.int64).copy()
    for k in range(width - 1, -1, -1):
        out[:, k] = (v % 10).astype(np.uint8) + ord("0")
        v //= 10
    return out


def log_csv(log: Log, unit: str = "ms", iso: bool = True) -> bytes:
    """The log as CSV text (header "case,activity,timestamp", LF line ends,
    rows in the log's row order): case "c" + 10 digits of the case id plus
    2^31, activity "Activity " + 4 digits, timestamp ISO-8601 UTC with 3 (ms)
    or 9 (ns) fraction digits, or the integer itself.  Fixed-width fields,
    built column by column with numpy."""
    n = log.n_events
    case_f = np.concatenate([np.full((n, 1), ord("c"), np.uint8),
                             _digits(log.case.astype(np.int64) + 2**31, 10)], axis=1)
    act_f = np.concatenate([np.frombuffer(b"Activity ", np.uint8)[None, :].repeat(n, axis=0),
                            _digits(log.act, 4)], axis=1)
    if iso:
        dt = log.ts.astype("datetime64[ms]" if unit == "ms" else "datetime64[ns]")
        s = np.datetime_as_string(dt, unit="ms" if unit == "ms" else "ns", timezone="UTC")
        w = len(s[0]) if n else 0
        ts_f = np.frombuffer(s.astype(f"S{w}").tobytes(), np.uint8).reshape(n, w)
    else:
        neg = log.ts < 0
        mag = np.where(neg, -log.ts, log.ts)
        ts_f = np.concatenate([np.where(neg, ord("-"), ord("+")).astype(np.uint8)[:, None], _digits(mag, 19)],
                              axis=1)
    comma = np.full((n, 1), ord(","), np.uint8)
    nl = np.full((n, 1), ord("\n"), np.uint8)
    body = np.concatenate([case_f, comma, act_f, comma, ts_f, nl], axis=1)
    return b"case,activity,timestamp\n" + body.tobytes()
