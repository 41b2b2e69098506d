"""Literal, brute-force restatement of the method's definitions, for tiny logs.

It is written independently of the C oracle so the two pin each other: no
sorting routine, no single linear walk.  The directly-follows relation is
checked by definition with an explicit search for an intermediate event
(Sec. 3: an event and the previous event of its case), cases are the
distinct case identifiers, variants are compared by list equality.
"""
from __future__ import annotations

import math

INT64_MAX = 2**63 - 1
INT64_MIN = -(2**63)


def precedes(c, t, i, j):
    """Event i comes before event j in the (case, timestamp, row) order."""
    return (c[i], t[i], i) < (c[j], t[j], j)


def to_i64(x: int) -> int:
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= (1 << 63) else x


def _by_case(c):
    groups = {}
    for i, ci in enumerate(c):
        groups.setdefault(ci, []).append(i)
    return groups


def directly_follows_pairs(c, t):
    """All (i, j) with j directly following i: same case, i before j, nothing between."""
    pairs = []
    for members in _by_case(c).values():
        for i in members:
            for j in members:
                if i == j or not precedes(c, t, i, j):
                    continue
                between = any(precedes(c, t, i, k) and precedes(c, t, k, j) for k in members if k not in (i, j))
                if not between:
                    pairs.append((i, j))
    return pairs


def trace(c, t, a, members):
    """Activities of one case, taking the earliest remaining event each time."""
    rest = list(members)
    out = []
    while rest:
        first = rest[0]
        for k in rest[1:]:
            if precedes(c, t, k, first):
                first = k
        out.append(a[first])
        rest.remove(first)
    return out


def dfg(c, a, t, A):
    cnt = [[0] * A for _ in range(A)]
    s = [[0] * A for _ in range(A)]
    mn = [[INT64_MAX] * A for _ in range(A)]
    mx = [[INT64_MIN] * A for _ in range(A)]
    for i, j in directly_follows_pairs(c, t):
        x, y = a[i], a[j]
        gap = to_i64(t[j] - t[i])
        cnt[x][y] += 1
        s[x][y] = to_i64(s[x][y] + gap)
        mn[x][y] = min(mn[x][y], gap)
        mx[x][y] = max(mx[x][y], gap)
    mean = [[(float(s[x][y]) / float(cnt[x][y]) if cnt[x][y] else math.nan) for y in range(A)] for x in range(A)]
    start = [0] * A
    end = [0] * A
    freq = [0] * A
    for i in range(len(a)):
        freq[a[i]] += 1
    span_total = 0
    groups = _by_case(c)
    for members in groups.values():
        first = [i for i in members if not any(precedes(c, t, k, i) for k in members)]
        last = [i for i in members if not any(precedes(c, t, i, k) for k in members)]
        assert len(first) == 1 and len(last) == 1
        start[a[first[0]]] += 1
        end[a[last[0]]] += 1
        span_total += t[last[0]] - t[first[0]]
    return dict(count=cnt, dt_sum=s, dt_min=mn, dt_max=mx, dt_mean=mean, start_count=start,
                end_count=end, act_count=freq, n_cases=len(groups),
                overflow=int(span_total > INT64_MAX))


def variants(c, a, t):
    groups = _by_case(c)
    classes = []   # [sequence, [case codes]]
    for code, members in groups.items():
        seq = trace(c, t, a, members)
        for cl in classes:
            if cl[0] == seq:
                cl[1].append(code)
                break
        else:
            classes.append([seq, [code]])
    classes.sort(key=lambda cl: (-len(cl[1]), min(cl[1])))
    var_id = {}
    for v, cl in enumerate(classes):
        for code in cl[1]:
            var_id[code] = v
    codes = sorted(groups)
    return dict(n_variants=len(classes), var_count=[len(cl[1]) for cl in classes],
                var_len=[len(cl[0]) for cl in classes], var_rep=[min(cl[1]) for cl in classes],
                sequences=[cl[0] for cl in classes], case_code=codes,
                case_variant=[var_id[x] for x in codes])


def view(c, a, t, A, case_lo, case_hi, t_lo, t_hi, members_of_subset):
    keep = [i for i in range(len(c)) if case_lo <= c[i] < case_hi and t_lo <= t[i] <= t_hi
            and a[i] in members_of_subset]
    out = dfg([c[i] for i in keep], [a[i] for i in keep], [t[i] for i in keep], A)
    out["n_events"] = len(keep)
    return out


def ordered_members(c, t, members):
    """Events of one case, taking the earliest remaining event each time."""
    rest = list(members)
    out = []
    while rest:
        first = rest[0]
        for k in rest[1:]:
            if precedes(c, t, k, first):
                first = k
        out.append(first)
        rest.remove(first)
    return out


def cases(c, a, t):
    """Cases dataframe by definition: for each distinct case (ascending), its
    number of events and the time from its earliest to its latest event."""
    groups = _by_case(c)
    codes = sorted(groups)
    out = {"case_code": codes, "n_events": [], "throughput": []}
    for code in codes:
        ev = ordered_members(c, t, groups[code])
        out["n_events"].append(len(ev))
        out["throughput"].append(to_i64(t[ev[-1]] - t[ev[0]]))
    return out


def filter_cases(c, a, t, min_events, max_events, min_thr, max_thr, act_set=None, path_set=None,
                 path_keep=True, contain=None, meet=None, start_set=None, end_set=None, variant_set=None,
                 variant_keep=True):
    """Events (case, act, ts) of the kept cases, cases ascending, events in order;
    a case's paths are the (a_i, a_j) of its directly-follows pairs (i, j);
    contain / meet are inclusive (lo, hi) windows the case's first and last
    timestamps must lie in / its [first, last] span must overlap."""
    groups = _by_case(c)
    pairs = directly_follows_pairs(c, t)
    var_of = {}
    if variant_set is not None:
        v = variants(c, a, t)
        var_of = dict(zip(v["case_code"], v["case_variant"]))
    kept_events = []
    n_cases = 0
    for code in sorted(groups):
        ev = ordered_members(c, t, groups[code])
        first, last = t[ev[0]], t[ev[-1]]
        thr = to_i64(last - first)
        keep = min_events <= len(ev) <= max_events and min_thr <= thr <= max_thr
        if keep and contain is not None:
            keep = contain[0] <= first and last <= contain[1]
        if keep and meet is not None:
            keep = first <= meet[1] and last >= meet[0]
        if keep and act_set is not None:
            keep = any(a[i] in act_set for i in ev)
        if keep and path_set is not None:
            has = any((a[i], a[j]) in path_set for (i, j) in pairs if c[i] == code)
            keep = has if path_keep else not has
        if keep and start_set is not None:
            keep = a[ev[0]] in start_set
        if keep and end_set is not None:
            keep = a[ev[-1]] in end_set
        if keep and variant_set is not None:
            keep = (var_of[code] in variant_set) == bool(variant_keep)
        if keep:
            n_cases += 1
            kept_events += [(c[i], a[i], t[i]) for i in ev]
    return kept_events, n_cases


def filter_df_events(c, a, t, pair_set, side, keep):
    """Events (case, act, ts) kept by the directly-follows-level filter, in
    (case, timestamp, row) order: an event matches when it is the target
    (side 0) or the source (side 1) of a directly-follows pair whose
    activities are in pair_set."""
    matched = set()
    for i, j in directly_follows_pairs(c, t):
        if (a[i], a[j]) in pair_set:
            matched.add(j if side == 0 else i)
    kept = []
    for code, members in sorted(_by_case(c).items()):
        for i in ordered_members(c, t, members):
            if (i in matched) == bool(keep):
                kept.append((c[i], a[i], t[i]))
    return kept, len({e[0] for e in kept})


def efg(c, a, t, A):
    """Eventually-follows pairs by enumeration with Python integers: per cell
    the count, the exact gap sum S and squared-gap sum Q; n_pairs."""
    count = [[0] * A for _ in range(A)]
    S = [[0] * A for _ in range(A)]
    Q = [[0] * A for _ in range(A)]
    pairs = 0
    for code, members in _by_case(c).items():
        ev = ordered_members(c, t, members)
        for x in range(len(ev)):
            for y in range(x + 1, len(ev)):
                i, j = ev[x], ev[y]
                d = t[j] - t[i]
                count[a[i]][a[j]] += 1
                S[a[i]][a[j]] += d
                Q[a[i]][a[j]] += d * d
                pairs += 1
    return dict(count=count, S=S, Q=Q, n_pairs=pairs)
