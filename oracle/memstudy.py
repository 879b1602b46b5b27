"""Statistics of the memory-subsystem study -- oracle, test infrastructure only.

The paper's Sec. 5 measures plain buffer reads and writes over the (M, N, K) grid: read A
(M x K), read B (K x N) and write D (M x N), each in a buffer allocated on its own ("isolated")
or alongside the other operands ("co-allocated"), in sequential (nested-loop) or randomized
order.  These are the statistics it reports, written out plainly:

* Table 4 -- co-allocation slowdown per configuration (co-allocated over isolated time): its
  mean and the fractions of configurations slowed by more than 20 % and 50 %;
* Sec. 5.3 -- temporal warm-up: Spearman rank correlation of a buffer's time with run order,
  and the drift of repeated measurements of one buffer size within a sequential block;
* Sec. 5.4 -- the spurious dependence of read-A time on N (correlation with N, the coefficient
  of variation across N per (M, K), its median);
* Sec. 5.1 -- read / write bandwidth and their ratio for identical buffers.
"""
from __future__ import annotations

import math


def average_ranks(values):
    """Ranks 1..n in ascending order; tied values share the mean of the ranks they span."""
    v = [float(x) for x in values]
    order = sorted(range(len(v)), key=lambda i: v[i])
    ranks = [0.0] * len(v)
    i = 0
    while i < len(order):
        j = i
        while j + 1 < len(order) and v[order[j + 1]] == v[order[i]]:
            j += 1
        r = (i + j) / 2.0 + 1.0             # mean of positions i..j, 1-based
        for t in range(i, j + 1):
            ranks[order[t]] = r
        i = j + 1
    return ranks


def pearson(x, y) -> float:
    n = len(x)
    mx = sum(x) / n
    my = sum(y) / n
    sxy = sum((a - mx) * (b - my) for a, b in zip(x, y))
    sxx = sum((a - mx) ** 2 for a in x)
    syy = sum((b - my) ** 2 for b in y)
    return sxy / math.sqrt(sxx * syy)


def spearman(x, y) -> float:
    """Spearman rank correlation: the Pearson correlation of the average ranks."""
    return pearson(average_ranks(x), average_ranks(y))


def slowdown_summary(t_coalloc, t_isolated):
    """Table 4: per configuration the ratio co-allocated / isolated time; mean ratio and the
    fractions of configurations above 1.2 and 1.5."""
    r = [c / i for c, i in zip(t_coalloc, t_isolated)]
    n = len(r)
    return {"mean": sum(r) / n, "over_20": sum(1 for x in r if x > 1.2) / n,
            "over_50": sum(1 for x in r if x > 1.5) / n}


def median(values) -> float:
    v = sorted(float(x) for x in values)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def cv_by_group(times, keys) -> float:
    """Coefficient of variation (population standard deviation / mean) of the times sharing a
    key -- e.g. read-A times of one (M, K) across N -- and its median over the keys."""
    groups = {}
    for t, k in zip(times, keys):
        groups.setdefault(k, []).append(float(t))
    cvs = []
    for ts in groups.values():
        m = sum(ts) / len(ts)
        sd = math.sqrt(sum((t - m) ** 2 for t in ts) / len(ts))
        cvs.append(sd / m)
    return median(cvs)


def revisit_drift(times, keys, run_order) -> float:
    """Temporal warm-up (Sec. 5.3): for every key measured more than once, the relative change
    from its first to its last measurement in run order, 1 - t_last / t_first; the mean over
    keys.  Positive: the same buffer size got faster later in the sweep."""
    first, last = {}, {}
    for t, k, o in zip(times, keys, run_order):
        if k not in first or o < first[k][0]:
            first[k] = (o, float(t))
        if k not in last or o > last[k][0]:
            last[k] = (o, float(t))
    d = [1.0 - last[k][1] / first[k][1] for k in first if last[k][0] != first[k][0]]
    return sum(d) / len(d)


def bandwidth_gbs(nbytes, seconds) -> float:
    return nbytes / seconds / 1e9
