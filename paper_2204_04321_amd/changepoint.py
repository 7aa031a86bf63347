"""Changepoint detection over benchmark time series (arXiv:2204.04321, Sec. 4.5).

The paper's nightly performance tests record a wall-clock metric per day and look for
abrupt, statistically significant changes in it.  This module does the same for the JSON
lines that `bench.py` prints (or any series of positive timings/throughputs):

* `changepoint(x, alpha, k)` - the single-changepoint test of the paper's Algorithm 1:
  the k largest jumps |x_(i+1) - x_i| are the candidate positions nu; for each, a
  two-sample t-test compares x_1 .. x_(nu-1) with x_nu .. x_n, and nu is a changepoint
  when |t| exceeds the two-sided critical value with the Bonferroni-adjusted level
  alpha / k (n - 2 degrees of freedom).
* `detect(series, ...)` - the sequential multiple-changepoint method of Sec. 4.5: the
  series is read in time order, each step tests the window of at most w observations
  since the last confirmed changepoint, a candidate is confirmed after m consecutive
  detections, data before a confirmed changepoint are no longer tested, values are
  log-transformed, and every t-test first drops outliers by the median absolute
  deviation (threshold ~3 standard deviations, at most 10% of the data).
* `segment_ratios` - relative performance between consecutive segments as
  exp(mean log x_after - mean log x_before) (eq. mean-transform) with a 99% t-interval.
* `paired(a, b)` - the paired comparison of two tests joined by date: the log
  differences are searched for changepoints and each subset's mean gets a 99% interval.

Readings where the paper is silent: the t-test is Student's pooled-variance test (its
n - 2 degrees of freedom match the critical value of Algorithm 1); the MAD threshold is
3 x 1.4826 x MAD (1.4826 MAD estimates the standard deviation of normal data); when more
than 10% of a test's data lie beyond it, only the 10% furthest from their median are
dropped; when several candidates are confirmed at one step, the one tested first (the
largest jump) is taken: the outlier rule can make a position next to a step significant
too, when the step's first value on the far side is dropped as an outlier.

Defaults are the paper's: alpha = 0.005, k = 10, m = 3, w = 30.

    python -m paper_2204_04321_amd.changepoint history.jsonl --key value [--alpha A] [-k K] [-m M] [-w W]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
from dataclasses import dataclass, field

import numpy as np
from scipy import stats

ALPHA, K_LARGEST, M_CONSECUTIVE, W_LOOKBACK = 0.005, 10, 3, 30
MAD_SIGMAS, MAD_TO_SIGMA, MAX_OUTLIER_FRAC = 3.0, 1.4826, 0.10


def drop_outliers(a: np.ndarray, b: np.ndarray, sigmas: float = MAD_SIGMAS,
                  max_frac: float = MAX_OUTLIER_FRAC):
    """Both samples of a t-test without their outliers: points further than `sigmas`
    MAD-estimated standard deviations from their own sample's median, at most
    floor(max_frac * (len(a) + len(b))) points in all (the furthest ones)."""
    budget = int(math.floor(max_frac * (a.size + b.size)))
    if budget == 0:
        return a, b
    scores = []
    for tag, s in ((0, a), (1, b)):
        med = np.median(s)
        mad = np.median(np.abs(s - med)) * MAD_TO_SIGMA
        z = np.abs(s - med) / mad if mad > 0 else np.zeros(s.size)
        for i in np.nonzero(z > sigmas)[0]:
            scores.append((float(z[i]), tag, int(i)))
    scores.sort(reverse=True)
    drop = [set(), set()]
    for _, tag, i in scores[:budget]:
        drop[tag].add(i)
    keep = lambda s, d: s[np.array([i not in d for i in range(s.size)], dtype=bool)] if d else s
    return keep(a, drop[0]), keep(b, drop[1])


def t_statistic(a: np.ndarray, b: np.ndarray) -> float:
    """Student's two-sample t statistic with the pooled variance (0 when undefined)."""
    n1, n2 = a.size, b.size
    if n1 < 1 or n2 < 1 or n1 + n2 < 3:
        return 0.0
    ss = ((a - a.mean()) ** 2).sum() + ((b - b.mean()) ** 2).sum()
    sp2 = ss / (n1 + n2 - 2)
    diff = b.mean() - a.mean()
    if sp2 <= 0:
        return 0.0 if diff == 0 else math.copysign(math.inf, diff)
    return float(diff / math.sqrt(sp2 * (1.0 / n1 + 1.0 / n2)))


def changepoint(x, alpha: float = ALPHA, k: int = K_LARGEST, outliers: bool = True):
    """Algorithm 1.  x: values x_1 .. x_n (already log-transformed if wanted).  Returns
    (C, S): the changepoints nu as 0-based indices of the first value after the change
    (x[:nu] vs x[nu:]), in the order tested, and their t statistics."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 3:
        return [], {}
    k = max(1, min(k, n - 1))
    t_crit = stats.t.ppf(1.0 - alpha / (2.0 * k), n - 2)
    jumps = np.abs(np.diff(x))
    cand = 1 + np.argsort(-jumps, kind="stable")       # nu: start of the second segment
    C, S = [], {}
    for nu in cand[:k]:
        a, b = x[:nu], x[nu:]
        if outliers:
            a, b = drop_outliers(a, b)
        t = t_statistic(a, b)
        if abs(t) > t_crit:
            C.append(int(nu))
            S[int(nu)] = t
    return C, S


@dataclass
class Detection:
    changepoints: list = field(default_factory=list)   # confirmed, 0-based indices into the series
    tstats: dict = field(default_factory=dict)         # t statistic at confirmation
    confirmed_at: dict = field(default_factory=dict)   # index of the observation that confirmed it


def detect(series, alpha: float = ALPHA, k: int = K_LARGEST, m: int = M_CONSECUTIVE,
           w: int = W_LOOKBACK, log: bool = True, outliers: bool = True) -> Detection:
    """Sequential multiple-changepoint detection (Sec. 4.5) over the series in time order."""
    x = np.log(np.asarray(series, dtype=np.float64)) if log else np.asarray(series, dtype=np.float64)
    det = Detection()
    start = 0
    streak: dict[int, int] = {}
    for end in range(1, x.size + 1):
        lo = max(start, end - w)
        C, S = changepoint(x[lo:end], alpha, k, outliers)
        found = {lo + c: S[c] for c in C if lo + c > start}     # in the order tested
        streak = {nu: streak.get(nu, 0) + 1 for nu in found}
        ready = [nu for nu in found if streak[nu] >= m]
        if ready:
            nu = ready[0]
            det.changepoints.append(nu)
            det.tstats[nu] = found[nu]
            det.confirmed_at[nu] = end - 1
            start = nu
            streak = {}
    return det


def mean_log_ci(v, level: float = 0.99):
    """Mean of v with its t-interval (half-width 0 for a single value)."""
    v = np.asarray(v, dtype=np.float64)
    mu = float(v.mean())
    if v.size < 2:
        return mu, (mu, mu)
    h = stats.t.ppf(0.5 + level / 2, v.size - 1) * v.std(ddof=1) / math.sqrt(v.size)
    return mu, (mu - h, mu + h)


def ratio_ci(before, after, level: float = 0.99):
    """exp(mean log after - mean log before) (eq. mean-transform) with the pooled
    two-sample t-interval of the difference of the log means."""
    a = np.log(np.asarray(before, dtype=np.float64))
    b = np.log(np.asarray(after, dtype=np.float64))
    d = b.mean() - a.mean()
    n1, n2 = a.size, b.size
    if n1 + n2 < 3:
        return float(math.exp(d)), (float(math.exp(d)), float(math.exp(d)))
    sp2 = (((a - a.mean()) ** 2).sum() + ((b - b.mean()) ** 2).sum()) / (n1 + n2 - 2)
    h = stats.t.ppf(0.5 + level / 2, n1 + n2 - 2) * math.sqrt(sp2 * (1 / n1 + 1 / n2))
    return float(math.exp(d)), (float(math.exp(d - h)), float(math.exp(d + h)))


def segment_ratios(series, changepoints, level: float = 0.99):
    """Per segment between changepoints: geometric mean and its interval; per changepoint:
    the ratio after / before with its interval."""
    x = np.asarray(series, dtype=np.float64)
    bounds = [0] + list(changepoints) + [x.size]
    segs = []
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        mu, (l, u) = mean_log_ci(np.log(x[lo:hi]), level)
        segs.append({"begin": lo, "end": hi, "geomean": math.exp(mu), "ci": [math.exp(l), math.exp(u)]})
    ratios = []
    for i, nu in enumerate(changepoints):
        r, ci = ratio_ci(x[bounds[i]:nu], x[nu:bounds[i + 2]], level)
        ratios.append({"at": nu, "ratio": r, "ci": list(ci)})
    return segs, ratios


def paired(a, b, level: float = 0.99, **kw):
    """Paired comparison of two tests observed on the same dates: d = log a - log b, its
    changepoints, and per subset the ratio exp(mean d) with its one-sample t-interval."""
    d = np.log(np.asarray(a, dtype=np.float64)) - np.log(np.asarray(b, dtype=np.float64))
    det = detect(d, log=False, **kw)
    bounds = [0] + det.changepoints + [d.size]
    out = []
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        mu, (l, u) = mean_log_ci(d[lo:hi], level)
        out.append({"begin": lo, "end": hi, "ratio": math.exp(mu), "ci": [math.exp(l), math.exp(u)]})
    return det, out


def _load(path, key):
    vals, tags = [], []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            rec = json.loads(line)
            v = rec
            for part in key.split("."):
                v = v[part]
            vals.append(float(v))
            tags.append(rec.get("date", rec.get("commit", len(tags))))
    return np.array(vals), tags


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("history", help="JSON lines, one benchmark record per line, oldest first")
    ap.add_argument("--key", default="value", help="dotted key of the metric in each record")
    ap.add_argument("--alpha", type=float, default=ALPHA)
    ap.add_argument("-k", type=int, default=K_LARGEST)
    ap.add_argument("-m", type=int, default=M_CONSECUTIVE)
    ap.add_argument("-w", type=int, default=W_LOOKBACK)
    a = ap.parse_args(argv)
    x, tags = _load(a.history, a.key)
    det = detect(x, a.alpha, a.k, a.m, a.w)
    segs, ratios = segment_ratios(x, det.changepoints)
    print(json.dumps({"n": int(x.size), "changepoints": [{"index": nu, "tag": tags[nu], "t": det.tstats[nu],
                                                          "confirmed_at": det.confirmed_at[nu]}
                                                         for nu in det.changepoints],
                      "segments": segs, "ratios": ratios}, indent=1, default=str))


if __name__ == "__main__":
    sys.exit(main())
