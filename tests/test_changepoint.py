"""Changepoint detection of Sec. 4.5 (Algorithm 1 and the sequential method) on seeded
synthetic series: statistics against SciPy's textbook routines, detection of planted
steps at the planted index, robustness to single outliers, no detections on most
change-free series, and the ratio intervals of eq. (mean-transform)."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2204_04321_amd import changepoint as cp


def test_t_statistic_is_the_pooled_two_sample_t():
    rng = np.random.default_rng(0)
    for n1, n2 in ((3, 5), (10, 17), (40, 2)):
        a, b = rng.normal(1.0, 0.3, n1), rng.normal(1.2, 0.5, n2)
        ref = stats.ttest_ind(b, a, equal_var=True).statistic
        assert cp.t_statistic(a, b) == pytest.approx(ref, rel=1e-12)


def test_algorithm1_finds_a_planted_step_at_its_index():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0.0, 1.0, 25), rng.normal(4.0, 1.0, 15)])
    C, S = cp.changepoint(x)
    assert 25 in C and abs(S[25]) > stats.t.ppf(1 - cp.ALPHA / (2 * cp.K_LARGEST), x.size - 2)
    # the critical value: two-sided, Bonferroni over k tests, n - 2 degrees of freedom
    assert S[25] > 0


def test_algorithm1_tests_only_the_k_largest_jumps():
    x = np.array([0.0] * 10 + [5.0] * 10)
    x[3] = 0.01                        # tiny jumps elsewhere
    C, _ = cp.changepoint(x, k=1, outliers=False)
    assert C == [10]


def test_change_free_series_rarely_fire():
    """On change-free normal series of 30 values, Algorithm 1 fires on ~1% of series without
    the outlier rule and ~3.5% with it (measured on 1000 series): the Bonferroni level
    covers the k tests, not their selection as the largest jumps, and the MAD rule can
    shrink a short sample's spread."""
    rng = np.random.default_rng(2)
    X = [rng.normal(0, 1, 30) for _ in range(400)]
    assert sum(bool(cp.changepoint(x, outliers=False)[0]) for x in X) <= 10
    assert sum(bool(cp.changepoint(x)[0]) for x in X) <= 24


def test_consecutive_detections_suppress_false_changepoints():
    """The sequential method tests every prefix, so single detections accumulate over a
    series; m = 3 consecutive detections of one position keep most of them out."""
    rng = np.random.default_rng(3)
    Y = [np.exp(rng.normal(0, 0.05, 60)) for _ in range(150)]
    r1 = sum(bool(cp.detect(y, m=1).changepoints) for y in Y)
    r3 = sum(bool(cp.detect(y).changepoints) for y in Y)
    assert r3 < r1 and r3 <= 0.25 * len(Y), (r1, r3)


def test_drop_outliers_rule():
    a = np.array([1.0, 1.1, 0.9, 1.05, 0.95, 50.0, 1.02, 0.98, 1.01, 0.99])
    b = np.array([2.0, 2.1, 1.9, 2.05, -40.0, 1.95, 2.02, 1.98, 2.01, 1.99])
    a2, b2 = cp.drop_outliers(a, b)
    assert 50.0 not in a2 and -40.0 not in b2 and a2.size + b2.size == 18
    # at most 10% of the data: with 12 values only one may go, the one with the largest
    # MAD score (50 lies 441 robust standard deviations out, -40 lies 377)
    a3, b3 = cp.drop_outliers(a[:6], np.array([2.0, 2.1, 1.9, 2.05, -40.0, 1.95]))
    assert a3.size + b3.size == 11 and 50.0 not in a3 and -40.0 in b3


def test_sequential_detection_confirms_a_step_after_m_detections():
    rng = np.random.default_rng(3)
    x = np.exp(np.concatenate([rng.normal(0.0, 0.02, 40), rng.normal(0.2, 0.02, 30)]))
    det = cp.detect(x)
    assert det.changepoints == [40]
    assert det.confirmed_at[40] >= 40 + cp.M_CONSECUTIVE - 1
    segs, ratios = cp.segment_ratios(x, det.changepoints)
    assert ratios[0]["ci"][0] < math.exp(0.2) < ratios[0]["ci"][1]
    assert len(segs) == 2 and segs[1]["geomean"] == pytest.approx(math.exp(0.2), rel=0.02)


def test_single_outlier_is_not_confirmed():
    rng = np.random.default_rng(4)
    x = np.exp(rng.normal(0.0, 0.02, 60))
    x[30] *= 1.5
    assert cp.detect(x).changepoints == []


def test_two_steps_found_in_order():
    rng = np.random.default_rng(5)
    x = np.exp(np.concatenate([rng.normal(0.0, 0.02, 35), rng.normal(-0.15, 0.02, 35),
                               rng.normal(0.1, 0.02, 35)]))
    assert cp.detect(x).changepoints == [35, 70]


def test_ratio_interval_matches_scipy():
    rng = np.random.default_rng(6)
    a, b = np.exp(rng.normal(0, 0.1, 20)), np.exp(rng.normal(0.3, 0.1, 25))
    r, (lo, hi) = cp.ratio_ci(a, b)
    la, lb = np.log(a), np.log(b)
    d = lb.mean() - la.mean()
    se = math.sqrt((((la - la.mean()) ** 2).sum() + ((lb - lb.mean()) ** 2).sum()) / 43 * (1 / 20 + 1 / 25))
    ref = stats.t.interval(0.99, 43, loc=d, scale=se)
    assert r == pytest.approx(math.exp(d), rel=1e-12)
    assert (lo, hi) == pytest.approx((math.exp(ref[0]), math.exp(ref[1])), rel=1e-12)


def test_paired_comparison_finds_where_the_ratio_changes():
    rng = np.random.default_rng(7)
    base = np.exp(rng.normal(1.0, 0.2, 80))          # shared day-to-day variation
    a = base * np.exp(rng.normal(0, 0.01, 80))
    ratio = np.where(np.arange(80) < 50, 2.0, 7.0)
    b = a / ratio * np.exp(rng.normal(0, 0.01, 80))
    det, subsets = cp.paired(a, b)
    assert det.changepoints == [50]
    assert subsets[0]["ci"][0] < 2.0 < subsets[0]["ci"][1]
    assert subsets[1]["ci"][0] < 7.0 < subsets[1]["ci"][1]


def test_cli_reads_bench_json_lines(tmp_path, capsys):
    rng = np.random.default_rng(9)
    vals = np.exp(np.concatenate([rng.normal(0, 0.01, 20), rng.normal(0.3, 0.01, 15)]))
    p = tmp_path / "h.jsonl"
    p.write_text("".join(f'{{"value": {v}, "date": "d{i}"}}\n' for i, v in enumerate(vals)))
    cp.main([str(p)])
    out = capsys.readouterr().out
    import json
    rec = json.loads(out)
    assert [c["index"] for c in rec["changepoints"]] == [20] and rec["changepoints"][0]["tag"] == "d20"
