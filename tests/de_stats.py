"""Statistics helpers for comparing DE result distributions.

``rank_scores`` is the scoring rule of Section 7.3.5 of arXiv 2405.16551:
rank all n*m trials of m algorithms together, best trial gets rank n*m,
ties share their average rank, an algorithm's score is the sum of its ranks
minus n(n+1)/2.  With two algorithms the score is the Mann-Whitney U count.
"""
from __future__ import annotations

import numpy as np
from scipy import stats


def rank_scores(groups, lower_is_better: bool = True):
    groups = [np.asarray(g, dtype=np.float64) for g in groups]
    n = len(groups[0])
    assert all(len(g) == n for g in groups), "equal trial counts expected"
    allv = np.concatenate(groups)
    # rankdata gives rank 1 to the smallest; the best must get the largest
    key = -allv if lower_is_better else allv
    ranks = stats.rankdata(key, method="average")
    out, k = [], 0
    for g in groups:
        out.append(float(ranks[k:k + len(g)].sum() - n * (n + 1) / 2))
        k += len(g)
    return out


def same_distribution(a, b, floor: float = 1e-8, alpha: float = 0.01):
    """Two-sided rank test (the paper's rank score, i.e. Mann-Whitney U) and
    a KS test on log10 of values floored at the success threshold."""
    la = np.log10(np.maximum(np.asarray(a, dtype=np.float64), floor))
    lb = np.log10(np.maximum(np.asarray(b, dtype=np.float64), floor))
    if np.array_equal(np.sort(la), np.sort(lb)):
        return True, 1.0, 1.0
    u = stats.mannwhitneyu(la, lb, alternative="two-sided")
    ks = stats.ks_2samp(la, lb)
    return (u.pvalue > alpha and ks.pvalue > alpha), float(u.pvalue), float(
        ks.pvalue)
