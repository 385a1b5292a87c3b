"""Small helpers for distribution (law) tests of the oracle."""
from fractions import Fraction

import numpy as np


def chi2_ok(counts, probs, min_expected=5.0, crit_per_dof=None):
    """Pearson chi-square of observed counts against exact probabilities.

    Cells with probability zero must have zero count.  Cells with small
    expected counts are pooled.  Returns (ok, chi2, dof).  The acceptance bound
    is the chi-square quantile at p = 1e-6 (Wilson-Hilferty approximation), so
    a correct oracle passes with overwhelming probability for the fixed seeds
    used and any real mistake (wrong term, index or sign) fails by far.
    """
    counts = np.asarray(counts, dtype=np.float64)
    probs = np.asarray([float(p) for p in probs], dtype=np.float64)
    total = counts.sum()
    if np.any((probs == 0) & (counts > 0)):
        return False, float("inf"), 0
    keep = probs > 0
    counts, probs = counts[keep], probs[keep]
    exp = probs * total
    order = np.argsort(exp)
    pooled_c, pooled_e = [], []
    acc_c = acc_e = 0.0
    for idx in order:
        acc_c += counts[idx]
        acc_e += exp[idx]
        if acc_e >= min_expected:
            pooled_c.append(acc_c)
            pooled_e.append(acc_e)
            acc_c = acc_e = 0.0
    if acc_e > 0 and pooled_e:
        pooled_c[-1] += acc_c
        pooled_e[-1] += acc_e
    pooled_c, pooled_e = np.array(pooled_c), np.array(pooled_e)
    dof = max(len(pooled_c) - 1, 1)
    chi2 = float(((pooled_c - pooled_e) ** 2 / pooled_e).sum())
    z = 4.753  # normal quantile at 1 - 1e-6
    crit = dof * (1 - 2 / (9 * dof) + z * np.sqrt(2 / (9 * dof))) ** 3
    return chi2 <= crit, chi2, dof


def frac_weights(w):
    return [Fraction(float(x)) for x in w]
