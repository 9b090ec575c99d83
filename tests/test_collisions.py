"""Collision statistics of the downsampled spectrum (Sec. II-C, Lemma 2,
Fig. 2), from the input generator's supports (CPU).

* the number of frequencies sharing a frequency's bin follows the
  hypergeometric law the autotuner's recovery model uses (K - 1 others among
  N - 1 positions, d - 1 of them in the bin), per N+ = N/(dK);
* Fig. 2's reading: at N+ >= 2 collisions of more than 4 are rare (under 1%
  of frequencies) and more than 2 uncommon (under 10%);
* Lemma 2: the probability that some bin holds more than a_m frequencies
  stays below (N/d) (d e K / (N (a_m + 1)))^(a_m + 1).
"""
import math

import numpy as np
import pytest
from scipy.stats import hypergeom

import sftgen


def occupancy_per_frequency(n, k, m, trials, seed0):
    """Histogram (a = 1, 2, ...) of the size of each frequency's bin."""
    hist = np.zeros(k + 1)
    for t in range(trials):
        locs, _, _ = sftgen.draw_spectrum(n, k, seed0 + t)
        per_bin = np.bincount(locs % m, minlength=m)
        a = per_bin[locs % m]
        hist += np.bincount(a, minlength=k + 1)[:k + 1]
    return hist / hist.sum()


@pytest.mark.parametrize("n_plus", [1, 2, 4])
def test_bin_occupancy_is_hypergeometric(n_plus):
    n, k = 1 << 16, 1 << 10
    m = n_plus * k
    d = n // m
    emp = occupancy_per_frequency(n, k, m, 40, 100 * n_plus)
    for a in range(1, 6):
        p = hypergeom.pmf(a - 1, n - 1, d - 1, k - 1)
        sd = math.sqrt(p * (1 - p) / (40 * k)) * 3.0   # frequencies of one signal are not independent
        assert abs(emp[a] - p) <= 4 * sd + 1e-4, (a, emp[a], p)


@pytest.mark.parametrize("n_plus", [2, 4, 8])
def test_fig2_reading(n_plus):
    n, k = 1 << 16, 1 << 10
    emp = occupancy_per_frequency(n, k, n_plus * k, 20, 7000 + n_plus)
    assert emp[5:].sum() < 0.01
    assert emp[3:].sum() < 0.10


@pytest.mark.parametrize("n_plus,a_m", [(1, 4), (2, 3), (4, 2), (8, 2)])
def test_lemma2_bound(n_plus, a_m):
    n, k = 1 << 16, 1 << 10
    m = n_plus * k
    d = n // m
    bound = (n / d) * (d * math.e * k / (n * (a_m + 1))) ** (a_m + 1)
    hits = 0
    trials = 200
    for t in range(trials):
        locs, _, _ = sftgen.draw_spectrum(n, k, 9000 + 1000 * n_plus + t)
        hits += np.bincount(locs % m, minlength=m).max() > a_m
    assert hits / trials <= min(1.0, bound) + 3 * math.sqrt(0.25 / trials)
