"""The plan autotuner (host only, no GPU): its recovery model against
scipy's binomial and hypergeometric distributions, the minimality of the
chosen M at the chosen L, and argument validation.

Model pinned here: a frequency is recovered when its bin holds at most L of
the K frequencies; the number of other frequencies in its bin is
hypergeometric (N - 1 other positions, d - 1 of them in the bin, K - 1
drawn)."""
import numpy as np
import pytest
from scipy import stats

import sftgen

pytestmark = []


@pytest.fixture(scope="module")
def sft():
    from paper_1407_8315_amd import _lib

    if not __import__("os").path.exists(_lib.LIB_PATH):
        from paper_1407_8315_amd import build

        build.build(verbose=False)
    import paper_1407_8315_amd as m

    return m


def binom_recovery(n, k, m, L):
    d = n // m
    return float(stats.binom.cdf(L - 1, k - 1, (d - 1) / (n - 1)))


def hyper_recovery(n, k, m, L):
    d = n // m
    return float(stats.hypergeom.cdf(L - 1, n - 1, d - 1, k - 1))


CASES = [(1 << 20, 1000), (1 << 14, 50), (1 << 24, 1 << 10), (1 << 24, 1 << 12), (1 << 24, 1 << 14),
         (1 << 14, 16), (1 << 22, 4096), (1 << 16, 1024), (1 << 18, 37)]


@pytest.mark.parametrize("n,k", CASES)
@pytest.mark.parametrize("target", [0.0, 0.99, 0.9999])
def test_choice_meets_target_and_is_smallest(sft, n, k, target):
    m, L, rec, us = sft.autotune(n, k, target=target)
    t = 0.999 if target == 0.0 else target
    assert n % m == 0 and (m & (m - 1)) == 0 and 1 <= L <= 4 and n // m >= 2 * L
    # the reported expected recovery is the hypergeometric CDF (to the
    # rounding of log-gamma differences of numbers near N log N); for K << N
    # it is close to the binomial one
    assert abs(rec - hyper_recovery(n, k, m, L)) < 1e-7
    assert abs(rec - binom_recovery(n, k, m, L)) < 1e-3
    assert rec >= t
    # at the chosen L, half the M would miss the target (cost grows with M)
    if m // 2 >= 2 and n // (m // 2) <= (1 << 22):
        assert hyper_recovery(n, k, m // 2, L) < t
    assert us > 0


def test_expected_recovery_matches_the_paper_style_choice(sft):
    # N = 2^20, K = 1000 at the default target: M = 4096 (about 4K), L = 4
    m, L, rec, _ = sft.autotune(1 << 20, 1000)
    assert (m, L) == (4096, 4)
    # Poisson check of the same figure: P(X <= 3), X ~ Poisson(K d / N)
    lam = 999 * 255 / ((1 << 20) - 1)
    assert abs(rec - stats.poisson.cdf(3, lam)) < 1e-5


def test_higher_target_never_lowers_expected_recovery(sft):
    for n, k in CASES:
        recs = [sft.autotune(n, k, target=t)[2] for t in (0.9, 0.99, 0.999, 0.9999)]
        assert all(a <= b + 1e-15 for a, b in zip(recs, recs[1:])), (n, k, recs)


def test_uneven_batch_choices(sft):
    # the batched uneven workload: every signal gets an admissible pair
    ns, ks = sftgen.uneven_batch_params(4096)
    ms = []
    for n, k in zip(ns.tolist(), ks.tolist()):
        m, L, rec, _ = sft.autotune(n, k)
        assert rec >= 0.999 and n // m >= 2 * L
        ms.append(m)
    assert len(set(ms)) > 5   # the choices really vary over the batch


@pytest.mark.parametrize("args", [(1000, 10), (1 << 14, 0), (1 << 14, (1 << 14) + 1), (1, 1)])
def test_invalid_arguments(sft, args):
    with pytest.raises(sft.SftError):
        sft.autotune(*args)
    with pytest.raises(sft.SftError):
        sft.autotune(1 << 14, 10, target=1.0)
