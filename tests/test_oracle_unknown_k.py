"""Pins of the unknown-K strategy of Sec. II-G (CPU).

The bottom-up loop stops at the first M = N/d whose run flags no bin.  In
exact arithmetic a bin is flagged exactly when it holds more than L
frequencies, so the chosen M is the smallest power of two at which no
residue class mod M holds more than L support locations: computed here from
the support alone.  The output at that M is x_hat.  The work of the rungs
tried sums to less than twice that of the last one (the paper's estimate that
the strategy costs double the known-K run).
"""
import numpy as np
import pytest

import oracle
import sftgen


def smallest_m(locs, n, L, m_min=1):
    m = m_min
    while m < n:
        counts = np.bincount(np.asarray(locs) % m, minlength=m)
        if counts.max() <= L:
            return m
        m *= 2
    return n


@pytest.mark.parametrize("n,k,L,seed", [(1 << 12, 3, 4, 1), (1 << 12, 40, 4, 2), (1 << 14, 100, 4, 3),
                                        (1 << 14, 100, 2, 4), (1 << 10, 200, 4, 5), (1 << 16, 64, 1, 6)])
def test_unknown_k_stops_at_the_first_collision_free_grid(n, k, L, seed):
    s = sftgen.make_signal(n, k, seed, amp="gauss", dtype=np.complex128)
    res, m = oracle.sfft_unknown_k(s.x, n, L)
    assert m == smallest_m(s.locs, n, L)
    assert res.flagged_bins == 0
    assert res.locs.tolist() == s.locs.tolist()
    assert np.max(np.abs(res.vals - s.vals)) < 1e-9


def test_unknown_k_few_tones_solve_at_d_equal_n():
    """K <= L: a single bin at d = N holds every tone and decodes them."""
    n = 1 << 12
    s = sftgen.make_signal(n, 4, 9, amp="unit", dtype=np.complex128)
    res, m = oracle.sfft_unknown_k(s.x, n, 4)
    assert m == 1 and res.locs.tolist() == s.locs.tolist()


def test_unknown_k_stops_at_m_max():
    n = 1 << 12
    s = sftgen.make_signal(n, 300, 10, amp="gauss", dtype=np.complex128)
    res, m = oracle.sfft_unknown_k(s.x, n, 4, m_max=16)
    assert m == 16 and res.flagged_bins > 0


def test_unknown_k_cost_is_below_twice_the_last_run():
    n = 1 << 14
    s = sftgen.make_signal(n, 100, 3, amp="gauss", dtype=np.complex128)
    _, m = oracle.sfft_unknown_k(s.x, n, 4)
    tried = [1 << j for j in range(int(np.log2(m)) + 1)]
    # 2L FFTs of M points per rung: sum over rungs of M log M < 2 M log M of the last
    cost = sum(8 * mm * max(1, np.log2(mm)) for mm in tried)
    assert cost < 2 * 8 * m * np.log2(m)
