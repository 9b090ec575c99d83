"""Pins of the iterative oracle (Alg. 1) against things other than itself (CPU).

* fold: syndromes folded to a coarser grid equal the alias sums of Eq. (3)
  on that grid, written out by brute force;
* SubFreq: removing solved frequencies leaves exactly the alias sums of the
  rest (brute force), and zero when everything is removed;
* the Fig. 1 toy: which frequency each iteration solves, and the FFT lengths;
* a support-only simulation of Alg. 1 (group the unsolved locations by
  s mod M_l; a group of exactly l + 1 is solved, any other fails) predicts
  the recovered support exactly on random supports with many collisions;
* with a_m = 1 the support equals that of the non-iterative oracle at L = 1;
* the paper's cost statement for a_m = 4 (Sec. II-F).
"""
import json
import math
import os
from collections import defaultdict

import numpy as np
import pytest

import sftgen
from oracle import sfft as osf
from oracle import iterative as oit

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def exact_signal(n, locs, vals):
    xh = np.zeros(n, np.complex128)
    xh[np.asarray(locs, np.int64)] = vals
    return np.fft.ifft(xh)


def alias_sum(locs, vals, n, m, l):
    """Eq. (3) written out: sum over the support of x_hat[s] e^{i 2 pi s l / N} in bin s mod M."""
    out = np.zeros(m, np.complex128)
    for s, v in zip(locs, vals):
        out[int(s) % m] += v * np.exp(2j * np.pi * int(s) * l / n)
    return out


def predicted_support(locs, m0, a_m):
    """Support-only simulation of Alg. 1: at iteration l the unsolved locations
    are grouped by s mod M_l; a group of exactly l + 1 locations is solved."""
    unsolved, solved, per_level = set(int(s) for s in locs), set(), []
    for l in range(a_m):
        m = m0 >> l
        groups = defaultdict(list)
        for s in unsolved:
            groups[s % m].append(s)
        now = set()
        for g in groups.values():
            if len(g) == l + 1:
                now |= set(g)
        per_level.append(now)
        solved |= now
        unsolved -= now
    return solved, per_level


# ------------------------------------------------------------------ fold

@pytest.mark.parametrize("n,m,c", [(256, 64, 1), (256, 64, 3), (1024, 16, 4), (64, 2, 1)])
def test_fold_equals_alias_sum_on_coarser_grid(n, m, c):
    """Folding c times (d -> 2^c d) gives the syndromes of the coarser grid,
    checked against the brute-force alias sum of Eq. (3) for several shifts."""
    g = np.random.default_rng(n + m + c)
    locs = g.choice(n, 12, replace=False)
    vals = g.standard_normal(12) + 1j * g.standard_normal(12)
    x = exact_signal(n, locs, vals)
    for l in (0, 1, 5):
        fine = osf.syndromes(x, n, m, [l])[0]
        coarse = oit.fold(fine, m >> c)
        ref = alias_sum(locs, vals, n, m >> c, l)
        assert np.max(np.abs(coarse - ref)) < 1e-11


def test_fold_of_a_dense_signal_matches_direct_fft():
    """For a dense (non-sparse) x the fold still equals d' * FFT at d' = 2d: the
    identity is the decimation property of the DFT, not a sparsity effect."""
    n, m = 512, 64
    g = np.random.default_rng(3)
    x = g.standard_normal(n) + 1j * g.standard_normal(n)
    for l in (0, 3):
        fine = osf.syndromes(x, n, m, [l])[0]
        d2 = 2 * (n // m)
        direct = d2 * np.array([sum(x[(d2 * kp + l) % n] * np.exp(-2j * np.pi * k * kp / (m // 2))
                                    for kp in range(m // 2)) for k in range(m // 2)])
        assert np.max(np.abs(oit.fold(fine, m // 2) - direct)) < 1e-9


# --------------------------------------------------------------- SubFreq

def test_sub_freq_leaves_the_alias_sum_of_the_rest():
    n, m = 1024, 32
    g = np.random.default_rng(5)
    locs = g.choice(n, 40, replace=False)
    vals = g.standard_normal(40) + 1j * g.standard_normal(40)
    x = exact_signal(n, locs, vals)
    rows = osf.syndromes(x, n, m, range(6))
    solved = {int(s): complex(v) for s, v in zip(locs[:25], vals[:25])}
    res = oit.sub_freq(rows, solved, n, m)
    for l in range(6):
        ref = alias_sum(locs[25:], vals[25:], n, m, l)
        assert np.max(np.abs(res[l] - ref)) < 1e-10
    everything = {int(s): complex(v) for s, v in zip(locs, vals)}
    assert np.max(np.abs(oit.sub_freq(rows, everything, n, m))) < 1e-10


# ---------------------------------------------------------------- Fig. 1

def test_fig1_iterative_toy():
    """Fig. 1 (c)-(d): the lone frequency first, the collision at the next d."""
    gold = json.load(open(os.path.join(GOLDEN, "fig1_iterative.json")))
    n, d0, a_m = gold["n"], gold["d0"], gold["a_m"]
    g = np.random.default_rng(11)
    vals = np.exp(2j * np.pi * g.random(len(gold["support"])))
    x = exact_signal(n, gold["support"], vals)
    res, levels = oit.sfft_iterative(x, n, n // d0, a_m)
    assert [sorted(lv.solved) for lv in levels] == gold["solved_per_iteration"]
    assert res.locs.tolist() == gold["support"]
    assert np.max(np.abs(res.vals - vals)) < 1e-12
    assert oit.fft_points(n // d0, a_m) == gold["fft_lengths"]
    assert [lv.d for lv in levels] == [d0, 2 * d0]


# ---------------------------------------------- support-level prediction

@pytest.mark.parametrize("n,m0,k,seed", [(4096, 64, 40, 1), (4096, 64, 100, 2), (1 << 14, 128, 200, 3),
                                         (1 << 14, 256, 64, 4), (2048, 16, 30, 5)])
def test_recovered_support_matches_simulation(n, m0, k, seed):
    """Random supports dense enough for collisions of every order: the oracle
    solves exactly the groups the simulation predicts, at the predicted
    iteration, with the true values."""
    g = np.random.default_rng(seed)
    locs = np.sort(g.choice(n, k, replace=False))
    vals = g.standard_normal(k) + 1j * g.standard_normal(k)
    x = exact_signal(n, locs, vals)
    res, levels = oit.sfft_iterative(x, n, m0, 4)
    want, per_level = predicted_support(locs, m0, 4)
    assert sorted(res.locs.tolist()) == sorted(want)
    for lv, exp in zip(levels, per_level):
        assert set(lv.solved) == exp
    truth = dict(zip(locs.tolist(), vals))
    got = np.array([truth[s] for s in res.locs.tolist()])
    assert np.max(np.abs(res.vals - got)) < 1e-9
    # unsolved locations are exactly those in the last iteration's failed bins
    m_last = m0 >> 3
    missing = set(locs.tolist()) - want
    assert {s % m_last for s in missing} == set(levels[-1].failed)


def test_simulation_cases_exercise_every_iteration():
    """The cases above are not trivial: across them every iteration solves something."""
    seen = [0, 0, 0, 0]
    for n, m0, k, seed in [(4096, 64, 40, 1), (4096, 64, 100, 2), (1 << 14, 128, 200, 3)]:
        g = np.random.default_rng(seed)
        locs = np.sort(g.choice(n, k, replace=False))
        _, per_level = predicted_support(locs, m0, 4)
        for l in range(4):
            seen[l] += len(per_level[l])
    assert all(v > 0 for v in seen)


def test_paper_setting_recovers_everything():
    """d = N / (4K) (Sec. II-E initialisation): a typical support is recovered in full."""
    n, k = 1 << 14, 64
    s = sftgen.make_signal(n, k, 21, dtype=np.complex128)
    res, levels = oit.sfft_iterative(s.x, n, 4 * k, 4)
    assert res.locs.tolist() == sorted(s.locs.tolist())
    assert res.flagged_bins == 0


def test_am1_support_equals_non_iterative_l1():
    """a_m = 1 is one iteration of order 1: the non-iterative oracle at L = 1
    (a different code path: rank test, canonical orders, least-squares values)
    finds the same support."""
    n, m, k = 4096, 128, 90
    s = sftgen.make_signal(n, k, 8, dtype=np.complex128)
    it, _ = oit.sfft_iterative(s.x, n, m, 1)
    ni = osf.sfft_exact(s.x, n, m, 1)
    assert it.locs.tolist() == ni.locs.tolist()
    assert np.max(np.abs(it.vals - ni.vals)) < 1e-9


def test_cost_bound_of_the_iterative_ffts():
    """Sec. II-F: the FFTs of a_m = 4 iterations cost at most (2 + 1 + 1/2 + 1/4)
    (N/d) log(N/d), against 2 a_m (N/d) log(N/d) for the non-iterative method."""
    m0 = 4096
    pts = oit.fft_points(m0, 4)
    cost = sum(p * math.log2(p) for p in pts)
    assert cost <= 3.75 * m0 * math.log2(m0)
    assert cost < 8 * m0 * math.log2(m0) / 2


def test_rejects_too_many_iterations_for_the_grid():
    with pytest.raises(ValueError):
        oit.sfft_iterative(np.zeros(64, np.complex128), 64, 4, 4)


def test_t_keeps_a_bin_whose_new_syndromes_vanish():
    """Alg. 1 line 9: a bin in T is decoded even when both new syndromes are
    zero.  Three frequencies share a bin down to M_2; their values span the
    null space of the shifts-4,5 rows, so m_4 = m_5 = 0 there.  Only T brings
    the bin to the order-3 decode of iteration 2; without it the three would
    meet order 4 at iteration 3 and stay unsolved."""
    n, m0, k = 1024, 64, 5
    locs = np.array([k + 1 * m0, k + 6 * m0, k + 11 * m0], np.int64)   # distinct z^4
    z = np.exp(2j * np.pi * locs / n)
    a = np.array([z ** 4, z ** 5])
    null = np.linalg.svd(a)[2][-1].conj()          # a @ null = 0
    assert np.max(np.abs(a @ null)) < 1e-14
    others = np.array([1, 2 + m0, 3 + 5 * m0], np.int64)
    all_locs = np.concatenate([locs, others])
    all_vals = np.concatenate([null, np.array([0.9, -0.4j, 0.3 + 0.3j])])
    x = exact_signal(n, all_locs, all_vals)
    rows = osf.syndromes(x, n, m0 >> 2, [4, 5])
    assert np.max(np.abs(rows[:, k % (m0 >> 2)])) < 1e-12
    res, levels = oit.sfft_iterative(x, n, m0, 4)
    assert sorted(levels[2].solved) == sorted(locs.tolist())
    assert res.locs.tolist() == sorted(all_locs.tolist())


def midpoint_pair(n, m0, k, t1, t2):
    """Two tones in bin k (slots t1, t2 with t1 + t2 even) whose values make
    the a = 1 test of iteration 0 exact for a third location: with p_1 = 1 and
    p_2 = e^{i (a_1 - a_2) / 2} (a_j the angles of the de-rotated roots),
    m_1 / m_0 is the root of the midpoint slot (t1 + t2) / 2."""
    d = n // m0
    a1, a2 = 2 * np.pi * t1 / d, 2 * np.pi * t2 / d
    locs = np.array([k + t1 * m0, k + t2 * m0], np.int64)
    vals = np.array([1.0, np.exp(1j * (a1 - a2) / 2)])
    return locs, vals, k + ((t1 + t2) // 2) * m0


def test_later_solution_corrects_an_earlier_one():
    """Line 32 read as x_hat[s] += p: iteration 0 accepts the midpoint of an
    equal-magnitude pair as one tone; iteration 2 solves the pair together with
    the negative of that tone, and the location cancels.  (Assignment would
    leave the midpoint in the output with the value -m_0.)"""
    n, m0, k = 1024, 64, 9
    locs, vals, mid = midpoint_pair(n, m0, k, 3, 11)
    others = np.array([2, 5 + 3 * m0, 40 + 7 * m0], np.int64)
    all_locs = np.concatenate([locs, others])
    all_vals = np.concatenate([vals, np.array([0.8, 0.5j, -0.7])])
    x = exact_signal(n, all_locs, all_vals)
    res, levels = oit.sfft_iterative(x, n, m0, 4)
    assert mid in levels[0].solved                       # the wrong a = 1 solution
    assert {mid, *locs.tolist()} <= set(levels[2].solved)  # corrected at a = 3
    assert res.locs.tolist() == sorted(all_locs.tolist())
    truth = dict(zip(all_locs.tolist(), all_vals))
    assert max(abs(v - truth[s]) for s, v in zip(res.locs.tolist(), res.vals)) < 1e-10
