"""Plain FP64 oracle of iterative sFFT-DT for exactly K-sparse signals (Alg. 1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The method (Sec. II-D, II-E, Alg. 1): iteration l = 0 .. a_m - 1 works on the
grid of M_l = N / d_l bins with d_l = 2^l d_0.  It computes the FFTs of the
two new shifts 2l and 2l + 1 at d_l, removes the contributions of the
frequencies solved so far (SubFreq), and decodes every bin that is still
unsolved or whose new syndromes are non-zero at order a = l + 1 from its
2l + 2 syndromes (SynDec).  A bin whose solution fails the grid check is kept
in T, which is taken modulo the next, coarser grid.

Readings where the algorithm as printed leaves something open (each one is
repeated where it is used):
  * earlier syndromes on the current grid: SynDec at iteration l needs the
    syndromes of shifts 0 .. 2l - 1 on the grid of d_l, which Alg. 1 computed
    on finer grids.  They are folded, m_{2d,j}[k] = m_{d,j}[k] + m_{d,j}[k + M/2]
    (exact: a residue class mod M/2 is the union of two classes mod M, Eq. (3));
  * SubFreq acts on all 2l + 2 syndromes of the current grid with the whole
    set S (the printed function names the two new ones only; the folded
    older ones also still hold the frequencies solved after they were taken);
  * activity (Alg. 1 "|x_{d,2l}[k]| > 0 or |x_{d,2l+1}[k]| > 0"): the residual
    energy of the two new syndromes exceeds tau_zero^2 times their mean energy
    before SubFreq;
  * T holds the bins whose SynDec failed in the latest iteration, reduced mod
    the next grid; a bin whose later decode succeeded leaves it (its residual
    is zero, so decoding it again could only produce a spurious solution);
  * grid check "s_j mod d = k" read as s_j mod M_l = k (reading R4 of the
    non-iterative oracle), plus the exact-mode judge ||m - V p||^2 <=
    tau_res^2 E (readings R8, R14 with nu = 0);
  * at l = 0 the value is p_0 = m_0 (Alg. 1 SynDec, the a = 1 case); at
    l >= 1 the values solve Step (iii) in least squares over the 2l + 2
    syndromes;
  * line 32 accumulates, x_hat[s_j] += p_j: SubFreq has already removed what
    S holds, so a later solution at a location already in S is a correction
    of its value (the printed assignment only agrees when s_j is new).  A
    location whose accumulated value cancels, |sum| < tau_amp max |part|,
    leaves the output (an earlier solution that a later iteration undid).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .roots import poly_roots
from .sfft import (
    TWO_PI,
    Result,
    Taus,
    _sorted,
    amplitudes,
    default_taus,
    locator,
    roots_to_grid,
    syndromes,
    vandermonde,
)


def fold(row, m: int) -> np.ndarray:
    """Syndromes of one shift on the grid of M bins from those on a finer grid
    of a multiple of M bins: bin k collects the finer bins k + i M (Eq. (3):
    the bin sums x_hat over its residue class mod M)."""
    row = np.asarray(row, np.complex128)
    if row.size % m:
        raise ValueError("the finer grid must be a multiple of M")
    return row.reshape(-1, m).sum(axis=0)


def sub_freq(rows, solved: dict, n: int, m: int) -> np.ndarray:
    """Alg. 1 SubFreq on all rows (shifts j = 0 .. len(rows) - 1) of the grid
    of M bins: m_j[s mod M] -= x_hat[s] e^{i 2 pi s j / N} for every solved s."""
    rows = np.array(rows, np.complex128)
    j = np.arange(rows.shape[0], dtype=np.int64)
    for s, p in solved.items():
        rows[:, s % m] -= p * np.exp(1j * TWO_PI * ((j * s) % n) / n)
    return rows


def syn_dec(mk, l: int, k: int, n: int, m: int, taus: Taus):
    """Alg. 1 SynDec at iteration l: order a = l + 1 from the 2l + 2 syndromes
    of bin k on the grid of M bins.  l = 0: z_0 = m_1 / m_0, p_0 = m_0.
    l >= 1: Steps (i)-(iii) of Sec. II-B at order a.  Then s_j = N arg(z_j) /
    2 pi, the grid check and the judge.  Returns (s, p) or None."""
    mk = np.asarray(mk, np.complex128)
    a = l + 1
    if l == 0:
        if mk[0] == 0:
            return None
        z = np.array([mk[1] / mk[0]])
        s = roots_to_grid(z, k, n, m, taus)
        if s is None:
            return None
        p = np.array([mk[0]])
        r = mk[:2] - vandermonde(s, n, 2) @ p
        r2 = float(np.real(np.vdot(r, r)))
    else:
        c = locator(mk, a)
        if c is None:
            return None
        z = poly_roots(c)
        s = roots_to_grid(z, k, n, m, taus)
        if s is None:
            return None
        p, r2 = amplitudes(mk, s, n)
    e = float(np.sum(np.abs(mk) ** 2))
    if not r2 <= taus.tau_res ** 2 * e:
        return None
    return s, p


@dataclasses.dataclass
class Level:
    d: int
    m: int
    active: int
    solved: list        # locations solved at this iteration
    failed: list        # bins (of this grid) whose SynDec failed


def sfft_iterative(x, n: int, m0: int, a_m: int = 4, taus: Taus | None = None,
                   fft_dtype=np.complex128):
    """Iterative sFFT-DT (Alg. 1) with d_0 = N / M_0 and a_m iterations.

    Returns (Result, levels): the recovered (location, value) pairs sorted by
    location (accumulated values; cancelled ones left out), with active_bins = bins decoded over all iterations and
    flagged_bins = bins whose decode failed in the last iteration; levels
    lists per iteration its grid, active bins, solved locations and failed
    bins.  fft_dtype as in sfft.syndromes."""
    if taus is None:
        taus = default_taus(np.asarray(x).dtype == np.complex128)
    if n % m0 or m0 < 1 or (m0 >> (a_m - 1)) < 1:
        raise ValueError("need M_0 dividing N and M_0 >= 2^(a_m - 1)")
    d = n // m0
    solved: dict = {}       # S and the solved values of x_hat
    largest: dict = {}      # per location, the largest |p| solved there
    t_bins: set = set()     # T
    base = {}               # shift j -> its FFT row (grid of the iteration that took it)
    levels = []
    res = Result(np.empty(0, np.int64), np.empty(0, np.complex128))
    for l in range(a_m):
        m = n // d
        # the two new FFTs at the current d, times d
        new = syndromes(x, n, m, [2 * l, 2 * l + 1], fft_dtype)
        base[2 * l], base[2 * l + 1] = new[0], new[1]
        e_ref = float(np.mean(np.abs(new[0]) ** 2 + np.abs(new[1]) ** 2))
        # every shift so far on the current grid, then SubFreq with all of S
        rows = sub_freq([fold(base[j], m) for j in range(2 * l + 2)], solved, n, m)
        lev = Level(d, m, 0, [], [])
        for k in range(m):
            e_new = abs(rows[2 * l, k]) ** 2 + abs(rows[2 * l + 1, k]) ** 2
            if not (k in t_bins or e_new > taus.tau_zero ** 2 * e_ref):
                continue
            lev.active += 1
            out = syn_dec(rows[:, k], l, k, n, m, taus)
            if out is None:
                lev.failed.append(k)
                continue
            for s_j, p_j in zip(*out):
                s_j = int(s_j)
                solved[s_j] = solved.get(s_j, 0.0) + complex(p_j)
                largest[s_j] = max(largest.get(s_j, 0.0), abs(p_j))
                lev.solved.append(s_j)
        levels.append(lev)
        res.active_bins += lev.active
        # double d; T modulo the new grid
        d *= 2
        if l + 1 < a_m:
            t_bins = {k % (n // d) for k in lev.failed}
    res.flagged_bins = len(levels[-1].failed)
    locs = [s for s in solved if abs(solved[s]) >= taus.tau_amp * largest[s]]
    vals = [solved[s] for s in locs]
    res.locs, res.vals = _sorted(locs, vals)
    return res, levels


def fft_points(m0: int, a_m: int) -> list:
    """Lengths of the FFTs Alg. 1 takes: two per iteration, M_0 / 2^l."""
    return [m0 >> l for l in range(a_m) for _ in range(2)]
