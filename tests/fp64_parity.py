"""Parity of complex64 runs (FP32 FFTs on the device) with the FP64 oracle.

The decisions of the method (rank test, locator, roots on the grid, residual
judge) are taken on the syndromes.  Complex64 input runs the FFTs in FP32, so
the device's syndromes carry rounding of about u sqrt(log2 M) of a line's rms
(u = 2^-24).  Almost every bin's decision is far from any threshold and the
device decides it as the FP64 oracle does; a bin whose FP64 decision changes
under perturbations of that size ("fragile": an ill-conditioned cluster of
aliased tones, e.g. two tones a few slots apart at large d, where any nearby
pair fits the 2L syndromes within the judge's tolerance) may come out either
way, including, rarely, a wrong pair that the perturbed FP64 oracle also
accepts.  The complex64 input itself is rounded (about 1e-6 of a tone per
bin), so a cluster whose Hankel matrix has sigma_a / sigma_1 below the
judge's tolerance tau_res (1e-4) cannot be resolved by the 2L syndromes at
that precision: nearby supports fit them within the tolerance, and the two
sides' arithmetic may settle such a bin differently.  These helpers compare
bin by bin with the FP64 oracle and require every differing bin to be
fragile or ill-conditioned in that sense, and such bins to stay a handful.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle import iterative as oit


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def per_bin(locs, m):
    out = {}
    for s in np.asarray(locs).tolist():
        out.setdefault(s % m, set()).add(s)
    return out


def oracle_decision(mk, b, n, m, L, taus):
    """The oracle's decision on one bin (rank test, canonical orders, judge):
    the decoded locations, or None when the bin is flagged."""
    a0 = oracle.rank_order(oracle.hankel_singular_values(mk, L), taus.tau_rank)
    out = oracle.decode_bin(mk, b, n, m, L, a0, float(np.sum(np.abs(mk) ** 2)), 0.0, taus)
    return None if out is None else frozenset(out[0].tolist())


def fp32_fragile(msyn64, b, n, m, L, taus, trials=16, seed=0):
    """True when the FP64 oracle's decision on bin b changes under complex
    Gaussian perturbations of the syndromes with rms u log2(M) times each
    line's rms (u = 2^-24): the first-order size of a single-precision FFT's
    rounding, so that the bin's decision is not fixed by the input at that
    precision."""
    base = oracle_decision(msyn64[:, b], b, n, m, L, taus)
    g = np.random.default_rng(seed + b)
    scale = np.sqrt(np.mean(np.abs(msyn64) ** 2, axis=1)) * 2.0 ** -24 * np.log2(m)
    for _ in range(trials):
        d = (g.standard_normal(len(scale)) + 1j * g.standard_normal(len(scale))) * scale / np.sqrt(2.0)
        if oracle_decision(msyn64[:, b] + d, b, n, m, L, taus) != base:
            return True
    return False


TAU_RES_C64 = 1e-4


def cluster_conditioning(locs, vals, n):
    """sigma_a / sigma_1 of the a x a Hankel matrix of Eq. (5) (the locator's
    system) built from the syndromes m_j = sum_i p_i e^{2 pi i s_i j / N},
    j < 2a, of a cluster of a tones (locations s_i, values p_i)."""
    locs = np.asarray(locs, np.int64)
    vals = np.asarray(vals, np.complex128)
    a = len(locs)
    if a < 2:
        return 1.0
    j = np.arange(2 * a)
    msyn = (vals[None, :] * np.exp(2j * np.pi * np.outer(j, locs % n) / n)).sum(axis=1)
    sv = np.linalg.svd(oracle.hankel(msyn, a), compute_uv=False)
    return float(sv[-1] / sv[0])


def ill_conditioned(locs, vals, n, tau=TAU_RES_C64):
    """True when the cluster's locator system has sigma_a / sigma_1 below the
    judge's tolerance (see the module doc)."""
    return cluster_conditioning(locs, vals, n) < tau


def exact_vs_fp64(loc, val, stats, x, n, m, L, max_diff, truth=None, value_tol=1e-5, say=print):
    """Exact mode, complex64 input: the device's output (loc, val, stats)
    against the FP64 oracle (FP64 FFTs, the complex64 thresholds), bin by bin.

    Every bin where the two differ must be FP32-fragile, or (truth = (true
    locations, true values) given) hold a cluster of at most L tones that is
    ill-conditioned at the judge's tolerance, and there are at
    most max_diff of them; the flagged-bin count differs only by those bins;
    values at the common locations within value_tol relative L2.  Returns the
    oracle's result and the differing bins."""
    ref = oracle.sfft_exact(x, n, m, L)
    gb, rb = per_bin(loc, m), per_bin(ref.locs, m)
    diff = sorted(b for b in set(gb) | set(rb) if gb.get(b) != rb.get(b))
    if diff:
        say(f"  {len(diff)} bin(s) differ from the FP64 oracle: {diff[:8]}")
    assert len(diff) <= max_diff, diff
    if diff:
        taus = oracle.default_taus(False)
        msyn64 = oracle.syndromes(x, n, m, range(2 * L))
        for b in diff:
            if truth is not None:
                sel = np.asarray(truth[0]) % m == b
                if 2 <= sel.sum() <= L and ill_conditioned(np.asarray(truth[0])[sel], np.asarray(truth[1])[sel], n):
                    continue
            assert fp32_fragile(msyn64, b, n, m, L, taus), b
    if stats is not None:
        lost = sum(1 for b in diff if b in rb and b not in gb)
        gained = sum(1 for b in diff if b in gb and b not in rb)
        assert stats["flagged_bins"] == ref.flagged_bins + lost - gained
        assert stats["active_bins"] == ref.active_bins
    common, ia, ib = np.intersect1d(loc, ref.locs, return_indices=True)
    if len(common):
        assert rel_l2(val[ia], ref.vals[ib]) <= value_tol
    return ref, diff


def iterative_flips(x, n, m0, L, trials=12, seed=0):
    """Locations whose presence in the FP64 iterative oracle's output changes
    when every syndrome line is perturbed by complex Gaussian noise of rms
    2 u sqrt(log2 M) times the line's rms (twice the first-order size of a
    single-precision FFT's rounding).  Decisions at iterations >= 1 work on
    folded syndromes minus the values solved before, so an ill-conditioned
    cluster there may go either way."""
    base, _ = oit.sfft_iterative(x, n, m0, L)
    ref = set(base.locs.tolist())
    g = np.random.default_rng(seed)
    orig = oit.syndromes

    def perturbed(xx, nn, mm, shifts, fft_dtype=np.complex128):
        out = orig(xx, nn, mm, shifts, fft_dtype)
        scale = np.sqrt(np.mean(np.abs(out) ** 2, axis=1, keepdims=True)) * 2.0 ** -23 * np.sqrt(np.log2(mm))
        return out + (g.standard_normal(out.shape) + 1j * g.standard_normal(out.shape)) * scale / np.sqrt(2.0)

    flips = set()
    try:
        oit.syndromes = perturbed
        for _ in range(trials):
            r, _ = oit.sfft_iterative(x, n, m0, L)
            flips |= ref ^ set(r.locs.tolist())
    finally:
        oit.syndromes = orig
    return base, flips


def iterative_ill_conditioned(levels, truth, c, n, m0, L, tau=TAU_RES_C64):
    """True when some decision of residue class c (mod M_{L-1}) has to resolve
    a cluster ill-conditioned at the judge's tolerance: at iteration l, a bin
    of the grid M_l in the class holding 2..l+1 true tones that the oracle had
    not solved at an earlier iteration (the cluster SubFreq leaves to SynDec
    of order l + 1)."""
    locs, vals = np.asarray(truth[0]), np.asarray(truth[1])
    ml = m0 >> (L - 1)
    sel = locs % ml == c
    locs, vals = locs[sel], vals[sel]
    done = set()
    for l in range(L):
        mgrid = m0 >> l
        left = np.array([v not in done for v in locs.tolist()], bool)
        for b in np.unique(locs[left] % mgrid):
            inb = left & (locs % mgrid == b)
            if 2 <= inb.sum() <= l + 1 and cluster_conditioning(locs[inb], vals[inb], n) < tau:
                return True
        done |= set(levels[l].solved)
    return False


def iterative_vs_fp64(loc, x, n, m0, L, max_classes=2, truth=None, say=print):
    """Iterative mode, complex64 input: the device's locations against the FP64
    iterative oracle.  Alg. 1 decides each residue class mod M_{L-1} on its
    own (folds and SubFreq never mix classes), so where an FP32-fragile
    location sits in a class, every decision of that class may differ.

    A class may differ from the oracle's only when it holds a location whose
    presence in the oracle's output flips under FP32-size perturbations of the
    syndromes (iterative_flips), or (truth = (true locations, true values)
    given) when one of its decisions faces a cluster ill-conditioned at the
    judge's tolerance (iterative_ill_conditioned).  At most max_classes
    classes differ.  Returns the oracle's result and the number of differing
    classes."""
    ref, levels = oit.sfft_iterative(x, n, m0, L)
    loc = np.asarray(loc)
    diff = set(loc.tolist()) ^ set(ref.locs.tolist())
    if not diff:
        return ref, 0
    ml = m0 >> (L - 1)
    classes = {s % ml for s in diff}
    say(f"  {len(diff)} locations in {len(classes)} classes differ from the FP64 oracle")
    assert len(classes) <= max_classes
    unexplained = set(classes)
    if truth is not None:
        for c in classes:
            if iterative_ill_conditioned(levels, truth, c, n, m0, L):
                say(f"  class {c}: a decision faces a cluster ill-conditioned at the judge's tolerance")
                unexplained.discard(c)
    if unexplained:
        _, flips = iterative_flips(x, n, m0, L)
        unexplained -= {s % ml for s in flips}
    assert not unexplained, sorted(unexplained)
    return ref, len(classes)
