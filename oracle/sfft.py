"""Plain FP64 oracle of non-iterative sFFT-DT (Hsieh, Lu, Pei; arXiv 1407.8315).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Notation follows the paper: N signal length, d downsampling factor, M = N/d
downsampled length, L = a_m the maximum number of collisions per bin, m_l the
syndromes of a bin, c the locator coefficients, z_j the roots, p_j the values,
s_j the recovered locations, n_j the random shifts of the CS step.

DFT convention (the paper contradicts itself; this is the only reading that
agrees with Eq. (1), Alg. 1's "FFT x d" and the a = 1 solver): forward DFT
unnormalised, x = IDFT(x_hat).  Then the syndrome of bin k at shift l is
    m_l[k] = d * DFT_M(x[d k' + l])[k] = sum_t x_hat[k + t M] e^{i 2 pi (k + t M) l / N}
(Sec. II-A, Eq. (2)-(3)), i.e. Eq. (3) with p_j = x_hat[s_j], z_j = e^{i 2 pi s_j / N}.

Readings of points where the paper is silent (each repeated in the function
that uses it):
  * activity: a bin is active when E_k = sum_l |m_l|^2 > tau_zero^2 * mean_k E_k;
  * order estimate (exact mode): numerical rank of the L x L Hankel matrix of
    m_0..m_{2L-2}; decoding then tries a0, a0+1..L, a0-1..1;
  * grid check: s_j = N arg(z_j) / 2 pi must sit within delta_grid * M of a
    point k + t M (the check "s_j mod (N/d) = k"), with ||z_j| - 1| <= delta_mag;
  * Step (iii) is solved in least squares over all 2L syndromes;
  * judge: accept when ||m - V p||^2 <= tau_res^2 E_k + c_res (2L - a) nu;
  * noise floor (general mode): nu = median_k E_k / (2L - 1/3);
  * CS step (general mode) only on the bins the decoder flags; pruning keeps
    the min(2 a, R, d) candidates with the smallest |P~(z)|; output keeps the K
    largest |values|.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .roots import poly_roots

TWO_PI = 2.0 * np.pi


@dataclasses.dataclass
class Taus:
    tau_zero: float
    tau_rank: float
    tau_res: float
    tau_amp: float
    c_res: float = 3.0
    delta_grid: float = 0.1
    delta_mag: float = 0.05


def default_taus(complex128_input: bool) -> Taus:
    """Thresholds for complex64 input (FP32 syndromes on the fast path) or complex128."""
    if complex128_input:
        return Taus(tau_zero=1e-9, tau_rank=1e-10, tau_res=1e-9, tau_amp=1e-9)
    return Taus(tau_zero=1e-4, tau_rank=1e-5, tau_res=1e-4, tau_amp=1e-4)


# ---------------------------------------------------------------- steps 1-2


def syndromes(x, n: int, m: int, shifts, fft_dtype=np.complex128) -> np.ndarray:
    """m_l[k] = d * FFT(x_{d,l})[k] with x_{d,l}[k'] = x[(d k' + l) mod N].

    Sec. II-A (x_{d,l}[k] = x[dk + l]) and Alg. 1, the two FFT lines scaled by
    d; Alg. 2, Part 1, for the random shifts n_j.  Indices wrap mod N, which
    only matters when d < 2L.  Returns an array [len(shifts), M] in FP64.

    fft_dtype=np.complex64 returns the transforms rounded to single
    precision (numpy evaluates them more accurately than single-precision
    arithmetic would), i.e. the syndromes a correctly rounded single-precision
    FFT would store, so that decisions which depend on that resolution (e.g.
    clusters whose smallest Hankel singular value is below it) are taken at
    the same resolution.  A single-precision FFT adds its own rounding error,
    about u sqrt(log2 M) of the line's rms, on top of this.
    """
    x = np.asarray(x).astype(fft_dtype)
    if n % m:
        raise ValueError("M must divide N")
    d = n // m
    kp = np.arange(m, dtype=np.int64)
    out = np.empty((len(shifts), m), np.complex128)
    for i, l in enumerate(shifts):
        out[i] = (fft_dtype(d) * np.fft.fft(x[(d * kp + int(l)) % n])).astype(np.complex128)
    return out


def bin_energy(msyn: np.ndarray) -> np.ndarray:
    """E_k = sum_l |m_l[k]|^2 over the 2L consecutive-shift syndromes."""
    return np.sum(np.abs(msyn) ** 2, axis=0)


# ---------------------------------------------------------------- step 3


def hankel(mk, a: int) -> np.ndarray:
    """The a x a matrix M with M_{ij} = m_{i+j} (Sec. II-B, Eq. (5))."""
    return np.array([[mk[i + j] for j in range(a)] for i in range(a)], np.complex128)


def hankel_singular_values(mk, L: int) -> np.ndarray:
    """Singular values (descending) of the L x L Hankel matrix of m_0..m_{2L-2}.

    Used for the order estimate (exact mode) and the vote of Pruning Step 1
    (Sec. III-C): SVD of M, whose singular values equal those of its symmetric
    SVD.
    """
    return np.linalg.svd(hankel(mk, L), compute_uv=False)


def rank_order(sv: np.ndarray, tau_rank: float) -> int:
    """a0 = #{sigma_i > tau_rank * sigma_1}, at least 1."""
    if sv[0] <= 0 or not np.isfinite(sv[0]):
        return 1
    return max(1, int(np.sum(sv > tau_rank * sv[0])))


def try_orders(a0: int, L: int):
    """Canonical order of hypotheses: a0, a0+1 .. L, then a0-1 .. 1."""
    return list(range(a0, L + 1)) + list(range(a0 - 1, 0, -1))


def locator(mk, a: int):
    """Step (i): solve M c = -[m_a .. m_{2a-1}] (Eq. (5)).  None if M is singular."""
    h = hankel(mk, a)
    rhs = -np.asarray(mk[a:2 * a], np.complex128)
    try:
        c = np.linalg.solve(h, rhs)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(c)):
        return None
    return c


def roots_to_grid(z, k: int, n: int, m: int, taus: Taus):
    """Alg. 1: s_j = ln(z_j) N / (i 2 pi), accepted when s_j mod M = k.

    With the reading that s_j must be within delta_grid * M of a point
    k + t M of the candidate set S_k, that |z_j| is within delta_mag of 1, and
    that the recovered locations are distinct.  Returns the integer
    locations s_j, or None.
    """
    d = n // m
    s_out = []
    for zj in z:
        if not np.isfinite(zj) or abs(abs(zj) - 1.0) > taus.delta_mag:
            return None
        s_real = (np.angle(zj) * n / TWO_PI) % n
        t_real = (s_real - k) / m
        t = int(np.floor(t_real + 0.5))
        if abs(t_real - t) > taus.delta_grid:
            return None
        s_out.append(k + (t % d) * m)
    if len(set(s_out)) != len(s_out):
        return None
    return np.array(s_out, np.int64)


def vandermonde(s, n: int, rows: int) -> np.ndarray:
    """V_{lj} = z_j^l = e^{i 2 pi s_j l / N} for l < rows (phase reduced in integers)."""
    s = np.asarray(s, np.int64)
    l = np.arange(rows, dtype=np.int64)
    return np.exp(1j * TWO_PI * ((l[:, None] * s[None, :]) % n) / n)


def amplitudes(mk, s, n: int):
    """Step (iii): p = argmin ||V p - m|| over all 2L syndromes; returns (p, residual^2)."""
    mk = np.asarray(mk, np.complex128)
    v = vandermonde(s, n, len(mk))
    p = np.linalg.lstsq(v, mk, rcond=None)[0]
    r = mk - v @ p
    return p, float(np.real(np.vdot(r, r)))


def decode_bin(mk, k: int, n: int, m: int, L: int, a0: int, e_k: float, nu: float, taus: Taus,
               only=None, skip=()):
    """Syndrome decoding of one bin (Sec. II-B Steps (i)-(iii), Alg. 1 grid check),
    over the canonical order of hypotheses, with the residual judge.

    Returns (locations, values, accepted order) or None when every order is
    rejected (the bin is flagged).  `only` restricts the hypotheses tried;
    `skip` removes some from the canonical order.
    """
    for a in (only if only is not None else try_orders(a0, L)):
        if a in skip:
            continue
        c = locator(mk, a)
        if c is None:
            continue
        z = poly_roots(c)
        s = roots_to_grid(z, k, n, m, taus)
        if s is None:
            continue
        p, r2 = amplitudes(mk[:2 * L], s, n)
        if r2 <= taus.tau_res ** 2 * e_k + taus.c_res * (2 * L - a) * nu:
            keep = np.abs(p) >= taus.tau_amp * np.max(np.abs(p))
            order = np.argsort(s[keep])
            return s[keep][order], p[keep][order], a
    return None


@dataclasses.dataclass
class Result:
    locs: np.ndarray
    vals: np.ndarray
    active_bins: int = 0
    flagged_bins: int = 0
    cs_bins: int = 0
    orders: dict = dataclasses.field(default_factory=dict)   # bin -> accepted order


def _sorted(locs, vals):
    locs = np.asarray(locs, np.int64)
    vals = np.asarray(vals, np.complex128)
    o = np.argsort(locs)
    return locs[o], vals[o]


def sfft_exact(x, n: int, m: int, L: int, taus: Taus | None = None, orders=None,
               fft_dtype=np.complex128) -> Result:
    """Non-iterative sFFT-DT for exactly K-sparse signals (Sec. II-B/II-C):
    2L consecutive shifts, one FFT each, then syndrome decoding of every
    active bin.  `orders` (optional, bin -> predicted order) is tried first,
    before the rank test and the canonical order (the learned predictor's
    hook); fft_dtype as in syndromes()."""
    if taus is None:
        taus = default_taus(np.asarray(x).dtype == np.complex128)
    msyn = syndromes(x, n, m, range(2 * L), fft_dtype)
    e = bin_energy(msyn)
    e_ref = float(np.mean(e))
    locs, vals = [], []
    res = Result(np.empty(0, np.int64), np.empty(0, np.complex128))
    for k in range(m):
        if not (e[k] > taus.tau_zero ** 2 * e_ref):
            continue
        res.active_bins += 1
        mk = msyn[:, k]
        a_pred = int(orders.get(k, 0)) if orders is not None else 0
        out = None
        if 1 <= a_pred <= L:
            out = decode_bin(mk, k, n, m, L, a_pred, float(e[k]), 0.0, taus, only=[a_pred])
        if out is None:
            a0 = rank_order(hankel_singular_values(mk, L), taus.tau_rank)
            skip = [a_pred] if 1 <= a_pred <= L else []
            out = decode_bin(mk, k, n, m, L, a0, float(e[k]), 0.0, taus, skip=skip)
        if out is None:
            res.flagged_bins += 1
            continue
        locs.extend(out[0])
        vals.extend(out[1])
        res.orders[k] = out[2]
    res.locs, res.vals = _sorted(locs, vals)
    return res


def sfft_unknown_k(x, n: int, L: int, m_min: int = 1, m_max: int | None = None, taus: Taus | None = None,
                   fft_dtype=np.complex128):
    """Sec. II-G, K unknown: start at d = N (M = m_min, normally 1) and run
    the exactly-K-sparse method; while some bin cannot be solved (a flagged
    bin), halve d and run again.  Returns (result, M) of the first run without
    a flagged bin, or of the run at m_max when every run before it had one."""
    if m_max is None:
        m_max = n
    m = m_min
    while True:
        res = sfft_exact(x, n, m, L, taus=taus, fft_dtype=fft_dtype)
        if res.flagged_bins == 0 or m >= m_max:
            return res, m
        m *= 2


# ------------------------------------------------------------ general mode


def noise_floor(e: np.ndarray, L: int) -> float:
    """nu = median_k(E_k) / (2L - 1/3).

    The paper has no noise floor (it relies on the K-vote); this is the
    project's rule: for a noise-only bin E_k is Gamma(2L, nu) distributed,
    whose median is close to nu (2L - 1/3).  The median is the lower median
    (sorted[(M-1)//2]).
    """
    srt = np.sort(e)
    return float(srt[(len(e) - 1) // 2]) / (2.0 * L - 1.0 / 3.0)


def vote(sv_all: np.ndarray, k_votes: int) -> np.ndarray:
    """Pruning Step 1 / Alg. 2 Part 2: the K largest of all M*L singular values
    vote for their bins; a0[k] = number of votes of bin k.  Ties: larger sigma
    first, then lower bin, then lower index within the bin."""
    m, L = sv_all.shape
    flat = sv_all.reshape(-1)
    idx = np.arange(flat.size)
    order = np.lexsort((idx, -flat))          # primary: -sigma, secondary: flat index
    chosen = order[:min(k_votes, flat.size)]
    return np.bincount(chosen // L, minlength=m)


def candidate_errors(c, k: int, n: int, m: int) -> np.ndarray:
    """|P~(z)| for all z in U_k = {e^{i 2 pi (k + t M) / N}, t < d} (Pruning Step 2)."""
    d = n // m
    t = np.arange(d, dtype=np.int64)
    z = np.exp(1j * TWO_PI * ((k + t * m) % n) / n)
    p = np.ones_like(z)
    for j in range(len(c) - 1, -1, -1):
        p = p * z + c[j]
    return np.abs(p)


def subspace_pursuit(y, phi, a: int, max_iter: int | None = None):
    """Subspace Pursuit (Dai & Milenkovic 2009), as cited for the CS step (Sec. III-A).

    Start from the a columns most correlated with y; each iteration merges the
    a columns most correlated with the residual, solves least squares on the
    merged set, keeps the a largest coefficients and re-solves; stops when the
    residual norm no longer decreases.  Ties go to the lower column index.
    Returns (support indices, coefficients)."""
    y = np.asarray(y, np.complex128)
    ncol = phi.shape[1]
    a = min(a, ncol)
    if max_iter is None:
        max_iter = 2 * a + 2

    def top(vals, cnt):
        o = np.lexsort((np.arange(len(vals)), -np.asarray(vals)))
        return np.sort(o[:cnt])

    def solve(sup):
        coef = np.linalg.lstsq(phi[:, sup], y, rcond=None)[0]
        return coef, y - phi[:, sup] @ coef

    sup = top(np.abs(phi.conj().T @ y), a)
    coef, res = solve(sup)
    for _ in range(max_iter):
        extra = top(np.abs(phi.conj().T @ res), a)
        merged = np.union1d(sup, extra)
        cm, _ = solve(merged)
        new = np.sort(merged[top(np.abs(cm), a)])
        cn, rn = solve(new)
        if np.linalg.norm(rn) >= np.linalg.norm(res):
            break
        sup, coef, res = new, cn, rn
    return sup, coef


def cs_bin(mk, yk, k: int, n: int, m: int, a0: int, rshifts, R: int):
    """CS recovery of one flagged bin (Sec. III-A Eq. (11), Sec. III-C Steps 2-3,
    SP): prune U_k to the min(2 a0, R, d) roots with the smallest |P~(z)|, where
    P~ comes from the order-a0 locator, build Phi_p with
    Phi_{j,t} = e^{i 2 pi (k + t M) n_j / N}, run SP with sparsity a0.
    Returns None when the order-a0 locator system is singular (the bin then
    stays flagged with no output)."""
    d = n // m
    c = locator(mk, a0)
    if c is None:
        return None                     # nothing to prune with: the bin stays flagged
    err = candidate_errors(c, k, n, m)
    keep = min(2 * a0, R, d)
    o = np.lexsort((np.arange(d), err))
    cand = np.sort(o[:keep]).astype(np.int64)
    s_cand = k + cand * m
    nj = np.asarray(rshifts, np.int64)
    phi = np.exp(1j * TWO_PI * ((nj[:, None] * s_cand[None, :]) % n) / n)
    sup, coef = subspace_pursuit(yk, phi, a0)
    return s_cand[sup], coef


def sfft_general(x, n: int, k_sparsity: int, m: int, L: int, rshifts, taus: Taus | None = None,
                 fft_dtype=np.complex128, sp_all: bool = False) -> Result:
    """Non-iterative sFFT-DT for generally K-sparse signals (Sec. III, Alg. 2),
    with the CS step run on the bins the syndrome decoder flags.

    Part 1: syndromes at 2L consecutive shifts and at the R random shifts n_j.
    Part 2: per-bin Hankel singular values, global K-vote for the order a0.
    Then per voted bin: syndrome decoding with the noise-aware judge; flagged
    bins go through pruning (Steps 2-3) and SP on the n_j syndromes.
    Finally the K largest values are kept (Eq. (9): the output is K-sparse).

    sp_all=True is Alg. 2 as printed: every voted bin goes straight to
    pruning (Steps 2-3) and SP with sparsity a0, no syndrome decoding first.
    """
    if taus is None:
        taus = default_taus(np.asarray(x).dtype == np.complex128)
    R = len(rshifts)
    msyn = syndromes(x, n, m, range(2 * L), fft_dtype)
    ysyn = syndromes(x, n, m, rshifts, fft_dtype)
    e = bin_energy(msyn)
    nu = noise_floor(e, L)
    sv_all = np.array([hankel_singular_values(msyn[:, k], L) for k in range(m)])
    a0s = vote(sv_all, k_sparsity)
    locs, vals = [], []
    res = Result(np.empty(0, np.int64), np.empty(0, np.complex128))
    for k in range(m):
        a0 = int(a0s[k])
        if a0 == 0:
            continue
        res.active_bins += 1
        mk = msyn[:, k]
        out = None if sp_all else decode_bin(mk, k, n, m, L, a0, float(e[k]), nu, taus)
        if out is None:
            res.flagged_bins += 1
            cs = cs_bin(mk, ysyn[:, k], k, n, m, a0, rshifts, R)
            if cs is None:
                continue
            res.cs_bins += 1
            s, p = cs
        else:
            s, p = out[0], out[1]
            res.orders[k] = out[2]
        locs.extend(s)
        vals.extend(p)
    locs = np.asarray(locs, np.int64)
    vals = np.asarray(vals, np.complex128)
    if len(locs) > k_sparsity:
        o = np.lexsort((locs, -np.abs(vals)))[:k_sparsity]
        locs, vals = locs[o], vals[o]
    res.locs, res.vals = _sorted(locs, vals)
    return res


# ------------------------------------------------------------------ metrics


def snr_db(xh, locs_out, vals_out) -> float:
    """SNR(x_out) = 10 log10(||x_out||^2 / ||x_hat - x_out||^2) (the SNR
    definition of Sec. III-F's experiments, with MSE over all N entries)."""
    xh = np.asarray(xh, np.complex128)
    locs_out = np.asarray(locs_out, np.int64)
    vals_out = np.asarray(vals_out, np.complex128)
    err = float(np.sum(np.abs(xh) ** 2))
    err += float(np.sum(np.abs(xh[locs_out] - vals_out) ** 2) - np.sum(np.abs(xh[locs_out]) ** 2))
    return 10.0 * np.log10(float(np.sum(np.abs(vals_out) ** 2)) / max(err, 1e-300))


def support_recovery(locs_true, locs_out) -> float:
    """Fraction of the true support found."""
    return len(np.intersect1d(locs_true, locs_out)) / max(1, len(locs_true))


def relative_l2(locs_true, vals_true, locs_out, vals_out) -> float:
    """||x_hat_s - x_hat_out|| / ||x_hat_s|| over the union of supports."""
    u = np.union1d(locs_true, locs_out)
    a = np.zeros(len(u), np.complex128)
    b = np.zeros(len(u), np.complex128)
    a[np.searchsorted(u, locs_true)] = vals_true
    b[np.searchsorted(u, locs_out)] = vals_out
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(a), 1e-300))
