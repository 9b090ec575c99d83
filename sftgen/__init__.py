"""Seeded synthetic inputs for sFFT-DT (arXiv 1407.8315), shared by the oracle
side (tests, CPU baseline) and the GPU side (bench, parity tests).

This module holds no arithmetic of the method itself.  It only draws a sparse
spectrum x_hat and returns the time signal x = IDFT(x_hat), which is how the
paper builds its test signals (Sec. II-H: generate a K-sparse spectrum, then
take its inverse FFT).  The DFT convention is the unnormalised forward
transform X[f] = sum_n x[n] e^{-2 pi i f n / N}, so x = ifft(x_hat) with the
1/N on the inverse.

Noise model of the generally-K-sparse case: x_hat = x_hat_s + eta with eta
i.i.d. complex Gaussian on all N bins, scaled so that
||x_hat_s||^2 / ||eta||^2 = 10^(SNR/10) exactly (the significant-to-
insignificant energy ratio of Eq. (22)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 0x14078315


@dataclasses.dataclass
class Sparse:
    """A drawn test signal: time samples and its significant spectrum."""

    x: np.ndarray          # time signal, complex64 or complex128, length n
    n: int
    locs: np.ndarray       # int64 sorted significant locations (the K-sparse support)
    vals: np.ndarray       # complex128 significant values at locs
    noise_var: float       # per-bin variance of eta (0 for exact signals)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def draw_spectrum(n: int, k: int, seed: int, amp: str = "unit"):
    """K distinct locations uniform on [0, n) and their values.

    amp = "unit": unit magnitude, uniform phase.  amp = "gauss": CN(0, 1).
    """
    if not (1 <= k <= n):
        raise ValueError("need 1 <= k <= n")
    g = _rng(seed)
    locs = np.sort(g.choice(n, size=k, replace=False)).astype(np.int64)
    if amp == "unit":
        vals = np.exp(2j * np.pi * g.random(k))
    elif amp == "gauss":
        vals = (g.standard_normal(k) + 1j * g.standard_normal(k)) / math.sqrt(2.0)
    else:
        raise ValueError(amp)
    return locs, vals.astype(np.complex128), g


def make_signal(n: int, k: int, seed: int, amp: str = "unit", snr_db=None,
                dtype=np.complex64, locs=None, vals=None) -> Sparse:
    """x = IDFT(x_hat) for a K-sparse x_hat (+ white spectral noise at snr_db)."""
    if locs is None:
        locs, vals, g = draw_spectrum(n, k, seed, amp)
    else:
        locs = np.asarray(locs, np.int64)
        vals = np.asarray(vals, np.complex128)
        g = _rng(seed)
    xh = np.zeros(n, np.complex128)
    xh[locs] = vals
    noise_var = 0.0
    if snr_db is not None:
        eta = (g.standard_normal(n) + 1j * g.standard_normal(n)) / math.sqrt(2.0)
        es = float(np.sum(np.abs(vals) ** 2))
        en = float(np.sum(np.abs(eta) ** 2))
        scale = math.sqrt(es / (en * 10.0 ** (snr_db / 10.0)))
        eta *= scale
        noise_var = scale * scale
        xh += eta
    x = np.fft.ifft(xh).astype(dtype)
    return Sparse(x=x, n=n, locs=locs, vals=vals, noise_var=noise_var)


@dataclasses.dataclass
class Mixture:
    """A mixture-Gaussian test signal (its dense spectrum kept for SNR)."""

    x: np.ndarray          # time signal
    xh: np.ndarray         # complex128 spectrum, length n
    locs: np.ndarray       # the positions drawn from the "on" component (x_hat_s)
    snr_db: float          # SNR(x_hat_s) = 10 log10(||x_hat_s||^2 / ||x_hat - x_hat_s||^2), exact


def mixture_signal(n: int, k: int, snr_db: float, seed: int, dtype=np.complex64) -> Mixture:
    """The mixture-Gaussian model of Eq. (21): each entry of x_hat is drawn
    from CN(0, s_on^2) with probability p = K/N, else from CN(0, s_off^2);
    s_off is then set so that SNR(x_hat_s) equals snr_db exactly."""
    g = _rng(seed)
    on = g.random(n) < (k / n)
    xh = (g.standard_normal(n) + 1j * g.standard_normal(n)) / math.sqrt(2.0)
    es = float(np.sum(np.abs(xh[on]) ** 2))
    en = float(np.sum(np.abs(xh[~on]) ** 2))
    xh[~on] *= math.sqrt(es / (en * 10.0 ** (snr_db / 10.0)))
    locs = np.flatnonzero(on).astype(np.int64)
    return Mixture(x=np.fft.ifft(xh).astype(dtype), xh=xh, locs=locs, snr_db=float(snr_db))


def torch_mixture(n: int, k: int, snr_db: float, seed: int, device):
    """Device-side variant of mixture_signal (same draws; the inverse FFT runs
    in torch's complex128 on the device, cast to complex64).  Returns
    (x_device complex64, xh_device complex128, number of significant entries)."""
    import torch

    g = _rng(seed)
    on = g.random(n) < (k / n)
    xh = (g.standard_normal(n) + 1j * g.standard_normal(n)) / math.sqrt(2.0)
    es = float(np.sum(np.abs(xh[on]) ** 2))
    en = float(np.sum(np.abs(xh[~on]) ** 2))
    xh[~on] *= math.sqrt(es / (en * 10.0 ** (snr_db / 10.0)))
    xh_d = torch.from_numpy(xh).to(device)
    x = torch.fft.ifft(xh_d).to(torch.complex64)
    return x, xh_d, int(on.sum())


def make_batch(n: int, k: int, count: int, seed0: int = BASE_SEED, **kw):
    """count signals of one shape with seeds seed0 + i."""
    return [make_signal(n, k, seed0 + i, **kw) for i in range(count)]


def colliding_spectrum(n: int, m: int, bin_k: int, slots, vals):
    """Locations k + t*M for the given alias slots t of one bin (forced collisions)."""
    locs = np.array([bin_k + int(t) * m for t in slots], np.int64)
    order = np.argsort(locs)
    return locs[order], np.asarray(vals, np.complex128)[order]


def uneven_batch_params(count: int, seed: int = BASE_SEED):
    """Per-signal (N, K) of the batched uneven workload.

    N = 2^e with e uniform on {14..22}; K = round(2^u), u uniform on [4, 12],
    then K = min(K, N/64) so every signal keeps a downsampling factor >= 16.
    """
    g = _rng(seed)
    e = g.integers(14, 23, size=count)
    u = g.uniform(4.0, 12.0, size=count)
    ns = (1 << e).astype(np.int64)
    ks = np.minimum(np.round(2.0 ** u).astype(np.int64), ns // 64)
    return ns, ks


def torch_signal(n: int, k: int, seed: int, device, amp: str = "unit", snr_db=None):
    """Device-side variant of make_signal for large batches (same draw of
    locations/values; the inverse FFT runs in torch's complex128 on device and
    is cast to complex64).  Returns (x_device, locs, vals)."""
    import torch

    locs, vals, g = draw_spectrum(n, k, seed, amp)
    xh = torch.zeros(n, dtype=torch.complex128, device=device)
    xh[torch.from_numpy(locs).to(device)] = torch.from_numpy(vals).to(device)
    if snr_db is not None:
        eta = (g.standard_normal(n) + 1j * g.standard_normal(n)) / math.sqrt(2.0)
        es = float(np.sum(np.abs(vals) ** 2))
        en = float(np.sum(np.abs(eta) ** 2))
        eta *= math.sqrt(es / (en * 10.0 ** (snr_db / 10.0)))
        xh += torch.from_numpy(eta).to(device)
    x = torch.fft.ifft(xh).to(torch.complex64)
    return x, locs, vals
