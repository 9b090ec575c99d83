"""Collision and recovery statistics on the device (Sec. II-C, Lemma 2, Fig. 2;
the non-iterative recovery-versus-K curve of Sec. II-H, Fig. 4), through the C
ABI.

A sweep cell is a batch of exactly K-sparse signals (unit amplitudes,
complex64 input, FP64 FFTs so that no single-precision effect enters) decoded
with one (M, L).  Checked per cell: every signal's support equals the FP64
oracle's; the recovered fraction follows the collision model (a frequency is
recovered when its bin holds at most L frequencies: hypergeometric, K - 1
others among N - 1 positions, d - 1 of them in its bin) within the sampling
spread; the fraction of signals missing a frequency stays under Lemma 2's
bound (N/d) (d e K / (N (L + 1)))^(L + 1) where that bound is below 1."""
import math
import sys

import numpy as np
import pytest
from scipy.stats import hypergeom

import oracle
import sftgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def sft():
    import paper_1407_8315_amd as m

    return m


@pytest.mark.parametrize("n,k,m,L", [
    (1 << 20, 1000, 2048, 2),       # N+ = N/(dK) = 2: collisions of 3 lose frequencies
    (1 << 20, 1000, 4096, 4),       # the exact workload's (M, L)
    (1 << 20, 1 << 12, 1 << 14, 4),  # Fig. 4's d = N/(4K), K = 2^12 (two FFT passes)
    (1 << 20, 1 << 8, 1 << 10, 1),  # Fig. 4's d = N/(4K), K = 2^8, one collision decoded
])
def test_sweep_cell_matches_oracle_and_model(torch, sft, n, k, m, L):
    B = 16
    d = n // m
    say(f"[sweep cell] N={n} K={k} M={m} L={L}, {B} signals")
    sigs = [sftgen.make_signal(n, k, sftgen.BASE_SEED + 60000 + 100 * L + i, amp="unit", dtype=np.complex64)
            for i in range(B)]
    plan = sft.Plan([dict(n=n, k=k, m=m, l=L, flags=sft.SFT_FLAG_FFT64)] * B)
    outs = plan.batch([torch.from_numpy(s.x).cuda() for s in sigs], stats=True)
    found, imperfect = 0, 0
    for i, (o, s) in enumerate(zip(outs, sigs)):
        loc, val = o.host()
        ref = oracle.sfft_exact(s.x, n, m, L)
        assert loc.tolist() == ref.locs.tolist(), i
        if len(loc):
            assert np.max(np.abs(val - ref.vals)) <= 1e-9 * max(1.0, np.max(np.abs(ref.vals))), i
        got = len(np.intersect1d(loc, s.locs))
        found += got
        imperfect += got < k
    plan.close()
    rec = found / (B * k)
    model = float(hypergeom.cdf(L - 1, n - 1, d - 1, k - 1))
    lemma2 = (n / d) * (d * math.e * k / (n * (L + 1))) ** (L + 1)
    # the frequencies of one signal are not independent: allow 4 sigma of
    # a binomial over the signals' totals, inflated by 2
    sd = 2.0 * math.sqrt(model * (1 - model) / (B * k))
    say(f"  recovery {rec:.6f}, model {model:.6f} (4 sd {4 * sd:.1e}); signals with a miss {imperfect}/{B}, "
        f"Lemma 2 bound {min(1.0, lemma2):.4f}")
    assert abs(rec - model) <= 4 * sd + 2e-4
    if lemma2 < 1:
        assert imperfect / B <= lemma2 + 3 * math.sqrt(0.25 / B)
