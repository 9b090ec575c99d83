"""GPU parity of the sFFT-DT path against the FP64 oracle, through the C ABI.

Tolerances: complex128 input runs the FFT in FP64 (syndromes within 1e-12 of
the oracle's, values within 1e-10; supports and flags compared exactly);
complex64 input runs it in FP32 (syndromes within 2e-6 relative L2, values
within 1e-5 relative L2 — the target of the exact-input workload) and is
compared with the FP64 oracle bin by bin: a bin may differ only where the FP64
decision itself is fragile at single-precision rounding (fp64_parity).
"""
import sys

import numpy as np
import pytest

import oracle
import sftgen
from fp64_parity import exact_vs_fp64

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


def to_dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------ syndromes


@pytest.mark.parametrize("n,m,L,dtype,mode", [
    (1 << 14, 128, 4, "c128", "exact"),
    (1 << 20, 4096, 4, "c64", "exact"),
    (1 << 20, 4096, 4, "c64", "general"),
    (1 << 12, 16, 2, "c64", "exact"),
    (1 << 10, 32, 3, "c128", "general"),
    (32, 8, 4, "c128", "exact"),            # d = 4 < 2L: indices wrap
    (1 << 16, 8192, 4, "c64", "exact"),     # largest M held in one block (FP32)
    (1 << 16, 4096, 1, "c128", "exact"),    # largest M held in one block (FP64)
    (1 << 16, 16384, 4, "c64", "exact"),    # two FFT passes, 128 x 128
    (1 << 18, 32768, 2, "c64", "general"),  # two FFT passes, 256 x 128, random shifts
    (1 << 16, 8192, 2, "c128", "exact"),    # two FFT passes in FP64, 64 x 128
    (1 << 24, 65536, 4, "c64", "exact"),    # N = 2^24, K = 2^14: 256 x 256
])
def test_syndromes_match_oracle(torch, sft, n, m, L, dtype, mode):
    say(f"[syndromes] n={n} m={m} L={L} {dtype} {mode}")
    npdt = np.complex128 if dtype == "c128" else np.complex64
    s = sftgen.make_signal(n, max(1, m // 4), 11, amp="gauss", dtype=npdt)
    plan = sft.Plan(dict(n=n, k=max(1, m // 4), m=m, l=L, dtype=dtype, mode=mode, seed=7))
    got = plan.syndromes(to_dev(torch, s.x)).cpu().numpy()
    torch.cuda.synchronize()
    info = plan.info()
    shifts = list(range(2 * L)) + info["rshifts"]
    ref = oracle.syndromes(s.x, n, m, shifts)
    assert got.shape == ref.shape
    if dtype == "c128":
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    else:
        assert rel_l2(got, ref) <= 2e-6
        assert np.max(np.abs(got - ref)) <= 2e-5 * np.max(np.abs(ref))
    plan.close()


# ------------------------------------------------------------ exact mode


def run_exact(torch, sft, x, n, m, L, dtype, **kw):
    plan = sft.Plan(dict(n=n, k=1, m=m, l=L, dtype=dtype, **kw))
    res = plan.exact(to_dev(torch, x), stats=True)
    loc, val = res.host()
    plan.close()
    return loc, val, res.stats


@pytest.mark.parametrize("seed", range(6))
def test_exact_small_complex128(torch, sft, seed):
    """N = 2^14, K = 50, M = 128, L = 4, unit amplitudes, complex128."""
    n, k, m, L = 1 << 14, 50, 128, 4
    say(f"[exact c128] seed={seed}")
    s = sftgen.make_signal(n, k, sftgen.BASE_SEED + seed, amp="unit", dtype=np.complex128)
    loc, val, st = run_exact(torch, sft, s.x, n, m, L, "c128")
    ref = oracle.sfft_exact(s.x, n, m, L)
    assert loc.tolist() == ref.locs.tolist()
    assert np.max(np.abs(val - ref.vals)) <= 1e-10
    assert st["flagged_bins"] == ref.flagged_bins and st["active_bins"] == ref.active_bins


@pytest.mark.parametrize("seed", range(2))
def test_exact_n20_complex64_fft64(torch, sft, seed):
    """complex64 input with SFT_FLAG_FFT64 (FP64 FFTs): decisions equal the
    oracle's with FP64 FFTs and the complex64 thresholds, values within 1e-9."""
    n, k, m, L = 1 << 20, 1000, 4096, 4
    say(f"[exact c64 fft64 N=2^20] seed={seed}")
    s = sftgen.make_signal(n, k, sftgen.BASE_SEED + 150 + seed, amp="gauss", dtype=np.complex64)
    loc, val, st = run_exact(torch, sft, s.x, n, m, L, "c64", flags=sft.SFT_FLAG_FFT64)
    ref = oracle.sfft_exact(s.x, n, m, L)
    assert loc.tolist() == ref.locs.tolist()
    assert st["flagged_bins"] == ref.flagged_bins and st["active_bins"] == ref.active_bins
    assert rel_l2(val, ref.vals) <= 1e-9


@pytest.mark.parametrize("seed", range(3))
def test_exact_n20_complex64(torch, sft, seed):
    """N = 2^20, K = 1000, M = 4096, L = 4, complex Gaussian values, complex64:
    support and flags equal to the FP64 oracle's except in FP32-fragile bins
    (at most 2), values within 1e-5 relative L2."""
    n, k, m, L = 1 << 20, 1000, 4096, 4
    say(f"[exact c64 N=2^20] seed={seed}")
    s = sftgen.make_signal(n, k, sftgen.BASE_SEED + 100 + seed, amp="gauss", dtype=np.complex64)
    loc, val, st = run_exact(torch, sft, s.x, n, m, L, "c64")
    ref, diff = exact_vs_fp64(loc, val, st, s.x, n, m, L, max_diff=2, truth=(s.locs, s.vals), say=say)
    assert len(loc) >= 0.99 * k
    if ref.flagged_bins == 0 and not diff:
        assert loc.tolist() == s.locs.tolist()


COLLISIONS = [
    (4096, 64, 5, [3, 4]),
    (4096, 64, 63, [0, 63]),
    (4096, 64, 0, [10, 11, 12]),
    (4096, 64, 17, [0, 1, 2, 3]),
    (4096, 64, 33, [2, 19, 40, 61]),
    (1 << 16, 256, 200, [1, 2, 100, 255]),
    (32, 8, 3, [0, 1, 2, 3]),
    (64, 32, 7, [0, 1]),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,m,k,slots", COLLISIONS)
def test_forced_collisions(torch, sft, n, m, k, slots, dtype):
    """Bins holding a = 2..4 aliased tones (adjacent slots, wrap-around, d < 2L)."""
    say(f"[collisions] n={n} m={m} bin={k} slots={slots} {dtype}")
    g = np.random.default_rng(len(slots) * 1000 + k)
    locs, vals = sftgen.colliding_spectrum(n, m, k, slots, np.exp(2j * np.pi * g.random(len(slots))))
    npdt = np.complex128 if dtype == "c128" else np.complex64
    x = sftgen.make_signal(n, len(locs), 0, locs=locs, vals=vals, dtype=npdt).x
    loc, val, st = run_exact(torch, sft, x, n, m, 4, dtype)
    ref = oracle.sfft_exact(x, n, m, 4)
    if dtype == "c128":
        assert loc.tolist() == ref.locs.tolist() == locs.tolist()
        assert rel_l2(val, ref.vals) <= 1e-10
        return
    # FP32 syndromes: equal to the FP64 oracle unless the bin is fragile
    exact_vs_fp64(loc, val, st, x, n, m, 4, max_diff=1, truth=(locs, vals), say=say)


def test_more_than_L_is_flagged_and_zero_signal_is_empty(torch, sft):
    n, m, k = 4096, 64, 11
    g = np.random.default_rng(3)
    for L in (1, 2, 3, 4):
        say(f"[flag] L={L}")
        slots = g.choice(n // m, L + 1, replace=False)
        locs, vals = sftgen.colliding_spectrum(n, m, k, slots, np.exp(2j * np.pi * g.random(L + 1)))
        x = sftgen.make_signal(n, len(locs), 0, locs=locs, vals=vals, dtype=np.complex128).x
        loc, val, st = run_exact(torch, sft, x, n, m, L, "c128")
        assert len(loc) == 0 and st["flagged_bins"] == 1
    say("[zero signal]")
    loc, val, st = run_exact(torch, sft, np.zeros(n, np.complex64), n, m, 4, "c64")
    assert len(loc) == 0 and st["active_bins"] == 0


def test_flags_match_oracle_dense(torch, sft):
    """Many a > L bins (K/M > 1): same flags and the same recovered set."""
    n, k, m, L = 1 << 14, 300, 256, 2
    say("[dense flags]")
    s = sftgen.make_signal(n, k, 101, dtype=np.complex128)
    loc, val, st = run_exact(torch, sft, s.x, n, m, L, "c128")
    ref = oracle.sfft_exact(s.x, n, m, L)
    assert st["flagged_bins"] == ref.flagged_bins > 0
    assert loc.tolist() == ref.locs.tolist()


def test_capacity_and_nonfinite(torch, sft):
    n, k, m = 1 << 14, 50, 128
    s = sftgen.make_signal(n, k, 5, dtype=np.complex64)
    say("[capacity]")
    plan = sft.Plan(dict(n=n, k=k, m=m, l=4))
    res = plan.exact(to_dev(torch, s.x), capacity=10, stats=True)
    assert res.stats.get("capacity_exceeded")
    assert int(res.count.item()) == 50
    assert res.loc[:10].cpu().numpy().tolist() == s.locs[:10].tolist()
    plan.close()
    say("[nonfinite]")
    x = s.x.copy()
    x[(n // m) * 5 + 1] = np.nan        # a gathered sample (shift 1, k' = 5)
    plan = sft.Plan(dict(n=n, k=k, m=m, l=4, flags=sft.SFT_FLAG_CHECK_FINITE))
    with pytest.raises(sft.SftError) as e:
        plan.exact(to_dev(torch, x), stats=True)
    assert "NONFINITE" in str(e.value)
    plan.close()


def test_async_call_and_plan_reuse(torch, sft):
    """Calls without stats are asynchronous; a plan is reused across inputs."""
    n, k, m, L = 1 << 16, 200, 1024, 4
    plan = sft.Plan(dict(n=n, k=k, m=m, l=L))
    for seed in range(3):
        say(f"[reuse] seed={seed}")
        s = sftgen.make_signal(n, k, 40 + seed, dtype=np.complex64)
        res = plan.exact(to_dev(torch, s.x))
        torch.cuda.synchronize()
        loc, val = res.host()
        ref = oracle.sfft_exact(s.x, n, m, L)
        assert loc.tolist() == ref.locs.tolist()
    plan.close()


@pytest.mark.parametrize("k", [1 << 10, 1 << 12, 1 << 14])
def test_exact_n24(torch, sft, k):
    """N = 2^24, K in {2^10, 2^12, 2^14}, M = 4K (one and two FFT passes),
    L = 4, unit amplitudes, complex64.

    Decisions are compared bin by bin with the FP64 oracle: a bin may differ
    only when its decision is fragile at FP32 FFT rounding (an ill-conditioned
    cluster of 3-4 aliased tones, or two tones a few slots apart), and such
    bins stay a handful.  Values at the common locations within 1e-5;
    recovery is at least 99%."""
    n, m, L = 1 << 24, 4 * k, 4
    say(f"[exact N=2^24] K={k} M={m}")
    s = sftgen.make_signal(n, k, sftgen.BASE_SEED + 24, amp="unit", dtype=np.complex64)
    loc, val, st = run_exact(torch, sft, s.x, n, m, L, "c64")
    exact_vs_fp64(loc, val, st, s.x, n, m, L, max_diff=max(2, k // 4096), truth=(s.locs, s.vals), say=say)
    assert len(loc) >= 0.99 * k


@pytest.mark.parametrize("layout", ["spread", "clustered"])
def test_long_output_lists_sorted(torch, sft, layout):
    """Output lists longer than one LDS sort (2048 entries), complex128 (FP64
    FFTs), N = 2^20, M = 8192, L = 4, K = 3000.  Locations spread over [0, N)
    go through the bucket sort (about 3 entries per bucket of 1024
    locations); locations packed below 4096 (one tone per bin) fill four
    buckets beyond the bucket limit and go through the chunked rank.  Either
    way the list equals the oracle's (sorted by location, values within
    1e-10), and a capacity of 2500 keeps its first 2500 entries."""
    n, m, L, k = 1 << 20, 8192, 4, 3000
    g = np.random.default_rng(11)
    hi = n if layout == "spread" else 4096
    locs = np.sort(g.choice(hi, size=k, replace=False)).astype(np.int64)
    vals = np.exp(2j * np.pi * g.random(k))
    s = sftgen.make_signal(n, k, 0, locs=locs, vals=vals, dtype=np.complex128)
    say(f"[long output] {layout}")
    ref = oracle.sfft_exact(s.x, n, m, L)
    assert len(ref.locs) > 2048
    plan = sft.Plan(dict(n=n, k=k, m=m, l=L, dtype="c128"))
    res = plan.exact(to_dev(torch, s.x), stats=True)
    loc, val = res.host()
    assert loc.tolist() == ref.locs.tolist()
    assert np.max(np.abs(val - ref.vals)) <= 1e-10
    res = plan.exact(to_dev(torch, s.x), capacity=2500, stats=True)
    assert res.stats.get("capacity_exceeded")
    assert int(res.count.item()) == len(ref.locs)
    assert res.loc[:2500].cpu().numpy().tolist() == ref.locs[:2500].tolist()
    plan.close()
