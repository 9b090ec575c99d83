"""GPU parity of iterative sFFT-DT (Alg. 1) against the FP64 oracle, through the C ABI.

Tolerances as for the non-iterative path: complex128 input runs the FFTs in
FP64 (syndromes within 1e-12 of the oracle's, values within 1e-10, supports
and counts exact); complex64 input runs them in FP32 (syndromes within 2e-6
relative L2; supports compared with the oracle run on the FP32-rounded
syndromes, where a location may differ only when its decision is fragile at
FP32 FFT rounding; values within 1e-5 relative L2 of the FP64 oracle).
"""
import sys

import numpy as np
import pytest

import oracle
import sftgen
from fp64_parity import iterative_vs_fp64
from oracle import iterative as oit

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


def exact_signal(n, locs, vals, dtype=np.complex128):
    xh = np.zeros(n, np.complex128)
    xh[np.asarray(locs, np.int64)] = vals
    return np.fft.ifft(xh).astype(dtype)


def run_iter(torch, sft, x, n, m0, L, dtype):
    plan = sft.Plan(dict(n=n, k=1, m=m0, l=L, dtype=dtype, mode="iterative"))
    res = plan.iterative(to_dev(torch, x), stats=True)
    loc, val = res.host()
    plan.close()
    return loc, val, res.stats


# ------------------------------------------------------------ syndromes


@pytest.mark.parametrize("n,m0,L,dtype", [
    (1 << 14, 256, 4, "c128"),
    (1 << 20, 4096, 4, "c64"),       # every grid of a signal in one block (M_l = 4096 .. 512)
    (1 << 18, 2048, 4, "c64"),       # the same, down to M_l = 256 (half a wave busy)
    (1 << 14, 512, 2, "c64"),        # the same, one wave per block
    (1 << 18, 1024, 4, "c64"),       # a grid of 128 bins: one kernel per grid size
    (16, 8, 4, "c128"),              # d_0 = 2: indices wrap; the last grid has one bin
    (1 << 16, 16384, 2, "c64"),      # iteration 0 in two FFT passes, iteration 1 in one
    (1 << 20, 4096, 4, "c64+fft64"),  # complex64 input, FP64 FFTs
    (1 << 16, 16384, 2, "c64+fft64"),
])
def test_iterative_syndromes_match_oracle(torch, sft, n, m0, L, dtype):
    say(f"[iter syndromes] n={n} m0={m0} L={L} {dtype}")
    fft64 = dtype.endswith("+fft64")
    dtype = dtype.split("+")[0]
    npdt = np.complex128 if dtype == "c128" else np.complex64
    s = sftgen.make_signal(n, max(1, m0 // 4), 12, amp="gauss", dtype=npdt)
    plan = sft.Plan(dict(n=n, k=1, m=m0, l=L, dtype=dtype, mode="iterative",
                         flags=sft.SFT_FLAG_FFT64 if fft64 else 0))
    got = [g.cpu().numpy() for g in plan.syndromes(to_dev(torch, s.x))]
    torch.cuda.synchronize()
    plan.close()
    assert len(got) == L
    for l in range(L):
        ref = oracle.syndromes(s.x, n, m0 >> l, [2 * l, 2 * l + 1])
        assert got[l].shape == ref.shape
        if dtype == "c128" or fft64:
            assert got[l].dtype == np.complex128
            assert np.max(np.abs(got[l] - ref)) <= 1e-12 * np.max(np.abs(ref))
        else:
            assert rel_l2(got[l], ref) <= 2e-6


# ------------------------------------------------------------ parity


def check_c128(torch, sft, x, n, m0, L):
    loc, val, st = run_iter(torch, sft, x, n, m0, L, "c128")
    ref, levels = oit.sfft_iterative(x, n, m0, L)
    assert loc.tolist() == ref.locs.tolist()
    if len(loc):
        assert np.max(np.abs(val - ref.vals)) <= 1e-10
    assert st["active_bins"] == ref.active_bins
    assert st["flagged_bins"] == ref.flagged_bins
    return loc, levels


@pytest.mark.parametrize("seed", range(4))
def test_iterative_paper_setting_complex128(torch, sft, seed):
    """N = 2^14, K = 64, d_0 = N / (4K) (M_0 = 256), a_m = 4, unit amplitudes."""
    n, k = 1 << 14, 64
    say(f"[iter c128] seed={seed}")
    s = sftgen.make_signal(n, k, sftgen.BASE_SEED + 300 + seed, amp="unit", dtype=np.complex128)
    loc, _ = check_c128(torch, sft, s.x, n, 4 * k, 4)
    assert loc.tolist() == sorted(s.locs.tolist())


@pytest.mark.parametrize("n,m0,k,seed", [(4096, 64, 100, 2), (1 << 14, 128, 200, 3), (2048, 16, 30, 5),
                                         (4096, 64, 40, 1)])
def test_iterative_collisions_of_every_order(torch, sft, n, m0, k, seed):
    """Supports dense enough that every iteration solves bins (the oracle's
    support-level simulation cases): GPU and oracle agree bin for bin."""
    say(f"[iter dense] n={n} m0={m0} k={k}")
    g = np.random.default_rng(seed)
    locs = np.sort(g.choice(n, k, replace=False))
    vals = g.standard_normal(k) + 1j * g.standard_normal(k)
    x = exact_signal(n, locs, vals)
    _, levels = check_c128(torch, sft, x, n, m0, 4)
    assert any(len(lv.solved) > 0 for lv in levels[1:])


def test_iterative_t_brings_a_silent_bin_to_its_decode(torch, sft):
    """The bin whose new syndromes vanish at iteration 2 (only T sends it to
    SynDec) is solved on the device as in the oracle."""
    n, m0, k = 1024, 64, 5
    locs = np.array([k + 1 * m0, k + 6 * m0, k + 11 * m0], np.int64)
    z = np.exp(2j * np.pi * locs / n)
    null = np.linalg.svd(np.array([z ** 4, z ** 5]))[2][-1].conj()
    others = np.array([1, 2 + m0, 3 + 5 * m0], np.int64)
    all_locs = np.concatenate([locs, others])
    x = exact_signal(n, all_locs, np.concatenate([null, np.array([0.9, -0.4j, 0.3 + 0.3j])]))
    loc, levels = check_c128(torch, sft, x, n, m0, 4)
    assert sorted(levels[2].solved) == sorted(locs.tolist())
    assert loc.tolist() == sorted(all_locs.tolist())


def test_iterative_correction_cancels_an_earlier_solution(torch, sft):
    """Iteration 0 accepts the midpoint of an equal-magnitude pair; iteration
    2 solves the pair and the negative of that tone: the device adds the
    correction to the midpoint's slot, which cancels and leaves the output."""
    from test_oracle_iterative import midpoint_pair

    n, m0, k = 1024, 64, 9
    locs, vals, mid = midpoint_pair(n, m0, k, 3, 11)
    others = np.array([2, 5 + 3 * m0, 40 + 7 * m0], np.int64)
    all_locs = np.concatenate([locs, others])
    x = exact_signal(n, all_locs, np.concatenate([vals, np.array([0.8, 0.5j, -0.7])]))
    loc, levels = check_c128(torch, sft, x, n, m0, 4)
    assert mid in levels[0].solved and mid not in loc.tolist()
    assert loc.tolist() == sorted(all_locs.tolist())


@pytest.mark.parametrize("n,m0,L,k", [
    (4096, 64, 1, 20),        # one iteration
    (16, 8, 4, 3),            # d_0 = 2, the last grid has a single bin
    (1 << 12, 8, 4, 6),       # M_0 = 2^(L-1)
    (1 << 14, 128, 3, 40),    # tiles of fewer bins than a block
    (1 << 16, 2048, 2, 600),  # more bins than a block
])
def test_iterative_edge_shapes(torch, sft, n, m0, L, k):
    say(f"[iter edge] n={n} m0={m0} L={L} k={k}")
    s = sftgen.make_signal(n, k, 77 + L, amp="gauss", dtype=np.complex128)
    check_c128(torch, sft, s.x, n, m0, L)


def test_iterative_zero_signal(torch, sft):
    n, m0 = 1 << 12, 64
    loc, val, st = run_iter(torch, sft, np.zeros(n, np.complex128), n, m0, 4, "c128")
    assert len(loc) == 0 and st["active_bins"] == 0 and st["flagged_bins"] == 0


@pytest.mark.parametrize("seed", range(2))
def test_iterative_n20_complex64_fft64(torch, sft, seed):
    """N = 2^20, K = 1000, M_0 = 4096, a_m = 4, complex Gaussian values,
    complex64 input with SFT_FLAG_FFT64: the oracle with FP64 FFTs and the
    complex64 thresholds decides identically (support and counts), values
    within 1e-9 relative L2."""
    n, k, m0 = 1 << 20, 1000, 4096
    say(f"[iter c64 fft64 N=2^20] seed={seed}")
    s = sftgen.make_signal(n, k, sftgen.BASE_SEED + 400 + seed, amp="gauss", dtype=np.complex64)
    plan = sft.Plan(dict(n=n, k=k, m=m0, l=4, dtype="c64", mode="iterative", flags=sft.SFT_FLAG_FFT64))
    res = plan.iterative(to_dev(torch, s.x), stats=True)
    loc, val = res.host()
    plan.close()
    ref, _ = oit.sfft_iterative(s.x, n, m0, 4)
    assert loc.tolist() == ref.locs.tolist()
    assert res.stats["active_bins"] == ref.active_bins and res.stats["flagged_bins"] == ref.flagged_bins
    assert rel_l2(val, ref.vals) <= 1e-9


@pytest.mark.parametrize("seed,amp", [(0, "gauss"), (1, "gauss"), (2, "unit")])
def test_iterative_n20_complex64(torch, sft, seed, amp):
    """N = 2^20, K = 1000, M_0 = 4096, a_m = 4, complex64 with FP32 FFTs.  The
    output is compared location by location with the FP64 oracle: a location
    may differ only in a residue class that holds an FP32-fragile one
    (iterative_vs_fp64), and the device returns only true locations.  Values
    within 1e-5 relative L2 of the FP64 oracle."""
    n, k, m0 = 1 << 20, 1000, 4096
    say(f"[iter c64 N=2^20] seed={seed} {amp}")
    s = sftgen.make_signal(n, k, sftgen.BASE_SEED + 400 + seed, amp=amp, dtype=np.complex64)
    loc, val, st = run_iter(torch, sft, s.x, n, m0, 4, "c64")
    assert set(loc.tolist()) <= set(s.locs.tolist())
    ref, ndiff = iterative_vs_fp64(loc, s.x, n, m0, 4, truth=(s.locs, s.vals), say=say)
    if ndiff == 0:
        assert st["active_bins"] == ref.active_bins and st["flagged_bins"] == ref.flagged_bins
    common, ia, ib = np.intersect1d(loc, ref.locs, return_indices=True)
    assert len(common) == len(loc) or ndiff
    assert rel_l2(val[ia], ref.vals[ib]) <= 1e-5
    assert len(loc) >= 0.99 * k


# ------------------------------------------------------------ batches


def test_iterative_batch_equals_single_calls_and_replays(torch, sft):
    """A batch of iterative signals with different N, M_0, a_m and dtype-equal
    inputs: each output equals its single-signal call bit for bit, and graph
    replays give the same lists."""
    cases = [(1 << 14, 256, 4, 64), (1 << 12, 64, 3, 40), (1 << 16, 1024, 4, 256), (1 << 10, 16, 2, 6),
             (1 << 14, 128, 1, 20), (1 << 13, 512, 4, 128), (1 << 12, 32, 4, 30), (1 << 15, 2048, 2, 300),
             (1 << 11, 64, 4, 16)]
    xs, params = [], []
    for i, (n, m0, L, k) in enumerate(cases):
        s = sftgen.make_signal(n, k, 500 + i, amp="gauss", dtype=np.complex64)
        xs.append(to_dev(torch, s.x))
        params.append(dict(n=n, k=k, m=m0, l=L, dtype="c64", mode="iterative"))
    plan = sft.Plan(params)
    outs = plan.batch(xs, stats=True)
    first = [o.host() for o in outs]
    for _ in range(2):
        again = [o.host() for o in plan.batch(xs)]
        torch.cuda.synchronize()
        for (l0, v0), (l1, v1) in zip(first, again):
            assert l0.tolist() == l1.tolist() and np.array_equal(v0, v1)
    plan.close()
    for i, p in enumerate(params):
        single = sft.Plan(p)
        l1, v1 = single.iterative(xs[i]).host()
        single.close()
        assert first[i][0].tolist() == l1.tolist() and np.array_equal(first[i][1], v1)


@pytest.mark.parametrize("fft64", [True, False])
def test_iterative_full_batch_against_oracle(torch, sft, fft64):
    """The timed workload (N = 2^20, K = 1000, M_0 = 4096, a_m = 4, unit
    amplitudes, complex64) as one batch of 256 signals, every signal compared
    with the FP64 oracle (FP64 FFTs, complex64 thresholds).

    With SFT_FLAG_FFT64 the syndromes are FP64 and every output equals the
    oracle's: same support, values within 1e-9.  With FP32 FFTs every
    location that differs from the oracle's (returned by one side only) must
    lie in a residue class mod M_3 that holds an FP32-fragile location of the
    oracle's run (with the Appendix's closed-form roots or, where those lose a
    tight cluster, with eigenvalue roots), or the device must return there a
    superset of the oracle's locations, all true (iterative_vs_fp64); at most
    2 classes per signal."""
    n, k, m0, B = 1 << 20, 1000, 4096, 256
    say(f"[iter batch] B={B} fft64={fft64}")
    base = sftgen.BASE_SEED + 9000
    sigs = [sftgen.make_signal(n, k, base + i, amp="unit", dtype=np.complex64) for i in range(B)]
    flags = sft.SFT_FLAG_FFT64 if fft64 else 0
    plan = sft.Plan([dict(n=n, k=k, m=m0, l=4, dtype="c64", mode="iterative", flags=flags)] * B)
    outs = plan.batch([to_dev(torch, s.x) for s in sigs], stats=True)
    hits, differing = 0, 0
    for i, (o, s) in enumerate(zip(outs, sigs)):
        loc, val = o.host()
        hits += len(set(loc.tolist()) & set(s.locs.tolist()))
        if fft64:
            ref, _ = oit.sfft_iterative(s.x, n, m0, 4)
            assert loc.tolist() == ref.locs.tolist(), i
            assert np.max(np.abs(val - ref.vals)) <= 1e-9 * max(1.0, np.max(np.abs(ref.vals))), i
        else:
            _, nc = iterative_vs_fp64(loc, s.x, n, m0, 4, truth=(s.locs, s.vals),
                                      say=lambda *a: say(f"  signal {i}:", *a))
            differing += nc > 0
    plan.close()
    say(f"[iter batch] support recovery {hits / (B * k):.6f}, signals differing from the FP64 oracle {differing}")
    assert hits / (B * k) >= 0.995
