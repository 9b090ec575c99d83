"""GPU parity and training of the learned order predictor, through the C ABI."""
import sys
import time

import numpy as np
import pytest

import oracle
import sftgen
from oracle import mlp as omlp

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


def test_forward_matches_reference(torch, sft):
    """Logits of 300 random rows (4 full tiles and a ragged one) against the
    FP64 network with the device's BF16 rounding points."""
    say("[mlp forward]")
    g = np.random.default_rng(0)
    net = sft.Mlp(seed=5)
    theta = net.get_params().astype(np.float64)
    theta[omlp.unpack(np.arange(omlp.NPARAMS))["b1"].astype(int)] = g.standard_normal(128) * 0.1
    net.set_params(theta)
    x = g.standard_normal((300, 32)).astype(np.float32)
    got = net.forward(to_dev(torch, x)).cpu().numpy()
    ref, _ = omlp.forward(net.get_params(), x, bf16=True)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say(f"  max rel err {err:.2e}")
    assert err < 2e-3
    net.close()


def test_gradient_matches_reference(torch, sft):
    """Gradient of the mean cross-entropy against the FP64 reference gradient
    with the device's BF16 rounding points (weights, inputs and hidden
    activations in the forward pass; dZ3 for dH2 and dW3, dZ2 and dZ1 in the
    backward pass), entry by entry: |g - g_ref| <= 1e-3 max|g_ref| + 1e-2
    |g_ref| within each parameter block.  An FP32 emulation of the device's
    arithmetic stays within 2e-5 max|g_ref| of this reference (FP32
    accumulation, the polynomial erf and rare BF16 rounding flips of the
    activations make the rest)."""
    say("[mlp grad]")
    g = np.random.default_rng(1)
    net = sft.Mlp(seed=6)
    theta = net.get_params().astype(np.float64)
    for name in ("b1", "b2", "b3"):   # non-zero biases, so that every term of the gradient is exercised
        idx = omlp.unpack(np.arange(omlp.NPARAMS))[name].astype(int)
        theta[idx] = g.standard_normal(len(idx)) * 0.1
    net.set_params(theta)
    x = g.standard_normal((257, 32)).astype(np.float32)   # 4 full tiles of 64 rows and a ragged one
    y = g.integers(0, 5, 257).astype(np.int32)
    gd, loss = net.grad(to_dev(torch, x), to_dev(torch, y))
    gd = gd.cpu().numpy().astype(np.float64)
    ref_loss, ref = omlp.loss_and_grad(net.get_params(), x, y, bf16=True, bf16_backward=True)
    assert abs(float(loss.item()) - ref_loss) < 1e-4 * ref_loss
    for name, part_g in omlp.unpack(gd).items():
        part_r = omlp.unpack(ref)[name]
        scale = np.max(np.abs(part_r))
        err = np.abs(part_g - part_r)
        bound = 1e-3 * scale + 1e-2 * np.abs(part_r)
        worst = float(np.max(err / bound))
        say(f"  {name}: max |g - g_ref| / max|g_ref| {np.max(err) / scale:.2e}, worst error / bound {worst:.3f}")
        assert scale > 0
        assert np.all(err <= bound), (name, int(np.sum(err > bound)))
    net.close()


def _dataset(torch, sft, seeds, snrs):
    """Features of active bins (exact-mode plan, N = 2^20, K = 1000, M = 4096)
    with labels = true number of tones in the bin, clipped to 4."""
    n, k, m = 1 << 20, 1000, 4096
    plan = sft.Plan(dict(n=n, k=k, m=m, l=4))
    feats, labels = [], []
    for i, seed in enumerate(seeds):
        s = sftgen.make_signal(n, k, seed, amp="gauss", dtype=np.complex64, snr_db=snrs[i % len(snrs)])
        f, b = plan.features(to_dev(torch, s.x))
        counts = np.bincount(s.locs % m, minlength=m)
        feats.append(f.clone())
        labels.append(np.minimum(counts[b.cpu().numpy()], 4))
    plan.close()
    return torch.cat(feats), to_dev(torch, np.concatenate(labels).astype(np.int32))


def test_features_match_reference(torch, sft):
    say("[features]")
    n, k, m = 1 << 20, 1000, 4096
    s = sftgen.make_signal(n, k, 11, amp="gauss", dtype=np.complex64)
    plan = sft.Plan(dict(n=n, k=k, m=m, l=4))
    f, b = plan.features(to_dev(torch, s.x))
    f, b = f.cpu().numpy(), b.cpu().numpy()
    plan.close()
    ms = oracle.syndromes(s.x, n, m, range(8))
    e = np.sum(np.abs(ms) ** 2, axis=0)
    e_ref = float(np.mean(e))
    ref = oracle.sfft_exact(s.x, n, m, 4)
    assert len(b) == ref.active_bins
    l = np.arange(8)
    for row in range(0, len(b), 37):
        kk = int(b[row])
        mt = ms[:, kk] * np.exp(-2j * np.pi * ((kk * l) % n) / n)
        assert np.max(np.abs(f[row] - omlp.features(mt, e_ref))) < 2e-4


def test_training_and_learned_decode(torch, sft):
    """Train on bins the method generates (mixed SNR, exact included), then
    decode held-out exact signals with the predictor: same output as the plain
    decoder, high first-try acceptance, and the decode-stage time of both."""
    say("[train] data")
    seeds = [sftgen.BASE_SEED + 5000 + i for i in range(24)]
    x_tr, y_tr = _dataset(torch, sft, seeds, [None, 40, 30, 20, 10, None])
    say(f"  {x_tr.shape[0]} bins, class counts {np.bincount(y_tr.cpu().numpy(), minlength=5).tolist()}")
    net = sft.Mlp(seed=1)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    losses = []
    for step in range(600):
        idx = torch.randint(0, x_tr.shape[0], (4096,), device="cuda", generator=gen)
        net.train_step(x_tr[idx].contiguous(), y_tr[idx].contiguous(), 2e-3, loss)
        if step % 100 == 0 or step == 599:
            losses.append(float(loss.item()))
    say(f"  losses {np.round(losses, 4).tolist()}")
    assert losses[-1] < 0.5 * losses[0]
    # held-out exact signals
    n, k, m = 1 << 20, 1000, 4096
    x_te, y_te = _dataset(torch, sft, [sftgen.BASE_SEED + 9000 + i for i in range(4)], [None])
    pred = net.forward(x_te).argmax(1)
    acc = float((pred == y_te.long()).float().mean().item())
    say(f"  held-out exact accuracy {acc:.4f}")
    assert acc > 0.95
    plain = sft.Plan(dict(n=n, k=k, m=m, l=4))
    learned = sft.Plan(dict(n=n, k=k, m=m, l=4, flags=sft.SFT_FLAG_LEARNED))
    learned.attach(net)
    t_plain, t_learned, fb, act = 0.0, 0.0, 0, 0
    for i in range(4):
        s = sftgen.make_signal(n, k, sftgen.BASE_SEED + 9000 + i, amp="gauss", dtype=np.complex64)
        x = to_dev(torch, s.x)
        rp = plain.exact(x, stats=True)
        rl = learned.exact(x, stats=True)
        lp, vp = rp.host()
        ll, vl = rl.host()
        assert lp.tolist() == ll.tolist()
        assert np.max(np.abs(vp - vl)) <= 1e-12 * np.max(np.abs(vp))
        t_plain += sum(rp.stats["stage_ms"][1:3])
        t_learned += sum(rl.stats["stage_ms"][1:3])
        fb += rl.stats["mlp_fallbacks"]
        act += rl.stats["active_bins"]
    say(f"  fallbacks {fb}/{act}; order+decode ms plain {t_plain:.3f} learned {t_learned:.3f}")
    assert fb <= 0.05 * act
    plain.close()
    learned.close()
    net.close()


@pytest.mark.parametrize("kind", ["random", "always4", "always0"])
def test_sabotaged_weights_change_nothing(torch, sft, kind):
    """The predictor only orders the hypotheses: with untrained weights, or
    weights that predict one class for every bin, a learned plan returns the
    plain plan's output bit for bit (the rank test is the fallback and the
    residual check the judge, reading R24), with the fallbacks counted."""
    n, k, m = 1 << 20, 1000, 4096
    say(f"[sabotaged] {kind}")
    net = sft.Mlp(seed=123)
    if kind != "random":
        theta = np.zeros(omlp.NPARAMS)
        b3 = omlp.unpack(np.arange(omlp.NPARAMS))["b3"].astype(int)
        theta[b3[4 if kind == "always4" else 0]] = 10.0
        net.set_params(theta)
    plain = sft.Plan(dict(n=n, k=k, m=m, l=4))
    learned = sft.Plan(dict(n=n, k=k, m=m, l=4, flags=sft.SFT_FLAG_LEARNED))
    learned.attach(net)
    for seed in range(2):
        s = sftgen.make_signal(n, k, sftgen.BASE_SEED + 7700 + seed, amp="gauss", dtype=np.complex64)
        x = to_dev(torch, s.x)
        rp = plain.exact(x, stats=True)
        rl = learned.exact(x, stats=True)
        lp, vp = rp.host()
        ll, vl = rl.host()
        say(f"  seed {seed}: fallbacks {rl.stats['mlp_fallbacks']} of {rl.stats['active_bins']} active bins")
        assert ll.tolist() == lp.tolist()
        assert np.array_equal(vl, vp)
        assert rl.stats["flagged_bins"] == rp.stats["flagged_bins"]
        if kind != "always0":   # class 0 gives no order: such bins go straight to the rank test
            assert rl.stats["mlp_fallbacks"] > 0
    plain.close()
    learned.close()
    net.close()
