"""Train the learned order predictor on bins the method itself generates.

Training set: signals of length N = 2^20 with K = 1000 complex Gaussian tones,
SNR cycling over {exact, 10, 20, 30, 40} dB, complex64; the features of every
active bin of an exact-mode plan (M = 4096, L = 4) with the label = number of
true tones in the bin, clipped to 4.  About 4M bins from 1200 signals.
Training uses the library's own forward/backward and Adam kernels.

    python -m paper_1407_8315_amd.train_order_mlp --out weights.npy --report report.json

Evaluation: held-out signals per SNR, accuracy of the predictor.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def build_set(torch, sft, sftgen, seeds, snrs, n=1 << 20, k=1000, m=4096):
    import numpy as np

    plan = sft.Plan(dict(n=n, k=k, m=m, l=4))
    feats, labels, tags = [], [], []
    for i, seed in enumerate(seeds):
        snr = snrs[i % len(snrs)]
        x, locs, _ = sftgen.torch_signal(n, k, seed, torch.device("cuda"), amp="gauss", snr_db=snr)
        f, b = plan.features(x)
        counts = np.bincount(locs % m, minlength=m)
        feats.append(f.clone())
        labels.append(np.minimum(counts[b.cpu().numpy()], 4).astype(np.int32))
        tags.append(np.full(len(labels[-1]), -1 if snr is None else snr, np.int32))
    plan.close()
    return (torch.cat(feats), torch.from_numpy(np.concatenate(labels)).cuda(), np.concatenate(tags))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--signals", type=int, default=1200)
    ap.add_argument("--test-signals", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", required=True)
    ap.add_argument("--report", default=None)
    a = ap.parse_args()

    import numpy as np
    import torch

    import sftgen
    import paper_1407_8315_amd as sft

    snrs = [None, 10, 20, 30, 40]
    t0 = time.time()
    x_tr, y_tr, _ = build_set(torch, sft, sftgen, [sftgen.BASE_SEED + 100000 + i for i in range(a.signals)], snrs)
    t_data = time.time() - t0
    print(f"training set: {x_tr.shape[0]} bins from {a.signals} signals in {t_data:.1f} s; classes "
          f"{np.bincount(y_tr.cpu().numpy(), minlength=5).tolist()}", flush=True)
    net = sft.Mlp(seed=a.seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(a.seed)
    steps_per_epoch = max(1, x_tr.shape[0] // a.batch)
    total = steps_per_epoch * a.epochs
    t1 = time.time()
    hist = []
    for step in range(total):
        lr = a.lr * (0.1 ** (step / max(1, total - 1)))          # exponential decay to lr / 10
        idx = torch.randint(0, x_tr.shape[0], (a.batch,), device="cuda", generator=gen)
        net.train_step(x_tr[idx].contiguous(), y_tr[idx].contiguous(), lr, loss)
        if step % steps_per_epoch == 0 or step == total - 1:
            hist.append(round(float(loss.item()), 5))
            print(f"step {step}/{total} loss {hist[-1]}", flush=True)
    torch.cuda.synchronize()
    t_train = time.time() - t1

    # held-out evaluation, per SNR
    report = {"train_bins": int(x_tr.shape[0]), "train_signals": a.signals, "epochs": a.epochs,
              "steps": total, "batch": a.batch, "data_s": round(t_data, 1), "train_s": round(t_train, 1),
              "loss_history": hist, "accuracy": {}}
    del x_tr, y_tr
    for snr in snrs:
        seeds = [sftgen.BASE_SEED + 900000 + 10 * i + (0 if snr is None else snr) for i in range(a.test_signals // 4)]
        x_te, y_te, _ = build_set(torch, sft, sftgen, seeds, [snr])
        pred = net.forward(x_te).argmax(1)
        acc = float((pred == y_te.long()).float().mean().item())
        report["accuracy"]["exact" if snr is None else f"{snr}dB"] = round(acc, 5)
        print(f"held-out {snr} dB accuracy {acc:.4f} over {x_te.shape[0]} bins", flush=True)
    net.save(a.out)
    if a.report:
        with open(a.report, "w") as f:
            json.dump(report, f, indent=1)
    print(json.dumps(report))


if __name__ == "__main__":
    main()
