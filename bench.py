"""Throughput of the sFFT-DT path on one MI355X.

Workload (default): generally K-sparse signals, N = 2^20, K = 1000 complex
Gaussian tones plus white spectral noise, SNR cycling over 10/20/30/40 dB
across the batch, complex64 input; M = 4096, L = 4, R = 12 random shifts;
B = 1024 signals resident in HBM, one sft_batch call per step (HIP graph).

Metric: recovered frequencies per second (true-support entries found, summed
over the batch, divided by the step time), with signals/s beside it.

Two timed regions on the plan's stream:
  1. K graph-replayed steps bracketed by synchronisation -> value, ms/step;
  2. K steps with per-stage HIP events (same kernels and launch shapes, not
     graph-replayed) -> average duration of each stage, and of the dominant
     kernel of the gather+FFT stage on its own, from which the roofline
     figures are computed.
The oracle (FP64 numpy, one host thread) is timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector, published
BF16_PEAK_TFLOPS = 2500.0      # MI355X dense BF16 MFMA, published

# HBM bytes of the dominant gather + FFT kernel per algorithmic byte read and
# written (fetched, written), from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by
# the plain-copy calibration (profiles/syndrome_kernel_random_shifts_general_n20_b1024_traffic.md,
# profiles/pair_syndrome_kernel_exact_n20_b1024_traffic.md,
# profiles/iter_pair_kernel_iterative_n20_b1024_traffic.md).  A kernel
# changed since its counters were taken gets no entry (its traffic is null).
TRAFFIC_RATIOS = {"general": (12.50, 1.00), "exact": (2.05, 1.18), "iterative": (6.09, 1.00)}

# Algorithmic FLOPs of the order predictor per row (matrix products only):
# forward 2 (32*128 + 128*128 + 128*5); training adds the three weight
# gradients and the two hidden-layer input gradients.
MLP_FWD_FLOP = 2 * (32 * 128 + 128 * 128 + 128 * 5)
MLP_TRAIN_FLOP = MLP_FWD_FLOP + 2 * (32 * 128 + 128 * 128 + 128 * 5 + 128 * 5 + 128 * 128)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--mode", choices=["general", "exact", "iterative"], default="general")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of each leg of the oracle sample")
    ap.add_argument("--parity-signals", type=int, default=32,
                    help="signals of the timed batch compared with the FP64 oracle (0: none)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for counter calibration)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain comparison")
    ap.add_argument("--no-uneven", action="store_true", help="skip the batched uneven workload")
    ap.add_argument("--no-iterative", action="store_true", help="skip the iterative-vs-non-iterative comparison")
    ap.add_argument("--fft64", action="store_true", help="FP64 FFTs for the complex64 input (SFT_FLAG_FFT64)")
    ap.add_argument("--no-model", action="store_true", help="skip the recovery-vs-collision-model section")
    ap.add_argument("--no-large", action="store_true", help="skip the N = 2^24 section")
    ap.add_argument("--only-large", type=int, choices=[10, 12, 14], default=None, metavar="LOG2K",
                    help="run only the N = 2^24 section at K = 2^LOG2K and print it (for profiling)")
    ap.add_argument("--paper-tables", action="store_true",
                    help="also run Alg. 2 as printed on the Tables II-IV workload (N = 2^24, mixture Gaussian)")
    return ap.parse_args()


WEIGHTS = os.path.join(ROOT, "paper_1407_8315_amd", "data", "order_mlp.npy")


def learned_vs_plain(steps, warmup, B=1024):
    """Exact-input batch (N = 2^20, K = 1000, M = 4096, L = 4), plain rank-test
    order estimate against the learned predictor (trained weights shipped in
    paper_1407_8315_amd/data), same signals, graph-replayed steps."""
    import numpy as np
    import torch

    import sftgen
    from paper_1407_8315_amd import SFT_FLAG_LEARNED, Mlp, Plan

    if not os.path.exists(WEIGHTS):
        return None
    n, k, m, L = 1 << 20, 1000, 4096, 4
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    out = {}
    with torch.cuda.stream(stream):
        xs, truth = [], []
        for i in range(B):
            x, locs, _ = sftgen.torch_signal(n, k, sftgen.BASE_SEED + 20000 + i, dev, amp="unit")
            xs.append(x)
            truth.append(locs)
        net = Mlp(seed=0, stream=stream)
        net.load(WEIGHTS)
        for name, flags in (("plain", 0), ("learned", SFT_FLAG_LEARNED)):
            plan = Plan([dict(n=n, k=k, m=m, l=L, flags=flags)] * B, stream=stream)
            if flags:
                plan.attach(net)
            outs = [plan.new_output(m * L, dev) for _ in range(B)]
            run = plan.prepare_batch(xs, outs)
            for _ in range(warmup):
                run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                run()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            found = sum(len(np.intersect1d(o.loc[:int(o.count.item())].cpu().numpy(), t)) for o, t in zip(outs, truth))
            st = run(stats=True)
            out[name] = {"ms_per_step": round(ms, 4), "signals_per_s": round(B / ms * 1e3, 1),
                         "freqs_per_s": round(found / ms * 1e3, 1), "support_recovery": round(found / (B * k), 5),
                         "stage_ms": [round(v, 4) for v in st["stage_ms"]], "mlp_fallbacks": st["mlp_fallbacks"],
                         "active_bins": st["active_bins"]}
            plan.close()
        net.close()
    out["speedup_learned_over_plain"] = round(out["plain"]["ms_per_step"] / out["learned"]["ms_per_step"], 4)
    out["workload"] = f"exact, N=2^20, K=1000, M=4096, L=4, unit amplitudes, complex64, batch {B}"
    return out


def iterative_vs_non_iterative(steps, warmup, B=1024):
    """Exactly K-sparse batch (N = 2^20, K = 1000, unit amplitudes, complex64):
    non-iterative sFFT-DT (M = 4096, L = 4: 8 FFTs of 4096 points) against
    iterative sFFT-DT (Alg. 1, M_0 = 4096, a_m = 4: FFTs of 2 x 4096, 2 x 2048,
    2 x 1024, 2 x 512 points) with FP32 and with FP64 FFTs, same signals,
    graph-replayed steps."""
    import numpy as np
    import torch

    import sftgen
    from paper_1407_8315_amd import SFT_FLAG_FFT64, Plan

    n, k, m, L = 1 << 20, 1000, 4096, 4
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    out = {}
    with torch.cuda.stream(stream):
        xs, truth = [], []
        for i in range(B):
            x, locs, _ = sftgen.torch_signal(n, k, sftgen.BASE_SEED + 40000 + i, dev, amp="unit")
            xs.append(x)
            truth.append(locs)
        for name, mode, flags in (("non_iterative", "exact", 0), ("iterative", "iterative", 0),
                                  ("iterative_fft64", "iterative", SFT_FLAG_FFT64)):
            plan = Plan([dict(n=n, k=k, m=m, l=L, mode=mode, flags=flags)] * B, stream=stream)
            outs = [plan.new_output(m * L, dev) for _ in range(B)]
            run = plan.prepare_batch(xs, outs)
            for _ in range(warmup):
                run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                run()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            found = sum(len(np.intersect1d(o.loc[:int(o.count.item())].cpu().numpy(), t)) for o, t in zip(outs, truth))
            st = run(stats=True)
            out[name] = {"ms_per_step": round(ms, 4), "signals_per_s": round(B / ms * 1e3, 1),
                         "freqs_per_s": round(found / ms * 1e3, 1), "support_recovery": round(found / (B * k), 5),
                         "stage_ms": [round(v, 4) for v in st["stage_ms"]], "active_bins": st["active_bins"],
                         "flagged_bins": st["flagged_bins"]}
            plan.close()
    out["speedup_iterative_over_non_iterative"] = round(out["non_iterative"]["ms_per_step"]
                                                        / out["iterative"]["ms_per_step"], 4)
    out["speedup_iterative_fft64_over_non_iterative"] = round(out["non_iterative"]["ms_per_step"]
                                                              / out["iterative_fft64"]["ms_per_step"], 4)
    out["workload"] = f"exact, N=2^20, K=1000, M(_0)=4096, L=a_m=4, unit amplitudes, complex64, batch {B}"
    out["stage_ms_meaning"] = {"non_iterative": "gather+FFT, activity+rank test, decode, output",
                               "iterative": "gather+FFT (all iterations), iteration 0, iterations 1-3, output"}
    out["fft_precision"] = {"non_iterative": "fp32", "iterative": "fp32", "iterative_fft64": "fp64"}
    return out


def recovery_vs_model(B=256):
    """Support recovery measured on the device against the collision model
    (Sec. II-C, Lemma 2; the autotuner's model): a frequency is recovered when
    its bin holds at most L frequencies, so the expected recovery is the
    hypergeometric P(at most L - 1 of the other K - 1 frequencies fall in the
    d - 1 other slots of its bin).  N = 2^20, K = 1000, N+ = N/(dK) from 1 to
    8, L = 1..4, B signals each, FP64 FFTs (so no FP32 effect enters).  Also
    the fraction of signals with a missed frequency against Lemma 2's bound
    (N/d) (d e K / (N (L + 1)))^(L + 1)."""
    import numpy as np
    import torch
    from scipy.stats import hypergeom

    import sftgen
    from paper_1407_8315_amd import SFT_FLAG_FFT64, Plan

    n, k = 1 << 20, 1000
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    rows = []
    with torch.cuda.stream(stream):
        xs, truth = [], []
        for i in range(B):
            x, locs, _ = sftgen.torch_signal(n, k, sftgen.BASE_SEED + 50000 + i, dev, amp="unit")
            xs.append(x)
            truth.append(locs)
        for m in (1024, 2048, 4096, 8192):
            d = n // m
            for L in (1, 2, 3, 4):
                if d < 2 * L:
                    continue
                plan = Plan([dict(n=n, k=k, m=m, l=L, flags=SFT_FLAG_FFT64)] * B, stream=stream)
                outs = plan.batch(xs)
                torch.cuda.synchronize()
                found, imperfect = 0, 0
                for o, t in zip(outs, truth):
                    got = len(np.intersect1d(o.host()[0], t))
                    found += got
                    imperfect += got < k
                plan.close()
                model = float(hypergeom.cdf(L - 1, n - 1, d - 1, k - 1))
                lemma2 = (n / d) * (d * math.e * k / (n * (L + 1))) ** (L + 1)
                rows.append({"m": m, "n_plus": round(m / k, 3), "l": L,
                             "measured_recovery": round(found / (B * k), 6), "model_recovery": round(model, 6),
                             "signals_with_a_miss": round(imperfect / B, 4), "lemma2_bound": round(min(1.0, lemma2), 6)})
        del xs
        # Fig. 4 (non-iterative): recovery against K at d = N/(4K), a_m = 4
        fig4 = []
        for lk in (6, 8, 10, 12, 14):
            kk, B4 = 1 << lk, 64
            m = 4 * kk
            d = n // m
            xs, truth = [], []
            for i in range(B4):
                x, locs, _ = sftgen.torch_signal(n, kk, sftgen.BASE_SEED + 51000 + 100 * lk + i, dev, amp="unit")
                xs.append(x)
                truth.append(locs)
            plan = Plan([dict(n=n, k=kk, m=m, l=4, flags=SFT_FLAG_FFT64)] * B4, stream=stream)
            outs = plan.batch(xs)
            torch.cuda.synchronize()
            found = sum(len(np.intersect1d(o.host()[0], t)) for o, t in zip(outs, truth))
            plan.close()
            model = float(hypergeom.cdf(3, n - 1, d - 1, kk - 1))
            fig4.append({"log2_k": lk, "m": m, "d": d, "measured_recovery": round(found / (B4 * kk), 6),
                         "model_recovery": round(model, 6), "signals": B4})
            del xs
    return {"workload": f"exact, N=2^20, K=1000, unit amplitudes, complex64 with FP64 FFTs, {B} signals per cell",
            "rows": rows,
            "fig4_workload": "exact, N=2^20, d=N/(4K) (M=4K), L=a_m=4, unit amplitudes, FP64 FFTs, 64 signals per K",
            "fig4_rows": fig4}


def paper_tables(reps=3, log2_ks=range(8, 17)):
    """Alg. 2 as printed (SFT_FLAG_SP_ALL) on the workload of Tables II-IV:
    N = 2^24, d = N/(32K), a_m = 3, R = 9, mixture-Gaussian x_hat (Eq. (21))
    at SNR(x_hat_s) = 30, 20, 10 dB, K = the significant entries drawn.
    Per cell: SNR(x_hat_out) and the device time of one call (mean of reps,
    HIP events), next to the paper's printed values (CPU seconds)."""
    import json as _json

    import torch

    import sftgen
    from paper_1407_8315_amd import SFT_FLAG_SP_ALL, Plan

    gold = _json.load(open(os.path.join(ROOT, "tests", "golden", "tables_2_4.json")))
    n = 1 << 24
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    rows = []
    with torch.cuda.stream(stream):
        for snr in (30, 20, 10):
            for lk in log2_ks:
                k_nom = 1 << lk
                m = 32 * k_nom
                x, xh, k = sftgen.torch_mixture(n, k_nom, snr, sftgen.BASE_SEED + 70000 + 100 * snr + lk, dev)
                plan = Plan(dict(n=n, k=k, m=m, l=3, r=min(9, n // m), mode="general", seed=lk,
                                 flags=SFT_FLAG_SP_ALL), stream=stream)
                out = plan.new_output(m * 3, dev)
                plan.general(x, out)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    plan.general(x, out)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                cnt = min(int(out.count.item()), out.loc.numel())
                loc, val = out.loc[:cnt], out.val[:cnt]
                err = float((xh.abs() ** 2).sum() + ((xh[loc] - val).abs() ** 2).sum() - (xh[loc].abs() ** 2).sum())
                snr_out = 10.0 * math.log10(float((val.abs() ** 2).sum()) / max(err, 1e-300))
                i = gold["log2_k"].index(lk)
                print(f"[paper tables] snr {snr} dB, K = 2^{lk}: SNR_out {snr_out:.2f} dB, {ms:.3f} ms",
                      file=sys.stderr, flush=True)
                rows.append({"snr_in_db": snr, "log2_k": lk, "k_drawn": k, "m": m,
                             "snr_out_db": round(snr_out, 2), "ms_per_call": round(ms, 3),
                             "paper_snr_out_db": gold["snr_out_with_pruning"][str(snr)][i],
                             "paper_seconds": gold["seconds_with_pruning"][str(snr)][i]})
                plan.close()
                del x, xh, out
                torch.cuda.empty_cache()
    return {"workload": "Alg. 2 as printed, N=2^24, d=N/(32K), a_m=3, R=9, mixture Gaussian, complex64",
            "rows": rows}


def uneven_batch(steps, warmup, count=4096):
    """The batched uneven workload: `count` exact signals with N = 2^e, e
    uniform on 14..22, K = round(2^u), u uniform on [4, 12], K <= N/64, unit
    magnitude, complex64, M and L chosen per signal by the autotuner, one plan
    (graph-replayed sft_batch calls)."""
    import numpy as np
    import torch

    import sftgen
    from paper_1407_8315_amd import SFT_FLAG_AUTOTUNE, Plan, autotune

    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    ns, ks = sftgen.uneven_batch_params(count)
    t0 = time.time()
    with torch.cuda.stream(stream):
        xs, truth = [], []
        for i, (n, k) in enumerate(zip(ns.tolist(), ks.tolist())):
            x, locs, _ = sftgen.torch_signal(n, k, sftgen.BASE_SEED + 40000 + i, dev, amp="unit")
            xs.append(x)
            truth.append(locs)
        torch.cuda.synchronize()
        t_gen = time.time() - t0
        t1 = time.time()
        plan = Plan([dict(n=n, k=k, flags=SFT_FLAG_AUTOTUNE) for n, k in zip(ns.tolist(), ks.tolist())],
                    stream=stream)
        t_plan = time.time() - t1
        caps = [inf["m"] * inf["l"] for inf in plan.infos]
        outs = [plan.new_output(c, dev) for c in caps]
        run = plan.prepare_batch(xs, outs, caps)
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        found = 0
        for o, t in zip(outs, truth):
            found += len(np.intersect1d(o.loc[:int(o.count.item())].cpu().numpy(), t))
        st = run(stats=True)
        tune = [autotune(n, k) for n, k in zip(ns.tolist(), ks.tolist())]
        ms_choices = sorted({(inf["m"], inf["l"]) for inf in plan.infos})
        plan.close()
    total_k = int(ks.sum())
    return {"workload": f"exact, {count} signals, N = 2^14..2^22 log-uniform, K = 16..4096 log-uniform (K <= N/64), "
                        "unit amplitudes, complex64, M and L autotuned per signal",
            "ms_per_step": round(ms, 4), "signals_per_s": round(count / ms * 1e3, 1),
            "freqs_per_s": round(found / ms * 1e3, 1), "support_recovery": round(found / total_k, 6),
            "expected_recovery": round(sum(k * r[2] for k, r in zip(ks.tolist(), tune)) / total_k, 6),
            "model_ms": round(sum(r[3] for r in tune) / 1e3, 4), "distinct_m_l": len(ms_choices),
            "input_gb": round(float(ns.sum()) * 8 / 1e9, 2), "sum_k": total_k,
            "stage_ms": [round(v, 4) for v in st["stage_ms"]], "plan_s": round(t_plan, 2),
            "input_generation_s": round(t_gen, 1)}


def large_scale(steps, warmup, batches=((10, 256), (12, 64), (14, 32))):
    """N = 2^24 with K in {2^10, 2^12, 2^14} and M = 4K, L = 4, complex64
    (unit amplitudes): per K, a batch of B exact signals (B = 256, 64, 32:
    enough blocks to fill the device at every M) decoded with the
    plain rank test and with the learned order (graph-replayed sft_batch
    calls), and a batch of B general-mode signals at 20 dB.  The gather + FFT
    stage's algorithmic bandwidth comes from the per-stage events (every
    gathered sample read once, every syndrome written once)."""
    import numpy as np
    import torch

    import sftgen
    from paper_1407_8315_amd import SFT_FLAG_LEARNED, Mlp, Plan

    n, L = 1 << 24, 4
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    rows = []
    with torch.cuda.stream(stream):
        net = None
        if os.path.exists(WEIGHTS):
            net = Mlp(seed=0, stream=stream)
            net.load(WEIGHTS)
        for lk, B in batches:
            k = 1 << lk
            m = 4 * k
            for variant in ("exact", "general_20db"):
                xs, truth = [], []
                for i in range(B):
                    x, locs, _ = sftgen.torch_signal(n, k, sftgen.BASE_SEED + 80000 + 100 * lk + i, dev, amp="unit",
                                                     snr_db=20 if variant != "exact" else None)
                    xs.append(x)
                    truth.append(locs)
                forms = [("plain", 0)] + ([("learned", SFT_FLAG_LEARNED)] if variant == "exact" and net else [])
                for form, flags in forms:
                    mode = "exact" if variant == "exact" else "general"
                    plan = Plan([dict(n=n, k=k, m=m, l=L, mode=mode, seed=lk, flags=flags)] * B, stream=stream)
                    if flags:
                        plan.attach(net)
                    outs = [plan.new_output(m * L, dev) for _ in range(B)]
                    run = plan.prepare_batch(xs, outs)
                    for _ in range(warmup):
                        run()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(steps):
                        run()
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / steps
                    found = sum(len(np.intersect1d(o.loc[:min(int(o.count.item()), o.loc.numel())].cpu().numpy(), t))
                                for o, t in zip(outs, truth))
                    st = run(stats=True)
                    lines = 2 * L + (plan.infos[0]["r"] if mode == "general" else 0)
                    stage_gbs = B * lines * m * 8 * 2 / (st["stage_ms"][0] * 1e-3) / 1e9
                    rows.append({"log2_k": lk, "m": m, "variant": variant, "form": form, "signals": B,
                                 "ms_per_step": round(ms, 4), "signals_per_s": round(B / ms * 1e3, 1),
                                 "freqs_per_s": round(found / ms * 1e3, 1),
                                 "support_recovery": round(found / (B * k), 6),
                                 "stage_ms": [round(v, 4) for v in st["stage_ms"]],
                                 "gather_fft_algorithmic_gbs": round(stage_gbs, 1),
                                 "gather_fft_frac_of_hbm_peak": round(stage_gbs / HBM_PEAK_GBS, 4),
                                 "mlp_fallbacks": st["mlp_fallbacks"], "active_bins": st["active_bins"]})
                    plan.close()
                del xs
                torch.cuda.empty_cache()
        if net:
            net.close()
    for lk in (10, 12, 14):
        p = [r for r in rows if r["log2_k"] == lk and r["variant"] == "exact"]
        if len(p) == 2:
            p[1]["speedup_over_plain"] = round(p[0]["ms_per_step"] / p[1]["ms_per_step"], 4)
    return {"workload": "N=2^24, K=2^10/2^12/2^14, M=4K, L=4, unit amplitudes, complex64, batches of "
                        + "/".join(str(b) for _, b in batches) + "; exact (plain and learned) and general mode at 20 dB",
            "rows": rows}


def mlp_throughput(steps, warmup, rows=1 << 18):
    """The order predictor's kernels on `rows` random feature rows: forward
    (inference) and one Adam training step (forward + backward), each timed
    over `steps` calls, as rows/s and algorithmic TFLOP/s against the BF16
    MFMA peak."""
    import torch

    from paper_1407_8315_amd import Mlp

    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    out = {}
    with torch.cuda.stream(stream):
        g = torch.Generator(device=dev)
        g.manual_seed(5)
        feat = torch.randn((rows, 32), generator=g, device=dev)
        labels = torch.randint(0, 5, (rows,), generator=g, device=dev, dtype=torch.int32)
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        net = Mlp(seed=1, stream=stream)
        for name, fn, flop in (("inference", lambda: net.forward(feat), MLP_FWD_FLOP),
                               ("training", lambda: net.train_step(feat, labels, 1e-4, loss), MLP_TRAIN_FLOP)):
            for _ in range(warmup):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            tflops = rows * flop / (ms * 1e-3) / 1e12
            out[name] = {"ms_per_call": round(ms, 4), "rows_per_s": round(rows / ms * 1e3, 1),
                         "algorithmic_tflops": round(tflops, 2), "frac_of_bf16_peak": round(tflops / BF16_PEAK_TFLOPS, 5),
                         "flop_per_row": flop}
        net.close()
    out["rows"] = rows
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np

    n, k, m, L, R = 1 << 20, 1000, 4096, 4, 12
    snrs = [10, 20, 30, 40]
    cpu = None
    if not a.no_cpu and not a.copy_calibration and a.only_large is None:
        # on the host, before anything initialises the GPU
        cpu = cpu_baseline(n, k, m, L, R, a.mode, a.cpu_seconds, snrs)

    import torch

    import sftgen
    from paper_1407_8315_amd import Plan

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if a.only_large is not None:
        b = {10: 256, 12: 64, 14: 32}[a.only_large]
        print(json.dumps({"large_scale_n24": large_scale(a.steps, a.warmup, batches=((a.only_large, b),))}))
        return
    if a.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.complex64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 8, "launches": 5}))
        return

    B = a.batch
    mode = a.mode
    stream = torch.cuda.Stream(device=dev)
    xs, truth, tvals = [], [], []
    t0 = time.time()
    with torch.cuda.stream(stream):
        for i in range(B):
            snr = snrs[i % 4] if mode == "general" else None
            x, locs, vals = sftgen.torch_signal(n, k, sftgen.BASE_SEED + i, dev, amp="gauss", snr_db=snr)
            xs.append(x)
            truth.append(locs)
            tvals.append(vals)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    flags = 16 if a.fft64 else 0   # SFT_FLAG_FFT64
    params = [dict(n=n, k=k, m=m, l=L, r=R if mode == "general" else 0, mode=mode, seed=sftgen.BASE_SEED + i,
                   flags=flags) for i in range(B)]
    with torch.cuda.stream(stream):
        plan = Plan(params, stream=stream)
        caps = [m * L] * B
        outs = [plan.new_output(c, dev) for c in caps]
        run = plan.prepare_batch(xs, outs, caps)
        for _ in range(a.warmup):
            run()
        torch.cuda.synchronize()
        # ---- timed region 1: graph-replayed steps
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(a.steps):
            run()
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_step = ev0.elapsed_time(ev1) / a.steps
        # recovery of the last step
        found = 0
        for o, t in zip(outs, truth):
            cnt = int(o.count.item())
            loc = o.loc[:min(cnt, o.loc.numel())].cpu().numpy()
            found += len(np.intersect1d(loc, t))
        # ---- timed region 2: per-stage HIP events
        stage = np.zeros(4)
        gather = np.zeros(2)
        st = None
        for _ in range(a.steps):
            st = run(stats=True)
            stage += np.array(st["stage_ms"])
            gather += np.array(st["gather_ms"])
        stage /= a.steps
        gather /= a.steps
    signals_per_s = B / (ms_step * 1e-3)
    freqs_per_s = found / (ms_step * 1e-3)
    recovery = found / (B * k)

    # samples gathered (= syndromes written) per signal: 2L (+ R) lines of M;
    # iterative: two lines per iteration on grids of M, M/2, ...
    samples = 2 * sum(m >> l for l in range(L)) if mode == "iterative" else (2 * L + (R if mode == "general" else 0)) * m
    per_sample = 8 + (16 if a.fft64 else 8)                # gather read (complex64) + syndrome write
    stage_gbs = B * samples * per_sample / (stage[0] * 1e-3) / 1e9
    # the dominant kernel of the gather + FFT stage, timed on its own (HIP
    # events around it on the plan's stream): general mode the R random-shift
    # lines, exact mode the 2L consecutive shifts (one pair kernel per call);
    # iterative mode the whole stage (one kernel for every grid)
    if mode == "general":
        k_samples, k_ms = R * m, gather[1]
        k_name = f"syndrome_kernel<{'double' if a.fft64 else 'float'}, 4096, float> (gather + FFT of the R random shifts)"
    elif mode == "exact":
        k_samples, k_ms = 2 * L * m, gather[0]
        k_name = ("syndrome_kernel<double, 4096, float>" if a.fft64 else "pair_syndrome_kernel<1, 12, 3>") \
            + " (gather + FFT of the 2L consecutive shifts)"
    else:
        k_samples, k_ms = samples, stage[0]
        k_name = "iter_pair_kernel<12> (gather + FFT of every iteration's lines, one launch)"
    k_bytes = B * k_samples * per_sample
    k_gbs = k_bytes / (k_ms * 1e-3) / 1e9
    ratios = None if a.fft64 else TRAFFIC_RATIOS.get(mode)
    # measured HBM bytes per launch (fetch + write), when counters were taken for this kernel
    traffic = int(B * k_samples * 8 * (ratios[0] + ratios[1])) if ratios else None
    # the least HBM traffic the access pattern allows (128-byte lines): the
    # random shifts need one line per 8-byte sample; exact mode's 2L = 8
    # consecutive shifts one line per 64-byte run; the iterative grids the
    # lines of grid 0 (16 bytes used of each; the later grids' samples lie in
    # them); syndromes written once.  Its ratio to the algorithmic bytes bounds
    # `frac` at full HBM speed.
    if a.fft64:
        floor = None
    elif mode == "general":
        floor = B * k_samples * (128 + 8)
    elif mode == "exact":
        floor = B * m * (128 + 2 * L * 8)
    else:
        floor = B * m * 128 + B * samples * 8
    roofline = {"bound": "hbm", "achieved": round(k_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(k_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "pattern_floor_bytes": floor,
                "pattern_ceiling_frac": round(k_bytes / floor, 4) if floor else None,
                "traffic_gbs": round(traffic / (k_ms * 1e-3) / 1e9, 1) if traffic else None,
                "kernel": k_name, "algorithmic_bytes_per_launch": k_bytes, "avg_launch_ms": round(k_ms, 4),
                "stage": {"achieved": round(stage_gbs, 1), "frac": round(stage_gbs / HBM_PEAK_GBS, 4),
                          "algorithmic_bytes": B * samples * per_sample, "avg_ms": round(stage[0], 4)}}

    for i, o in enumerate(outs[:a.parity_signals]):
        o.truth = (truth[i], tvals[i])
    parity = parity_sample(mode, n, k, m, L, xs, outs, plan.infos, min(a.parity_signals, B)) \
        if a.parity_signals else None
    plan.close()
    del xs, outs
    torch.cuda.empty_cache()
    lvp = None if a.no_learned else learned_vs_plain(a.steps, a.warmup)
    torch.cuda.empty_cache()
    unv = None if a.no_uneven else uneven_batch(a.steps, a.warmup)
    torch.cuda.empty_cache()
    mlp = None if a.no_learned else mlp_throughput(a.steps, a.warmup)
    torch.cuda.empty_cache()
    itv = None if a.no_iterative else iterative_vs_non_iterative(a.steps, a.warmup)
    torch.cuda.empty_cache()
    tables = paper_tables() if a.paper_tables else None
    torch.cuda.empty_cache()
    large = None if a.no_large else large_scale(a.steps, a.warmup)
    torch.cuda.empty_cache()
    model = None if a.no_model else recovery_vs_model()
    out = {
        "metric": {"general": "recovered freqs/s at N=2^20, K=1000 (general mode, SNR 10/20/30/40 dB)",
                   "exact": "recovered freqs/s at N=2^20, K=1000 (exact mode)",
                   "iterative": "recovered freqs/s at N=2^20, K=1000 (exact mode, iterative Alg. 1)"}[mode],
        "value": round(freqs_per_s, 1), "unit": "freqs/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp64" if a.fft64 else "fp32 FFT / fp64 decode", "data": "synthetic",
        "config": {"workload": f"sFFT-DT {mode}, N=2^20, K=1000, M{'_0' if mode == 'iterative' else ''}=4096, L=4"
                   + (", R=12, SNR cycling 10/20/30/40 dB" if mode == "general" else "")
                   + f", complex64, batch {B}", "global_batch": B, "n": n, "k": k, "m": m, "l": L},
        "signals_per_s": round(signals_per_s, 1),
        "support_recovery": round(recovery, 5),
        "stage_ms": [round(v, 4) for v in stage],
        "gather_ms": [round(v, 4) for v in gather],
        "stats_last_step": {kk: v for kk, v in st.items() if kk not in ("stage_ms", "gather_ms")} if st else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "learned_vs_plain": lvp,
        "uneven_batch": unv,
        "mlp_kernels": mlp,
        "iterative_vs_non_iterative": itv,
        "paper_tables_2_4": tables,
        "large_scale_n24": large,
        "recovery_vs_model": model,
        "input_generation_s": round(gen_s, 2),
    }
    print(json.dumps(out))


def _host_cpu():
    """Model name, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def _oracle_task(args):
    """One signal of the CPU baseline: generate (untimed), run the FP64 oracle
    (timed, one thread).  Returns (frequencies recovered, oracle seconds)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    import sftgen
    from oracle import iterative as oracle_iterative

    n, k, m, L, R, mode, seed, snr = args
    with threadpool_limits(1):
        s = sftgen.make_signal(n, k, seed, amp="gauss", dtype=np.complex64, snr_db=snr)
        t0 = time.perf_counter()
        if mode == "general":
            d = n // m
            rsh = sorted(np.random.default_rng(seed).choice(d, R, replace=False).tolist())
            r = oracle.sfft_general(s.x, n, k, m, L, rsh)
        elif mode == "iterative":
            r, _ = oracle_iterative.sfft_iterative(s.x, n, m, L)
        else:
            r = oracle.sfft_exact(s.x, n, m, L)
        dt = time.perf_counter() - t0
    return len(np.intersect1d(r.locs, s.locs)), dt


def cpu_baseline(n, k, m, L, R, mode, budget_s, snrs):
    """The FP64 oracle on a bounded sample of the same workload (the batch's
    seeds and SNRs; general mode draws its R random shifts per signal), timed
    on the host before the GPU is touched: one thread, then one process per
    available CPU (at most 16) running signals side by side, each with one
    BLAS thread.  Signal generation is excluded from both."""
    import concurrent.futures
    import multiprocessing

    import sftgen

    def task(i):
        return (n, k, m, L, R, mode, sftgen.BASE_SEED + i, snrs[i % 4] if mode == "general" else None)

    found, t_tot, i = 0, 0.0, 0
    while t_tot < budget_s and i < 256:
        f, dt = _oracle_task(task(i))
        found += f
        t_tot += dt
        i += 1
    single = {"value": round(found / t_tot, 1), "unit": "freqs/s", "cores": 1, "signals": i,
              "signals_per_s": round(i / t_tot, 3), "oracle_seconds": round(t_tot, 1)}
    procs = max(1, min(16, _host_cpu()["affinity"]))
    ctx = multiprocessing.get_context("fork")
    found_p, t_sum, done = 0, 0.0, 0
    t0 = time.perf_counter()
    with concurrent.futures.ProcessPoolExecutor(max_workers=procs, mp_context=ctx) as ex:
        j = 0
        while time.perf_counter() - t0 < budget_s and j < 1024:
            batch = [task(j + q) for q in range(procs)]
            for f, dt in ex.map(_oracle_task, batch):
                found_p += f
                t_sum += dt
                done += 1
            j += procs
    # signals run side by side: the rate is procs x the mean per-process rate
    multi_value = found_p / t_sum * procs
    return {"value": round(multi_value, 1), "unit": "freqs/s", "cores": procs, "kind": "oracle",
            "sample": f"{mode} workload, first {done} signals of the batch's seeds in {procs} processes "
                      f"(one BLAS thread each, {t_sum:.1f} s of oracle time); single-thread leg: first {i} "
                      f"signals, {t_tot:.1f} s; signal generation excluded",
            "single_thread": single, "host": _host_cpu()}


def parity_sample(mode, n, k, m, L, xs, outs, infos, count):
    """The GPU's outputs of the timed batch against the FP64 oracle run on the
    same complex64 inputs, for the first `count` signals: exact and iterative
    mode, the locations returned by one side only and the largest relative
    amplitude error at common locations; general mode (an approximation,
    compared on metrics), support recovery and relative L2 error of both."""
    import numpy as np

    import oracle
    from oracle import iterative as oracle_iterative

    diff_locs, diff_sigs, max_rel = 0, 0, 0.0
    sr_g = sr_o = rl_g = rl_o = 0.0
    for i in range(count):
        x = xs[i].cpu().numpy()
        loc, val = outs[i].host()
        if mode == "general":
            r = oracle.sfft_general(x, n, k, m, L, infos[i]["rshifts"])
        elif mode == "iterative":
            r, _ = oracle_iterative.sfft_iterative(x, n, m, L)
        else:
            r = oracle.sfft_exact(x, n, m, L)
        d = len(set(loc.tolist()) ^ set(r.locs.tolist()))
        diff_locs += d
        diff_sigs += d > 0
        common, ia, ib = np.intersect1d(loc, r.locs, return_indices=True)
        if len(common):
            max_rel = max(max_rel, float(np.max(np.abs(val[ia] - r.vals[ib]) / np.abs(r.vals[ib]))))
        if mode == "general":
            t = outs[i].truth
            sr_g += oracle.support_recovery(t[0], loc) / count
            sr_o += oracle.support_recovery(t[0], r.locs) / count
            rl_g += oracle.relative_l2(t[0], t[1], loc, val) / count
            rl_o += oracle.relative_l2(t[0], t[1], r.locs, r.vals) / count
    out = {"signals": count, "reference": "FP64 oracle (FP64 FFTs, complex64 thresholds) on the same inputs",
           "locations_returned_by_one_side": diff_locs, "signals_with_a_difference": diff_sigs,
           "max_rel_amplitude_error_common": float(f"{max_rel:.3g}")}
    if mode == "general":
        out.update({"support_recovery_gpu": round(sr_g, 6), "support_recovery_oracle": round(sr_o, 6),
                    "rel_l2_gpu": round(rl_g, 6), "rel_l2_oracle": round(rl_o, 6)})
    return out


if __name__ == "__main__":
    main()
