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
     graph-replayed) -> average duration of the gather+FFT stage and the
     decode stage, from which the roofline figures are computed.
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

# HBM bytes of the gather + FFT kernel (syndrome_kernel<float, 4096, float>) per
# algorithmic byte read and written, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# scaled by the plain-copy calibration (profiles/syndrome_kernel_n20_b1024_traffic.md,
# profiles/syndrome_kernel_iterative_n20_b1024_traffic.md).
TRAFFIC_RATIOS = {"exact": (2.01, 1.00), "general": (7.98, 1.00), "iterative": (5.27, 1.00)}

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
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for counter calibration)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain comparison")
    ap.add_argument("--no-uneven", action="store_true", help="skip the batched uneven workload")
    ap.add_argument("--no-iterative", action="store_true", help="skip the iterative-vs-non-iterative comparison")
    ap.add_argument("--fft64", action="store_true", help="FP64 FFTs for the complex64 input (SFT_FLAG_FFT64)")
    ap.add_argument("--no-model", action="store_true", help="skip the recovery-vs-collision-model section")
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
    return {"workload": f"exact, N=2^20, K=1000, unit amplitudes, complex64 with FP64 FFTs, {B} signals per cell",
            "rows": rows}


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
    import torch

    import sftgen
    from paper_1407_8315_amd import Plan

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if a.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.complex64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 8, "launches": 5}))
        return

    n, k, m, L, R = 1 << 20, 1000, 4096, 4, 12
    B = a.batch
    snrs = [10, 20, 30, 40]
    mode = a.mode
    stream = torch.cuda.Stream(device=dev)
    xs, truth = [], []
    t0 = time.time()
    with torch.cuda.stream(stream):
        for i in range(B):
            snr = snrs[i % 4] if mode == "general" else None
            x, locs, _ = sftgen.torch_signal(n, k, sftgen.BASE_SEED + i, dev, amp="gauss", snr_db=snr)
            xs.append(x)
            truth.append(locs)
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
        st = None
        for _ in range(a.steps):
            st = run(stats=True)
            stage += np.array(st["stage_ms"])
        stage /= a.steps
    signals_per_s = B / (ms_step * 1e-3)
    freqs_per_s = found / (ms_step * 1e-3)
    recovery = found / (B * k)

    # samples gathered (= syndromes written) per signal: 2L (+ R) lines of M;
    # iterative: two lines per iteration on grids of M, M/2, ...
    samples = 2 * sum(m >> l for l in range(L)) if mode == "iterative" else (2 * L + (R if mode == "general" else 0)) * m
    synd_bytes = B * samples * 8 * (3 if a.fft64 else 2)   # gather read (8 B) + syndrome write (8 or 16 B)
    fft_gbs = synd_bytes / (stage[0] * 1e-3) / 1e9
    ratios = None if a.fft64 else TRAFFIC_RATIOS.get(mode)
    # measured HBM bytes per launch (fetch + write), when counters were taken for this mode
    traffic = int(B * samples * 8 * (ratios[0] + ratios[1])) if ratios else None
    roofline = {"bound": "hbm", "achieved": round(fft_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(fft_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_gbs": round(traffic / (stage[0] * 1e-3) / 1e9, 1) if traffic else None,
                "kernel": "syndrome_kernel<double, 4096, float> (gather + FFT)" if a.fft64
                else "syndrome_kernel<float, 4096, float> (gather + FFT)",
                "algorithmic_bytes_per_launch": synd_bytes, "avg_launch_ms": round(stage[0], 4)}

    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(n, k, m, L, R, mode, plan, a.cpu_seconds, snrs)
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
        "stats_last_step": {kk: v for kk, v in st.items() if kk != "stage_ms"} if st else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "learned_vs_plain": lvp,
        "uneven_batch": unv,
        "mlp_kernels": mlp,
        "iterative_vs_non_iterative": itv,
        "paper_tables_2_4": tables,
        "recovery_vs_model": model,
        "input_generation_s": round(gen_s, 2),
    }
    print(json.dumps(out))


def cpu_baseline(n, k, m, L, R, mode, plan, budget_s, snrs):
    """The FP64 oracle on a bounded sample of the same workload, one host thread."""
    import numpy as np

    import oracle
    import sftgen
    from oracle import iterative as oracle_iterative

    done, found, t_total, c_total = 0, 0, 0.0, 0.0
    i = 0
    while t_total < budget_s and i < min(256, len(plan.infos)):
        snr = snrs[i % 4] if mode == "general" else None
        s = sftgen.make_signal(n, k, sftgen.BASE_SEED + i, amp="gauss", dtype=np.complex64, snr_db=snr)
        t0, c0 = time.perf_counter(), time.process_time()
        if mode == "general":
            r = oracle.sfft_general(s.x, n, k, m, L, plan.infos[i]["rshifts"])
        elif mode == "iterative":
            r, _ = oracle_iterative.sfft_iterative(s.x, n, m, L)
        else:
            r = oracle.sfft_exact(s.x, n, m, L)
        t_total += time.perf_counter() - t0
        c_total += time.process_time() - c0
        found += len(np.intersect1d(r.locs, s.locs))
        done += 1
        i += 1
    return {"value": round(found / t_total, 1), "unit": "freqs/s", "cores": max(1, round(c_total / t_total)),
            "kind": "oracle",
            "signals_per_s": round(done / t_total, 3),
            "sample": f"first {done} signals of the batch (same seeds), {t_total:.1f} s of CPU time; "
                      "signal generation excluded"}


if __name__ == "__main__":
    main()
