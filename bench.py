"""Throughput of the exact demapper + fused GMI/MI reduction on one GPU.

Workload: 8-D M=2048 two-shell format, 16 SNR points (2..17 dB) x 1e7 seeded
AWGN samples each, generated on the device before the timed region. One
step = one mdgmi_gmi call over the whole batch (per-SNR staging, demapping
with exact per-bit LLRs, fused FP64 GMI/MI reduction). Metric: demapped
sample*points per second = n_snr * n * M / time.

Beside it: the FP32 direct-distance path and the bf16-split MFMA path on the
same samples, LLR output, hard decisions (BER/SER/Q), max-log and
s-optimised GMI, the paper's PAM/QAM formats, the streaming monitor, the
16-QAM FP64 and 4-D M=64 configurations, the ragged batch, the learned
demapper (trained on exact-LLR targets, then timed against the exact path on
the same held-out samples with per-SNR fallback), and the FP64 CPU oracle on
a bounded sample.

Prints one JSON line. `--gpus N` with N > 1 exits: the figure is one GPU's.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

# MI355X vector ALU: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz = 39.3e12 lane
# instructions/s for plain FP32 ops (the published 157.3 TFLOP/s counts 2
# flops per FMA and 2 per packed lane); v_exp_f32 takes twice the issue time
# of a plain op, so the exponential peak is 19.66e12/s = 157.3e12 / 8.
VALU_LANE_OPS = 157.3e12 / 4
EXP_PEAK = VALU_LANE_OPS / 2
HBM_PEAK = 8.0e12

# HBM traffic of one k_mfma launch on this workload, from two rocprofv3 --pmc
# passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what
# the same counter reads for a plain copy kernel of known size (a 1 GiB copy
# reads FETCH_SIZE = 0.5 GiB and WRITE_SIZE = 1 GiB: factors 2.0 and 1.0).
# Reported only while the kernel sources hash to the value they were taken on.
TRAFFIC = {"sources_sha1": "9c183599b721b4e3930c277069e91816175492cc", "fetch_kib": 2821978.9375, "write_kib": 1040.0,
           "fetch_scale": 2.0, "write_scale": 1.0}
KERNEL_SOURCES = ("mfma_core.h", "mfma_kernels.h", "device_common.h", "internal.h", "exact_mfma_d8_f16.hip")


def kernel_sources_sha1() -> str:
    import hashlib
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        h.update((ROOT / "paper_2011_13695_amd" / "csrc" / name).read_bytes())
    return h.hexdigest()


def measured_traffic():
    t = TRAFFIC
    if t["sources_sha1"] is None or t["sources_sha1"] != kernel_sources_sha1():
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0
METRIC = "demapped sample\u00b7points/sec at 8D M=2048 (exact vs learned) at |\u0394GMI|\u22640.01 b"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--path", default="mfma", choices=["mfma", "mfma_bf16", "direct", "f64", "auto"])
    ap.add_argument("--n", type=int, default=10_000_000, help="samples per SNR point")
    ap.add_argument("--cpu-seconds", type=float, default=18.0, help="target length of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true", help="skip timing the FP32 direct path beside")
    ap.add_argument("--learned-samples", type=float, default=2e8,
                    help="training samples of the learned demapper (0 skips the learned leg)")
    ap.add_argument("--learned-eval", type=float, default=1e8, help="held-out samples over the 16 SNR points")
    ap.add_argument("--learned-structured-samples", type=float, default=5e7,
                    help="training samples of the network on the structured 8-D M=4096 format (0 skips)")
    ap.add_argument("--learned-infer-only", action="store_true",
                    help="time the fused inference kernel on a random-initialised network and skip training")
    ap.add_argument("--no-ragged", action="store_true", help="skip the ragged-batch leg")
    ap.add_argument("--no-llr", action="store_true", help="skip timing the LLR-output mode")
    ap.add_argument("--no-hd", action="store_true", help="skip the hard-decision (BER/SER/Q) leg")
    ap.add_argument("--no-maxlog", action="store_true", help="skip the max-log / s-optimised GMI leg")
    ap.add_argument("--no-paper-formats", action="store_true", help="skip the PAM-N / QAM-N sweep")
    ap.add_argument("--no-stream", action="store_true", help="skip the streaming-monitor leg")
    ap.add_argument("--no-bf16", action="store_true", help="skip timing the bf16-split MFMA path beside")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the 16-QAM FP64 and 4-D M=64 configurations")
    ap.add_argument("--ragged-scale", type=float, default=1.0, help="scale of the ragged sample counts")
    ap.add_argument("--no-peak-probe", action="store_true", help="skip measuring the device's peak rates")
    ap.add_argument("--copy-probe", type=float, default=0,
                    help="only run a plain device copy of this many bytes (HBM counter calibration) and exit")
    return ap.parse_args()


def other_configs_leg(cpu_samples=20_000):
    """The two other single-GPU configurations beside the timed one, GPU and
    FP64 oracle on identical samples: 16-QAM (11 SNR x 1e5) on the FP64 GPU
    path against the oracle over all samples, and the 4-D M = 64 workload
    (21 SNR x 1e7) on every FP32 path, with the oracle timed and compared on
    the first cpu_samples samples of each SNR point."""
    import numpy as np
    import torch

    import oracle
    import workloads as w
    from paper_2011_13695_amd import mdgmi

    def gpu_time(gf, y, tx, s2, path, reps=3):
        ws = mdgmi.workspace(mdgmi.mdgmi_gmi_workspace_size(gf, y.shape[1], len(s2), path))
        out = mdgmi.mdgmi_gmi(gf, y, tx, s2, path=path, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            mdgmi.mdgmi_gmi(gf, y, tx, s2, path=path, ws=ws, out=out)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, out.cpu().numpy()

    res = {}
    # 16-QAM, FP64 on the GPU, every sample through the oracle
    wl = w.workload_qam16()
    f = wl.fmt
    gf = mdgmi.Format.of(f)
    y, tx = mdgmi.mdgmi_generate(gf, wl.seed, wl.sigma2, wl.n, dtype=torch.float64)
    t, out = gpu_time(gf, y, tx, wl.sigma2, "f64")
    yh, th = y.cpu().numpy(), tx.cpu().numpy().view(np.uint32)
    t0 = time.perf_counter()
    ref = oracle.gmi_per_snr(yh, th, f.X, f.labels, wl.sigma2)
    tc = time.perf_counter() - t0
    pairs = len(wl.sigma2) * wl.n * f.M
    res["16qam_f64"] = {"workload": wl.name, "gpu_f64_value": pairs / t, "gpu_ms": t * 1e3,
                        "oracle_value": pairs / tc, "oracle_cores": oracle.num_threads(),
                        "max_abs_dgmi_dmi_vs_oracle": float(np.abs(out[:, :2] - ref[:, :2]).max())}
    del y, tx
    # 4-D M = 64
    wl = w.workload_4d64()
    f = wl.fmt
    gf = mdgmi.Format.of(f)
    y, tx = mdgmi.mdgmi_generate(gf, wl.seed, wl.sigma2, wl.n, dtype=torch.float32)
    pairs = len(wl.sigma2) * wl.n * f.M
    row = {"workload": wl.name}
    for path in ("direct", "mfma", "mfma_bf16", "auto"):
        t, out = gpu_time(gf, y, tx, wl.sigma2, path)
        row[path] = {"value": pairs / t, "ms": t * 1e3, "exp_peak_frac": pairs / t / EXP_PEAK}
    ys = y[:, :cpu_samples].contiguous()
    ts = tx[:, :cpu_samples].contiguous()
    _, sub = gpu_time(gf, ys, ts, wl.sigma2, "auto", reps=1)
    yh, th = ys.cpu().numpy().astype(np.float64), ts.cpu().numpy().view(np.uint32)
    t0 = time.perf_counter()
    ref = oracle.gmi_per_snr(yh, th, f.X, f.labels, wl.sigma2)
    tc = time.perf_counter() - t0
    row["oracle_value"] = len(wl.sigma2) * cpu_samples * f.M / tc
    row["oracle_sample"] = f"first {cpu_samples} samples of each SNR point"
    row["max_abs_dgmi_dmi_vs_oracle_on_sample"] = float(np.abs(sub[:, :2] - ref[:, :2]).max())
    res["4d64"] = row
    del y, tx, ys, ts
    torch.cuda.empty_cache()
    return res


def cpu_baseline(wl, target_s: float):
    """The FP64 oracle on host cores over a bounded sample of the same
    workload (the first n_cpu samples of every SNR point, regenerated on the
    host from the same counters)."""
    import numpy as np

    import oracle
    import workloads as w
    f = wl.fmt
    threads = oracle.num_threads()
    # calibrate on a few samples, then size the sample to about target_s
    oracle.gmi(*w.channel_samples(f, float(wl.sigma2[0]), wl.seed, 0, n=64), f.X, f.labels, float(wl.sigma2[0]))
    y, tx = w.channel_samples(f, float(wl.sigma2[0]), wl.seed, 0, n=4096)
    t0 = time.perf_counter()
    oracle.gmi(y, tx, f.X, f.labels, float(wl.sigma2[0]))
    per_sample = max((time.perf_counter() - t0) / 4096, 1e-8)
    n_cpu = int(max(64, min(200_000, target_s / per_sample / len(wl.snr_db))))
    elapsed = 0.0
    for q, s2 in enumerate(wl.sigma2):
        y, tx = w.channel_samples(f, float(s2), wl.seed, q, n=n_cpu)
        t0 = time.perf_counter()
        oracle.gmi(y, tx, f.X, f.labels, float(s2))
        elapsed += time.perf_counter() - t0
    pairs = n_cpu * len(wl.snr_db) * f.M
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fp:
            model = next((l.split(":", 1)[1].strip() for l in fp if l.startswith("model name")), model)
    except OSError:
        pass
    return {"value": pairs / elapsed, "unit": "sample*points/s", "cores": threads, "kind": "oracle",
            "cpu_model": model,
            "sample": f"first {n_cpu} samples of each of the {len(wl.snr_db)} SNR points "
                      f"({pairs:.3g} sample*points, {elapsed:.1f} s, FP64, {threads} threads)"}


def copy_probe(nbytes: float):
    """A plain elementwise copy kernel of known size, for scaling the HBM
    byte counters of the profiler: reads and writes nbytes once each."""
    import torch
    n = int(nbytes) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 3}))


MLP_FLOPS_PER_SAMPLE = 2 * (9 * 256 + 256 * 256 + 256 * 256 + 256 * 11)   # 9 -> 256 -> 256 -> 256 -> 11
GELUS_PER_SAMPLE = 3 * 256
BF16_PEAK = 2.5e15


def timed_ms(fn, reps=3):
    """Mean device time of fn() over reps calls, HIP events on the current stream."""
    import torch
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


# The fused kernel's GELU costs the vector ALU 6 issue slots: 12 per pair of
# values (fp16 conversion, 8 packed fp16 FMAs for the clamped polynomial gate,
# two mixed-precision products, one bf16 pair conversion).
GELU_SLOTS = 6
GELU_PEAK = VALU_LANE_OPS / GELU_SLOTS


def learned_roofline(samples, ms):
    """The fused inference kernel against its binding roofline, the vector
    ALU's GELU rate (768 GELUs per sample of the 9-256-256-256-11 network),
    with the bf16 matrix-core figure (algorithmic flops) beside it."""
    flops = samples * MLP_FLOPS_PER_SAMPLE / (ms * 1e-3)
    gelus = samples * GELUS_PER_SAMPLE / (ms * 1e-3)
    return {"bound": "alu", "achieved": gelus / 1e12, "peak": GELU_PEAK / 1e12, "unit": "TGELU/s",
            "frac": gelus / GELU_PEAK,
            "mfma": {"achieved": flops / 1e12, "peak": BF16_PEAK / 1e12, "unit": "TFLOP/s", "frac": flops / BF16_PEAK},
            "kernel": "k_mlp_fused (bf16 MFMA; GELU on the vector ALU, 6 issue slots each)", "kernel_ms": ms}


def learned_route_leg(gf, fmt_name, snr, n_eval, net, log, train=None):
    """Held-out evaluation of a trained network on one format: the library's
    calibration (paired GMI loss per SNR point, route learned where <= 0.01
    bit), then learned-only, exact and routed (MDGMI_PATH_LEARNED_BF16) GMI
    timed on the same samples."""
    import numpy as np
    import torch

    from paper_2011_13695_amd import learned, mdgmi
    n_snr = snr.size
    ev, y, tx = learned.evaluate(net, gf, snr, n_eval, sopt=True)
    s2 = learned.sigma2_of(snr, gf.dim)
    out = torch.empty((n_snr, mdgmi.MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
    lws = mdgmi.workspace(mdgmi.mdgmi_mlp_gmi_workspace_size(net, min(1 << 20, n_eval)))
    ews = mdgmi.workspace(mdgmi.mdgmi_gmi_workspace_size(gf, n_eval, n_snr, "mfma"))
    rws = mdgmi.workspace(mdgmi.mdgmi_gmi_workspace_size(gf, n_eval, n_snr, "learned"))
    t_learned = timed_ms(lambda: mdgmi.mdgmi_mlp_gmi(net, gf, y, tx, snr, out=out, ws=lws))
    t_exact = timed_ms(lambda: mdgmi.mdgmi_gmi(gf, y, tx, s2, path="mfma", out=out, ws=ews))
    t_mixed = timed_ms(lambda: mdgmi.mdgmi_gmi(gf, y, tx, s2, path="learned", out=out, ws=rws))
    routed = out.cpu().numpy()
    pts = n_snr * n_eval * gf.M
    n_learned = sum(r == "learned" for r in ev.route)
    log(f"{fmt_name}: learned {t_learned:.1f} ms, exact {t_exact:.1f} ms, routed {t_mixed:.1f} ms, "
        f"{n_learned}/{n_snr} SNR points learned, max loss {max(ev.loss):.4f}")
    row = dict(train or {})
    row.update({
        "format": fmt_name, "eval_samples_per_snr": n_eval,
        "learned_value": pts / (t_learned * 1e-3), "learned_ms": t_learned,
        "exact_value_same_samples": pts / (t_exact * 1e-3), "exact_ms": t_exact,
        "speedup_learned_vs_exact": t_exact / t_learned,
        "mixed_value": pts / (t_mixed * 1e-3), "mixed_ms": t_mixed, "speedup_mixed_vs_exact": t_exact / t_mixed,
        "snr_db": [float(v) for v in snr],
        "gmi_exact": [float(v) for v in ev.gmi_exact], "gmi_learned": [float(v) for v in ev.gmi_learned],
        "gmi_loss": [float(v) for v in ev.loss], "route": ev.route,
        "gmi_routed": [float(v) for v in routed[:, 0]],
        "s_opt_learned": [float(v) for v in ev.s_opt],
        "gmi_loss_sopt": [float(a - b) for a, b in zip(ev.gmi_exact, ev.gmi_learned_sopt)],
        "n_learned_snr": int(n_learned), "max_loss_bound": 0.01,
        "roofline": learned_roofline(n_snr * n_eval, t_learned),
    })
    return row


def train_net(gf, samples, log, **kw):
    """Trains the network on gf; records the paired GMI loss on fixed
    held-out samples at six SNR points eight times along the way."""
    import torch
    from paper_2011_13695_amd import learned
    cfg = learned.TrainConfig(log_every=2000, **kw)
    cfg.steps = max(1, int(samples) // cfg.batch)
    tr = learned.Trainer(gf, cfg)
    held = learned.HeldOut(gf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = tr.train(log=log, held_out=held)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"trained {res.samples} samples in {train_s:.1f} s")
    return tr.net, {"train_samples": res.samples, "train_seconds": train_s, "train_steps": res.steps,
                    "batch": cfg.batch, "lr": cfg.lr,
                    "train_flops_per_s": 3 * MLP_FLOPS_PER_SAMPLE * res.samples / train_s,
                    "final_train_loss_nats": res.losses[-1][1] if res.losses else None,
                    "heldout_curve": {"snr_db": [float(v) for v in held.snr], "samples_per_snr": held.y.shape[1],
                                      "gmi_exact": [float(v) for v in held.exact],
                                      "samples_seen": [c[0] for c in res.curve],
                                      "gmi_loss": [c[1] for c in res.curve],
                                      "note": "paired GMI loss (bit) of the network on fixed held-out samples "
                                              "during training; train_seconds includes these evaluations"}}


def learned_leg(gf, wl, args, log):
    """Learned demapper on the timed format: train on exact-LLR targets, then
    learned vs exact vs routed GMI on the same held-out samples."""
    import numpy as np
    net, tr = train_net(gf, args.learned_samples, log)
    snr = np.asarray(wl.snr_db, dtype=np.float64)
    n_eval = max(1024, int(args.learned_eval) // snr.size)
    row = learned_route_leg(gf, wl.fmt.name, snr, n_eval, net, log, tr)
    row["note"] = ("learned value counts n*M sample*points per sample demapped by the network; routed = "
                   "MDGMI_PATH_LEARNED_BF16 (per-SNR route decided by mdgmi_learned_calibrate: learned where the "
                   "paired GMI loss <= 0.01 bit, else exact)")
    return row


def learned_structured_leg(args, log):
    """The same network on a structured 8-D format (M = 4096, a product of
    four Gray 8-QAM constellations), where it meets the 0.01-bit bound: what
    the trained network gains over the exact demapper."""
    import numpy as np
    import workloads as w
    from paper_2011_13695_amd import mdgmi
    f = w.qam_product(8, 12)
    gf = mdgmi.Format.of(f)
    net, tr = train_net(gf, args.learned_structured_samples, log)
    snr = np.arange(2.0, 18.0)
    n_eval = max(1024, int(args.learned_eval) // snr.size)
    row = learned_route_leg(gf, f.name, snr, n_eval, net, log, tr)
    row["note"] = "8-D M = 4096 Gray 8-QAM product; network and training as for the timed format"
    return row


def learned_infer_leg(gf, args, log):
    """Fused inference alone (random-initialised network of the timed shape,
    no training): GMI mode over learned_eval samples and LLR mode, for
    profiling and the kernel's roofline."""
    import numpy as np
    import torch
    from paper_2011_13695_amd import learned, mdgmi
    net = mdgmi.MLP([gf.dim + 1, 256, 256, 256, gf.m], seed=5)
    snr = np.arange(2.0, 18.0)
    n = max(1024, int(args.learned_eval) // snr.size)
    y, tx = mdgmi.mdgmi_generate(gf, 77, learned.sigma2_of(snr, gf.dim), n, snr_slot0=8_000_000)
    out = torch.empty((snr.size, mdgmi.MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
    lws = mdgmi.workspace(mdgmi.mdgmi_mlp_gmi_workspace_size(net, min(1 << 20, n)))
    t_gmi = timed_ms(lambda: mdgmi.mdgmi_mlp_gmi(net, gf, y, tx, snr, out=out, ws=lws))
    lam = torch.empty((n, gf.m), dtype=torch.float32, device="cuda")
    sn = torch.full((n,), 10.0, dtype=torch.float32, device="cuda")
    t_llr = timed_ms(lambda: net.llr(y[0], sn, out=lam))
    log(f"learned inference: GMI mode {t_gmi:.1f} ms for {snr.size * n} samples, LLR mode {t_llr:.2f} ms for {n}")
    return {"samples": int(snr.size * n), "gmi_mode_ms": t_gmi, "llr_mode_ms_per_snr_point": t_llr,
            "roofline": learned_roofline(snr.size * n, t_gmi)}


def q_crossing(snr_db, q_db, q_ref):
    """SNR (dB) at which the Q-factor curve first reaches q_ref, by linear
    interpolation between the bracketing SNR points (None if it never does)."""
    for k in range(len(snr_db) - 1):
        a, b = q_db[k], q_db[k + 1]
        if a is not None and a < q_ref and (b is None or b >= q_ref):
            if b is None:
                return float(snr_db[k + 1])
            return float(snr_db[k] + (q_ref - a) / (b - a) * (snr_db[k + 1] - snr_db[k]))
    return None


def hd_leg(gf, wl, y, tx, path, gmi_out, reps=3):
    """Hard decisions on the timed workload: bit error rate of the bitwise MAP
    decision, symbol error rate of the nearest-point decision and the Q-factor
    per SNR point, with the SNR at which Q reaches the HD-FEC thresholds the
    paper quotes (8.4 dB at 6.7 % overhead, 5.7 dB at 20 %)."""
    import numpy as np
    import torch
    from paper_2011_13695_amd import mdgmi

    n_snr = len(wl.sigma2)
    ws = mdgmi.workspace(mdgmi.mdgmi_gmi_hd_workspace_size(gf, wl.n, n_snr, path))
    out = torch.empty((n_snr, mdgmi.MDGMI_NFIELDS_HD), dtype=torch.float64, device="cuda")
    mdgmi.mdgmi_gmi_hd(gf, y, tx, wl.sigma2, path=path, out=out, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mdgmi.mdgmi_gmi_hd(gf, y, tx, wl.sigma2, path=path, out=out, ws=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    h = out.cpu().numpy()
    q_db = [mdgmi.mdgmi_q_factor_db(float(b)) for b in h[:, 6]]
    q_db = [None if not np.isfinite(v) else float(v) for v in q_db]   # BER 0: Q unbounded
    snr = [float(v) for v in wl.snr_db]
    return {"ms_per_call": ms, "value": n_snr * wl.n * gf.M / (ms * 1e-3),
            "ber": [float(v) for v in h[:, 6]], "ser": [float(v) for v in h[:, 7]], "q_db": q_db,
            "snr_db_at_q_8.4dB": q_crossing(snr, q_db, 8.4), "snr_db_at_q_5.7dB": q_crossing(snr, q_db, 5.7),
            "max_abs_dgmi_vs_timed_path": float(np.abs(h[:, :2] - gmi_out[:, :2]).max()),
            "note": "mdgmi_gmi_hd: GMI/MI plus BER/SER in one pass; Q = 20 log10(sqrt(2) erfc^-1(2 BER))"}


def maxlog_leg(gf, wl, y, tx, path, gmi_out, exact_ms, reps=3):
    """Max-log metrics on the timed workload: the GMI of max-log LLRs in one
    launch (timed), and per SNR point the s-optimised GMI of the exact and of
    the max-log LLRs (mdgmi_llr / mdgmi_llr_maxlog, then mdgmi_gmi_sopt)."""
    import numpy as np
    import torch
    from paper_2011_13695_amd import mdgmi

    n_snr = len(wl.sigma2)
    pairs = n_snr * wl.n * gf.M
    ws = mdgmi.workspace(mdgmi.mdgmi_gmi_workspace_size(gf, wl.n, n_snr, path))
    out = torch.empty((n_snr, mdgmi.MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
    mdgmi.mdgmi_gmi_maxlog(gf, y, tx, wl.sigma2, path=path, out=out, ws=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        mdgmi.mdgmi_gmi_maxlog(gf, y, tx, wl.sigma2, path=path, out=out, ws=ws)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    ml = out.cpu().numpy()
    del ws
    lam = torch.empty((wl.n, gf.m), dtype=torch.float32, device="cuda")
    lws = mdgmi.workspace(mdgmi.mdgmi_llr_workspace_size(gf, wl.n, path))
    sws = mdgmi.workspace(mdgmi.mdgmi_gmi_sopt_workspace_size(wl.n))
    sout = torch.empty(mdgmi.MDGMI_NFIELDS_S, dtype=torch.float64, device="cuda")
    rows = {"exact": [], "maxlog": []}
    sopt_ms = []
    for q in range(n_snr):
        for name, fn in (("exact", mdgmi.mdgmi_llr), ("maxlog", mdgmi.mdgmi_llr_maxlog)):
            fn(gf, y[q], float(wl.sigma2[q]), path=path, llr=lam, ws=lws)
            a.record(stream)
            mdgmi.mdgmi_gmi_sopt(gf, lam, tx[q], out=sout, ws=sws)
            b.record(stream)
            torch.cuda.synchronize()
            sopt_ms.append(a.elapsed_time(b))
            rows[name].append(sout.cpu().numpy().copy())
    del lam, lws, sws
    ex = np.array(rows["exact"])
    mx = np.array(rows["maxlog"])
    return {"ms_per_call": ms, "value": pairs / (ms * 1e-3), "speedup_vs_exact_gmi": exact_ms / ms,
            "gmi_maxlog_s1": [float(v) for v in ml[:, 0]],
            "gmi_exact_minus_maxlog_s1": [float(v) for v in gmi_out[:, 0] - ml[:, 0]],
            "s_opt_exact": [float(v) for v in ex[:, 2]], "gmi_sopt_exact": [float(v) for v in ex[:, 3]],
            "s_opt_maxlog": [float(v) for v in mx[:, 2]], "gmi_sopt_maxlog": [float(v) for v in mx[:, 3]],
            "ngmi_sopt_exact": [float(v) for v in ex[:, 5]],
            "sopt_passes_max": int(max(ex[:, 8].max(), mx[:, 8].max())),
            "sopt_ms_per_snr_point": float(np.mean(sopt_ms)),
            "note": "mdgmi_gmi_maxlog over all SNR points in one launch (timed); s-optimised GMI of the exact "
                    "and max-log LLRs per SNR point via mdgmi_gmi_sopt (1e7 x 11 LLRs each)"}


def paper_formats_leg(n=1 << 20, snr_db=None):
    """The paper's formats (Gray PAM-2/4/8/16, QAM-4/16/64) over AWGN: an SNR
    sweep of GMI, MI and bit error rate per format (mdgmi_gmi_hd, AUTO path,
    samples generated on the device), with the SNR at which the Q-factor
    reaches the HD-FEC thresholds the paper quotes (8.4 dB, 5.7 dB) and the
    GMI there. These are the AWGN references for the paper's OSNR results."""
    import numpy as np
    import torch
    import workloads as w
    from paper_2011_13695_amd import mdgmi

    snr = np.arange(0.0, 40.0 + 1e-9, 1.0) if snr_db is None else np.asarray(snr_db)
    res = {}
    t_all = 0.0
    for k, f in enumerate(w.paper_formats()):
        gf = mdgmi.Format.of(f)
        s2 = w.sigma2_from_snr_db(snr, f.dim)
        y, tx = mdgmi.mdgmi_generate(gf, 1000 + k, s2, n, dtype=torch.float32)
        ws = mdgmi.workspace(mdgmi.mdgmi_gmi_hd_workspace_size(gf, n, len(snr), "auto"))
        out = mdgmi.mdgmi_gmi_hd(gf, y, tx, s2, path="auto", ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = mdgmi.mdgmi_gmi_hd(gf, y, tx, s2, path="auto", ws=ws)
        torch.cuda.synchronize()
        t_all += time.perf_counter() - t0
        h = out.cpu().numpy()
        q = [mdgmi.mdgmi_q_factor_db(float(b)) for b in h[:, 6]]
        q = [None if not np.isfinite(v) else float(v) for v in q]
        row = {"m": f.m}
        for thr in (8.4, 5.7):
            x = q_crossing([float(v) for v in snr], q, thr)
            row[f"snr_db_at_q_{thr}dB"] = x
            row[f"gmi_at_q_{thr}dB"] = None if x is None else float(np.interp(x, snr, h[:, 0]))
        row["gmi"] = [round(float(v), 5) for v in h[:, 0]]
        res[f.name] = row
        del y, tx, ws, out
    return {"snr_db": [float(v) for v in snr], "n_per_snr": n, "ms_all_formats": t_all * 1e3, "formats": res,
            "note": "AWGN, unit-energy Gray formats, SNR per symbol; Q = 20 log10(sqrt(2) erfc^-1(2 BER))"}


BUFFER_SAMPLES = 1 << 22      # the paper's buffer: 2^22 ADC samples
BUFFER_BUDGET_MS = 1.049       # 2^22 samples at 4 GSa/s


def stream_leg(n_buffers=32, warm=4, lanes=4, distinct=8):
    """Streaming monitor: buffers of 2^22 samples pushed through
    mdgmi_stream on `lanes` HIP streams, from device memory and from pinned
    host memory (PCIe copy included), for the paper's 16-QAM and the 8-D
    M = 2048 format at 10 dB. `distinct` buffers are generated once and
    pushed in turn; the rate is over n_buffers pushes after `warm`."""
    import numpy as np
    import torch
    import workloads as w
    from paper_2011_13695_amd import mdgmi

    res = {"buffer_samples": BUFFER_SAMPLES, "budget_ms_per_buffer": BUFFER_BUDGET_MS, "lanes": lanes}
    for name, f in (("16-QAM", w.format_16qam()), ("8D-2048", w.format_8d2048())):
        gf = mdgmi.Format.of(f)
        s2 = float(w.sigma2_from_snr_db(10.0, f.dim))
        y, tx = mdgmi.mdgmi_generate(gf, 4242, [s2] * distinct, BUFFER_SAMPLES, dtype=torch.float32)
        row = {}
        for mode in ("device", "pinned_host"):
            if mode == "device":
                src = [(y[k], tx[k]) for k in range(distinct)]
            else:
                src = [(y[k].cpu().pin_memory(), tx[k].cpu().pin_memory()) for k in range(distinct)]
            st = mdgmi.Stream(gf, s2, BUFFER_SAMPLES, n_lanes=lanes, path="auto", ring=256)
            for k in range(warm):
                st.push(*src[k % distinct])
            st.wait()
            t0 = time.perf_counter()
            for k in range(n_buffers):
                st.push(*src[k % distinct])
            st.wait()
            dt = time.perf_counter() - t0
            tot = st.total()
            st.close()
            ms = dt / n_buffers * 1e3
            row[mode] = {"ms_per_buffer": ms, "real_time_factor": BUFFER_BUDGET_MS / ms,
                         "sample_points_per_s": BUFFER_SAMPLES * f.M / (ms * 1e-3),
                         "gmi": float(tot[0]), "mi": float(tot[1])}
            del src
        res[name] = row
        del y, tx
        torch.cuda.empty_cache()
    res["note"] = ("real_time_factor = 1.049 ms budget / measured ms per buffer (> 1 keeps up); pinned_host "
                   "includes the PCIe copy of y and tx for every buffer")
    return res


def ragged_leg(args, log, scale=None):
    """Ragged batch: 48 formats (dims 2/4/8, M = 4..4096) x 31 SNR points with
    log-uniform sample counts in [1e4, 1e7], paths and tiles from the
    autotuner, in one persistent hipGraph launch against one mdgmi_gmi call
    per instance on the same samples."""
    import numpy as np
    import torch

    import workloads as w
    from paper_2011_13695_amd import mdgmi
    fmts = w.ragged_formats()
    snr = w.RAGGED_SNR_DB
    counts = w.ragged_counts(len(fmts), len(snr))
    scale = args.ragged_scale if scale is None else scale
    if scale != 1.0:
        counts = np.maximum(1, np.round(counts * scale)).astype(np.int64)
    t0 = time.perf_counter()
    for dim, M in sorted({(f.dim, f.M) for f in fmts}):
        mdgmi.mdgmi_autotune(dim, M)
    tune_s = time.perf_counter() - t0
    gfs = [mdgmi.Format.of(f) for f in fmts]
    items, pairs = [], 0
    for a, (f, gf) in enumerate(zip(fmts, gfs)):
        for q, sdb in enumerate(snr):
            n = int(counts[a, q])
            s2 = float(w.sigma2_from_snr_db(float(sdb), f.dim))
            y, tx = mdgmi.mdgmi_generate(gf, 7 + a, [s2], n, snr_slot0=q, dtype=torch.float32)
            items.append((gf, y.view(n, f.dim), tx.view(n), s2))
            pairs += n * f.M
    torch.cuda.synchronize()
    log(f"ragged: {len(items)} instances, {int(counts.sum())} samples, {pairs:.3e} sample*points "
        f"(tuning {tune_s:.1f} s)")
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    plan = mdgmi.Batch(items, path="auto")
    out_b = torch.empty((len(items), mdgmi.MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
    t_batch = timed(lambda: plan.run(out=out_b, use_graph=True), 3)
    log(f"ragged: one graph launch {t_batch:.1f} ms")
    ws = mdgmi.workspace(max(mdgmi.mdgmi_gmi_workspace_size(gf, y.shape[0], 1, "auto") for gf, y, _, _ in items))
    out_i = torch.empty_like(out_b)

    def per_instance():
        for q, (gf, y, tx, s2) in enumerate(items):
            mdgmi.mdgmi_gmi(gf, y.view(1, -1, gf.dim), tx.view(1, -1), [s2], path="auto", out=out_i[q:q + 1], ws=ws)

    t_inst = timed(per_instance, 2)
    log(f"ragged: per-instance launches {t_inst:.1f} ms")
    ob, oi = out_b.cpu().numpy(), out_i.cpu().numpy()
    info = plan.info()
    plan.close()
    return {"instances": len(items), "formats": len(fmts), "snr_points": int(len(snr)),
            "samples": int(counts.sum()), "sample_points": int(pairs), "work_items": info["items"],
            "value_batched": pairs / (t_batch * 1e-3), "ms_batched": t_batch,
            "value_per_instance": pairs / (t_inst * 1e-3), "ms_per_instance": t_inst,
            "speedup_batched_vs_per_instance": t_inst / t_batch, "tune_seconds": tune_s,
            "max_abs_dgmi_batched_vs_per_instance": float(np.nanmax(np.abs(ob[:, 0] - oi[:, 0]))),
            "max_abs_dmi_batched_vs_per_instance": float(np.nanmax(np.abs(ob[:, 1] - oi[:, 1]))),
            "count_scale": scale, "unit": "sample*points/s"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "single-GPU benchmark: the GMI/MI engine runs on one GPU and has no "
                                   "multi-GPU mode (shards would all-reduce 5 doubles per SNR point)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as w
    from paper_2011_13695_amd import mdgmi

    torch.cuda.set_device(0)
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    wl = w.workload_8d2048(n=args.n)
    f = wl.fmt
    gf = mdgmi.Format.of(f)
    s2 = wl.sigma2
    n_snr = len(s2)
    y, tx = mdgmi.mdgmi_generate(gf, wl.seed, s2, wl.n, dtype=torch.float32)
    torch.cuda.synchronize()
    print(f"[bench] generated {n_snr} x {wl.n} samples of {f.name}", file=sys.stderr, flush=True)

    def run_path(path, steps, warmup):
        ws = mdgmi.workspace(mdgmi.mdgmi_gmi_workspace_size(gf, wl.n, n_snr, path))
        out = torch.empty((n_snr, mdgmi.MDGMI_NFIELDS), dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            mdgmi.mdgmi_gmi(gf, y, tx, s2, path=path, out=out, ws=ws)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            mdgmi.mdgmi_gmi(gf, y, tx, s2, path=path, out=out, ws=ws)
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        call_ms = [a.elapsed_time(b) for a, b in evs]
        return wall, call_ms, out.cpu().numpy()

    wall, call_ms, out = run_path(args.path, args.steps, args.warmup)
    print(f"[bench] {args.path}: {wall / args.steps * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    pairs = n_snr * wl.n * f.M
    ms_per_step = wall / args.steps * 1e3
    value = pairs / (wall / args.steps)
    kernel_ms = float(np.mean(call_ms))
    extra = {}
    if not args.no_direct and args.path != "direct":
        dwall, dms, dout = run_path("direct", max(2, args.steps // 3), 1)
        extra["direct_fp32"] = {"value": pairs / (dwall / max(2, args.steps // 3)),
                                "ms_per_step": dwall / max(2, args.steps // 3) * 1e3,
                                "max_abs_dgmi_vs_timed_path": float(np.abs(dout[:, :2] - out[:, :2]).max()),
                                "speedup_timed_path_vs_direct": dwall / max(2, args.steps // 3) / (wall / args.steps)}
    if not args.no_bf16 and args.path == "mfma":
        bsteps = max(2, args.steps // 3)
        bwall, bms, bout = run_path("mfma_bf16", bsteps, 1)
        extra["mfma_bf16"] = {"value": pairs / (bwall / bsteps), "ms_per_step": bwall / bsteps * 1e3,
                              "max_abs_dgmi_vs_timed_path": float(np.abs(bout[:, :2] - out[:, :2]).max()),
                              "note": "the same workload on the bf16 three-part split (any SNR range)"}
    if not args.no_llr:
        # LLR output of every sample (11 FP32 per sample written to HBM)
        lam = torch.empty((wl.n, f.m), dtype=torch.float32, device="cuda")
        lws = mdgmi.workspace(mdgmi.mdgmi_llr_workspace_size(gf, wl.n, args.path))
        stream = torch.cuda.current_stream()
        for q in range(min(2, n_snr)):
            mdgmi.mdgmi_llr(gf, y[q], float(s2[q]), path=args.path, llr=lam, ws=lws)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for q in range(n_snr):
            mdgmi.mdgmi_llr(gf, y[q], float(s2[q]), path=args.path, llr=lam, ws=lws)
        b.record(stream)
        torch.cuda.synchronize()
        lms = a.elapsed_time(b)
        extra["llr_mode"] = {"value": pairs / (lms * 1e-3), "ms_all_snr": lms,
                             "bytes_written": n_snr * wl.n * f.m * 4,
                             "note": "mdgmi_llr over every SNR point, one call each, LLRs of all samples written"}
        del lam, lws
    if not args.no_hd:
        extra["hard_decisions"] = hd_leg(gf, wl, y, tx, args.path, out)
    if not args.no_maxlog:
        extra["maxlog_sopt"] = maxlog_leg(gf, wl, y, tx, args.path, out, ms_per_step)
    if not args.no_paper_formats:
        extra["paper_formats"] = paper_formats_leg()
    if not args.no_stream:
        y = tx = None  # the workload's 5.7 GB are not needed any more
        torch.cuda.empty_cache()
        extra["stream"] = stream_leg()
    if not args.no_other_configs:
        y = tx = None
        torch.cuda.empty_cache()
        extra["other_configs"] = other_configs_leg()
    achieved = pairs / (kernel_ms * 1e-3)
    peaks = None if args.no_peak_probe else mdgmi.mdgmi_probe_rates()
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "sample*points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.path == "f64" else "f32",
        "data": "synthetic: seeded Philox-4x32-10 / Box-Muller AWGN samples generated on the device",
        "config": {"workload": wl.name, "format": f.name, "dim": f.dim, "M": f.M, "n_snr": n_snr,
                   "n_per_snr": wl.n, "snr_db": [float(v) for v in wl.snr_db], "path": args.path,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": EXP_PEAK / 1e12, "unit": "Texp/s",
                     "frac": achieved / EXP_PEAK, "traffic": measured_traffic(),
                     "traffic_unit": "bytes per launch",
                     "kernel": "k_mfma (demap + fused reduction); 1 v_exp_f32 per (sample, point)",
                     "kernel_ms": kernel_ms,
                     "measured_peak": None if peaks is None else peaks["exp_per_s"] / 1e12,
                     "frac_of_measured_peak": None if peaks is None else achieved / peaks["exp_per_s"]},
        "measured_peaks": peaks,
        "gmi": [float(v) for v in out[:, 0]],
        "mi": [float(v) for v in out[:, 1]],
    }
    line.update(extra)
    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)
    if args.learned_infer_only:
        line["learned_inference"] = learned_infer_leg(gf, args, lambda m: log("learned: " + m))
    elif args.learned_samples > 0:
        y = tx = None
        torch.cuda.empty_cache()
        line["learned"] = learned_leg(gf, wl, args, lambda m: log("learned: " + m))
        if args.learned_structured_samples > 0:
            line["learned_structured"] = learned_structured_leg(args, lambda m: log("learned: " + m))
    if not args.no_ragged:
        y = tx = None
        torch.cuda.empty_cache()
        line["ragged_batch"] = ragged_leg(args, log)
        # the same set with 1/100 of the samples: launch-bound per instance
        line["ragged_batch_small"] = ragged_leg(args, log, scale=args.ragged_scale * 0.01)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
