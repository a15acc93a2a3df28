"""Throughput of the exact demapper + fused GMI/MI reduction on one GPU.

Workload: 8-D M=2048 two-shell format, 16 SNR points (2..17 dB) x 1e7 seeded
AWGN samples each, generated on the device before the timed region. One
step = one mdgmi_gmi call over the whole batch (per-SNR staging, demapping
with exact per-bit LLRs, fused FP64 GMI/MI reduction). Metric: demapped
sample*points per second = n_snr * n * M / time.

Prints one JSON line. `--gpus N` with N > 1 exits: this build measures the
one-GPU share only.
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

# MI355X published peaks (vector ALU): FP32 157.3 TFLOP/s = 78.6e12 lane FMA/s;
# the transcendental unit (v_exp_f32) issues at a quarter of the FMA rate.
VALU_LANE_OPS = 157.3e12 / 2
EXP_PEAK = VALU_LANE_OPS / 4
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--path", default="mfma", choices=["mfma", "direct", "f64", "auto"])
    ap.add_argument("--n", type=int, default=10_000_000, help="samples per SNR point")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true", help="skip timing the FP32 direct path beside")
    return ap.parse_args()


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
    y, tx = w.channel_samples(f, float(wl.sigma2[0]), wl.seed, 0, n=64)
    t0 = time.perf_counter()
    oracle.gmi(y, tx, f.X, f.labels, float(wl.sigma2[0]))
    per_sample = max((time.perf_counter() - t0) / 64, 1e-7)
    n_cpu = int(max(64, min(200_000, target_s / per_sample / len(wl.snr_db))))
    elapsed = 0.0
    for q, s2 in enumerate(wl.sigma2):
        y, tx = w.channel_samples(f, float(s2), wl.seed, q, n=n_cpu)
        t0 = time.perf_counter()
        oracle.gmi(y, tx, f.X, f.labels, float(s2))
        elapsed += time.perf_counter() - t0
    pairs = n_cpu * len(wl.snr_db) * f.M
    return {"value": pairs / elapsed, "unit": "sample*points/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_cpu} samples of each of the {len(wl.snr_db)} SNR points "
                      f"({pairs:.3g} sample*points, {elapsed:.1f} s, FP64, {threads} threads)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this build measures one GPU: the exact GMI/MI path has no "
                                   "multi-GPU mode here (shards would all-reduce 5 doubles per SNR)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as w
    from paper_2011_13695_amd import mdgmi

    torch.cuda.set_device(0)
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
                                "max_abs_dgmi_vs_timed_path": float(np.abs(dout[:, :2] - out[:, :2]).max())}
    achieved = pairs / (kernel_ms * 1e-3)
    line = {
        "metric": "demapped sample*points/sec at 8D M=2048 (exact)",
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
                     "frac": achieved / EXP_PEAK, "traffic": None,
                     "kernel": "k_mfma (demap + fused reduction); 1 v_exp_f32 per (sample, point)",
                     "kernel_ms": kernel_ms},
        "gmi": [float(v) for v in out[:, 0]],
        "mi": [float(v) for v in out[:, 1]],
    }
    line.update(extra)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
