"""Benchmark: batched transmission forward models (and gradients) on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision bf16x2]

One step is one pass of the whole forward path (geometry, opacity, optical
depth, depth, binning) over the batched live-point workload: 4096 models with
50-200 layers and wavenumber windows of 5000-40000 points on a 40000-point
grid, 5 absorbers with CIA and Rayleigh, 50 channels (synthetic, seeded).
Inputs are resident in device memory before the timed region.

Prints one JSON line with the throughput (spectra/s), the roofline of the
dominant kernel (timed live with HIP events on the library's stream), the
plain FP64 GPU path on the same batch, the error of sampled models against
the FP64 oracle and the oracle's own rate on the host (CPU baseline leg).
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS_TFLOPS = {"bf16x2": 2500.0, "bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--precision", default="bf16x2", choices=list(PEAKS_TFLOPS))
    p.add_argument("--models", type=int, default=4096)
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-fp64", action="store_true")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the batched "
              "path shards by model across GPUs with no exchange, which this build does "
              "not launch.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1912_07759_amd import trx
    from synth.workloads import make_config, CONFIG_NAMES

    t0 = time.time()
    tables, batch, ch = make_config(3, B=args.models)
    log(f"inputs generated in {time.time() - t0:.1f} s: B={batch.B}, W={tables.n_wn}")
    ctx = trx.Context(0)
    T = trx.Tables.from_synth(ctx, tables)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=200)
    B = batch.B
    native = torch.empty((B, tables.n_wn), dtype=torch.float64, device="cuda")
    binned = torch.empty((B, bins.n), dtype=torch.float64, device="cuda")
    status = torch.empty(B, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    def step(prec):
        return lambda: trx.forward(ctx, T, db, bins, prec, native=False, out_binned=binned,
                                   out_status=status)

    ms = time_steps(step(args.precision), args.steps, args.warmup)
    log(f"{args.precision}: {ms:.3f} ms/step")
    assert int((status != 0).sum()) == 0

    # dominant kernel, timed live with HIP events around each launch
    ctx.profile(True)
    for _ in range(args.steps):
        step(args.precision)()
    kms = {}
    for k, name in ((trx.KERNEL_GEOMETRY, "geometry"), (trx.KERNEL_FORWARD, "forward"),
                    (trx.KERNEL_BINNING, "binning")):
        tot, n = ctx.profile_read(k)
        kms[name] = tot / max(n, 1)
    ctx.profile(False)
    n_l = batch.n_layers.astype(np.float64)
    w_l = (batch.wn_hi - batch.wn_lo).astype(np.float64)
    flops = float(np.sum(n_l * (n_l + 1.0) * w_l))        # triangular dl.kappa, 2 flop/MAC
    achieved = flops / (kms["forward"] * 1e-3) / 1e12
    peak = PEAKS_TFLOPS[args.precision]
    roofline = {"bound": "mfma" if args.precision != "fp64" else "alu",
                "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None,
                "kernel": "k_fwd_mfma" if args.precision != "fp64" else "k_fwd64",
                "kernel_ms": round(kms["forward"], 4),
                "algorithmic_tflop_per_launch": round(flops / 1e12, 4)}

    # plain FP64 GPU path on the same batch (the speed-up reference)
    fp64 = None
    if not args.no_fp64 and args.precision != "fp64":
        ms64 = time_steps(step("fp64"), max(2, args.steps // 3), 1)
        fp64 = {"ms_per_step": round(ms64, 3), "spectra_per_s": round(B / (ms64 * 1e-3), 1),
                "speedup": round(ms64 / ms, 2)}
        log(f"fp64: {ms64:.3f} ms/step")

    # oracle leg: CPU baseline rate and the error stamp of sampled models
    cpu = None
    err = None
    if not args.no_cpu:
        import oracle
        from threadpoolctl import threadpool_limits
        step(args.precision)()
        torch.cuda.synchronize()
        gb = binned.cpu().numpy()
        order = np.argsort(batch.n_layers * (batch.wn_hi - batch.wn_lo))
        pick = [int(order[-1]), int(order[0])] + [int(i) for i in
                                                  np.random.default_rng(0).permutation(B)]
        done, errs, t_cpu = [], [], 0.0
        with threadpool_limits(limits=1):
            for b in pick:
                if done and t_cpu > args.cpu_seconds:
                    break
                t1 = time.perf_counter()
                r = oracle.forward_model(batch.model(b), tables, ch)
                t_cpu += time.perf_counter() - t1
                done.append(b)
                ref = r["binned"]
                ok = ~np.isnan(ref)
                errs.append(float(np.max(np.abs(gb[b][ok] - ref[ok]) / ref[ok])) if ok.any() else 0.0)
        work = float(np.sum(n_l[done] * w_l[done]))
        mean_work = float(np.mean(n_l * w_l))
        cpu = {"value": round(len(done) / t_cpu * (work / len(done)) / mean_work, 4),
               "unit": "spectra/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(done)} of {B} models (largest, smallest, then random), "
                         f"{t_cpu:.1f} s single-threaded numpy FP64, rate scaled to the "
                         f"batch's mean layers x window"}
        err = {"max_rel_err_binned": max(errs), "models_checked": len(done)}
        log(f"oracle: {len(done)} models in {t_cpu:.1f} s; max rel err {max(errs):.2e}")

    out = {"metric": "forward spectra/s at <=1e-6 rel err (batched, split-precision "
                     "matrix cores) vs plain FP64",
           "value": round(B / (ms * 1e-3), 1), "unit": "spectra/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"bf16x2": "bf16", "bf16x3": "bf16", "fp32": "f32", "fp64": "f64"}[args.precision],
           "data": "synthetic",
           "config": {"workload": CONFIG_NAMES[3], "models": B, "layers": "50-200",
                      "wavenumbers": tables.n_wn, "window": "5000-40000", "absorbers": 5,
                      "channels": bins.n, "precision": args.precision},
           "roofline": roofline, "cpu_baseline": cpu, "fp64_gpu": fp64, "error": err,
           "kernel_ms": {k: round(v, 4) for k, v in kms.items()}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
