"""Benchmark: batched transmission forward models (and gradients) on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision bf16x2]

One step is one pass of the whole forward path (geometry, opacity, optical
depth, depth, binning) over the batched live-point workload: 4096 models with
50-200 layers and wavenumber windows of 5000-40000 points on a 40000-point
grid, 5 absorbers with CIA and Rayleigh, 50 channels (synthetic, seeded).
Inputs are resident in device memory before the timed region.

Prints one JSON line with the throughput (spectra/s), the roofline of the
dominant kernel (timed live with HIP events on the library's stream), the
plain FP64 GPU path on the same batch, the error of a stratified sample of
models against the FP64 oracle and the oracle's own rate on the host's cores
(CPU baseline leg, a pool of worker processes forked before the GPU is
touched), and the other legs: chi^2 gradients (FP32 forward, FP64 forward as
a second figure), emission spectra, single-model latencies, cloud decks, a
synthetic retrieval and the large workload.
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
    p.add_argument("--cpu-seconds", type=float, default=30.0,
                   help="budget of single-process oracle work (large workload checks)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--variant", default=None,
                   help="force a plan variant (e.g. 'persistent=1 group=32') instead of "
                        "the autotuner's choice")
    p.add_argument("--fp64-looped", type=int, default=256, metavar="M",
                   help="time the plain FP64 path one model per launch on M models "
                        "(0: skip); the rate is scaled to the batch")
    p.add_argument("--no-grad", action="store_true",
                   help="skip the gradient leg (chi^2 gradients of the 256-point workload)")
    p.add_argument("--grad-precision", default="fp32", choices=["fp32", "bf16x2", "bf16x3", "fp64"],
                   help="forward pass of the gradient leg (FP64 is always timed as well)")
    p.add_argument("--no-emission", action="store_true", help="skip the emission leg")
    p.add_argument("--emission-precision", default="fp32", choices=["fp32", "bf16x2", "bf16x3", "fp64"],
                   help="the emission leg's fast mode (FP64 is always timed as well)")
    p.add_argument("--no-exp-t", action="store_true",
                   help="skip the leg with the exponential temperature scheme")
    p.add_argument("--no-two-layer", action="store_true",
                   help="skip the leg with two-layer mixing profiles")
    p.add_argument("--no-clouds", action="store_true",
                   help="skip the leg with cloud decks on the main batch")
    p.add_argument("--no-retrieval", action="store_true",
                   help="skip the synthetic nested-sampling retrieval")
    p.add_argument("--no-single", action="store_true",
                   help="skip the single-model leg (one model per graph replay)")
    p.add_argument("--no-large", action="store_true",
                   help="skip the large workload (1024 models of 100-200 layers, 10 absorbers, "
                        "40 x 30 x 100000 tables): split-bf16 forward and gradients")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="also run one plain device copy of this many MiB (reference "
                        "for the HBM byte counters of a profiler run)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# the oracle on the host's cores: worker processes forked before the GPU is
# initialised, the workload arrays shared with them copy-on-write
# ---------------------------------------------------------------------------
_SHARED = {}


def pool_size():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _ping(_):
    return os.getpid()


def _oracle_task(job):
    """One oracle evaluation in a worker (one BLAS thread), with its wall
    interval and its own duration."""
    import oracle
    from threadpoolctl import threadpool_limits
    kind, b, extra = job
    with threadpool_limits(limits=1):
        t0 = time.time()
        p0 = time.perf_counter()
        if kind in ("forward", "clouds", "exp_t", "two_layer"):
            tables, batch, ch = _SHARED["cfg3"]
            src = {"clouds": "cfg3_clouds", "two_layer": "cfg3_two_layer"}.get(kind)
            m = (_SHARED[src] if src else batch).model(b)
            if kind == "exp_t":
                m = dict(m, t_interp="exp")
            r = oracle.forward_model(m, tables, ch)
            out = (r["depth"], r["binned"])
        elif kind == "emission":
            tables, batch, ch = _SHARED["cfg3"]
            r = oracle.emission_model(batch.model(b), tables, ch, n_mu=extra[0],
                                      T_star=float(_SHARED["T_star"][b]))
            out = (r["fpfs"], r["binned"])
        else:   # gradient
            tables, batch, ch = _SHARED["cfg4"]
            obs, sigma = extra
            g = oracle.chi2_and_grad(batch.model(b), tables, ch, obs, sigma)
            out = (g["dT"], g["dlog10_vmr"], g["dRp"], g["chi2"])
        dt = time.perf_counter() - p0
    return b, out, t0, time.time(), dt


def run_oracle(pool, kind, picks, extra=None):
    """Results by model index, the wall time of the pool (first start to
    last end) and the summed per-model time."""
    res = list(pool.map(_oracle_task, [(kind, int(b), extra) for b in picks], chunksize=1))
    wall = max(r[3] for r in res) - min(r[2] for r in res)
    return {r[0]: r[1] for r in res}, wall, sum(r[4] for r in res)


def stratified(batch, k, seed):
    """Models spread evenly over the batch's work (layers x window) ranks,
    the largest and the smallest included, about k of them."""
    work = batch.n_layers.astype(np.float64) * (batch.wn_hi - batch.wn_lo)
    order = np.argsort(work, kind="stable")
    ranks = np.unique(np.linspace(0, batch.B - 1, min(k, batch.B)).round().astype(int))
    pick = [int(order[-1]), int(order[0])] + [int(order[r]) for r in ranks]
    return list(dict.fromkeys(pick))


def rel_err(g, r):
    g, r = np.asarray(g), np.asarray(r)
    ok = ~np.isnan(r)
    if not ok.any():
        return 0.0
    if not np.all(np.isfinite(g[ok])):
        return float("inf")
    return float(np.max(np.abs(g[ok] - r[ok]) / np.abs(r[ok])))


def grad_err(v, r):
    """Norm-wise and per-component (components above 1e-3 of the largest)."""
    big = np.abs(r) >= 1e-3 * np.max(np.abs(r))
    return max(np.linalg.norm(v - r) / np.linalg.norm(r),
               float(np.max(np.abs(v[big] - r[big]) / np.abs(r[big]))))


# ---------------------------------------------------------------------------
# helpers on the GPU side
# ---------------------------------------------------------------------------
def traffic_of(kernel, precision):
    """HBM bytes per launch of `kernel` from the committed profiler summary,
    if it was taken on the current source of the kernel, else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_bytes_{kernel}_{precision}_batched4096.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in fields.get("sources", "").split():
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if not fields.get("sources") or h.hexdigest() != fields.get("sources_sha256"):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def observation(ctx, trx, T, bins, batch, cfg, n_layers, n_ch):
    """The synthetic observation of a gradient workload: the library's FP64
    binned spectrum of point 0 plus seeded 50 ppm noise (the oracle only
    checks)."""
    from synth.workloads import observation_noise
    one = trx.DeviceBatch.from_synth(batch.subset([0]), max_layers=n_layers)
    _, tb, st = trx.forward(ctx, T, one, bins, "fp64", native=False)
    assert int(st[0]) == 0
    noise, sigma = observation_noise(cfg, 1, n_ch)
    return np.tile(tb[0].cpu().numpy() + noise[0], (batch.B, 1)), sigma


def kernel_times(ctx, trx, fn, reps, classes):
    ctx.profile(True)
    for _ in range(reps):
        fn()
    out = {}
    for k, name in classes:
        tot, n = ctx.profile_read(k)
        out[name] = round(tot / max(n, 1), 4)
    ctx.profile(False)
    return out


def step_stats(fn, steps):
    """Median and quartiles (ms) of `steps` launches, each between its own
    pair of events on the current stream."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for s, e in ev:
        s.record()
        fn()
        e.record()
    torch.cuda.synchronize()
    t = np.array([s.elapsed_time(e) for s, e in ev])
    return float(np.median(t)), float(np.percentile(t, 25)), float(np.percentile(t, 75))


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


# ---------------------------------------------------------------------------
# legs
# ---------------------------------------------------------------------------
def gradient_leg(args, ctx, trx, torch, pool):
    """chi^2 gradients of 256 parameter points (100-layer perturbed Guillot
    profiles, 7 absorbers, 50000-point tables, 100 channels, 50 ppm noise on
    the truth's binned spectrum) from one graph-captured gradient plan, with
    the workload's FP32 forward (--grad-precision) and, as a second figure,
    the FP64 forward; every point against the oracle's reference gradient."""
    tables, batch, ch = _SHARED["cfg4"]
    T = trx.Tables.from_synth(ctx, tables)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=100)
    B = batch.B
    obs, sigma = observation(ctx, trx, T, bins, batch, 4, 100, bins.n)
    res = None
    for prec in dict.fromkeys([args.grad_precision, "fp64"]):
        plan = trx.Plan(ctx, T, bins, B_max=B, N_max=100, precision=prec, graph=True, grad=True)
        plan.autotune(db)
        ms = time_steps(lambda: plan.launch_grad(db, obs, sigma), args.steps, args.warmup)
        out = plan.launch_grad(db, obs, sigma)
        torch.cuda.synchronize()
        assert int((out["status"] != 0).sum()) == 0
        kms = kernel_times(ctx, trx, lambda: plan.launch_grad(db, obs, sigma), max(2, args.steps // 3),
                           ((trx.KERNEL_FORWARD, "forward"), (trx.KERNEL_ADJOINT, "adjoint_item"),
                            (trx.KERNEL_GEOM_ADJ, "chi2_and_geometry_adjoint")))
        log(f"gradient ({prec} forward): {ms:.3f} ms/step ({B / (ms * 1e-3):.1f} evals/s)")
        g = {k: v.cpu().numpy().copy() for k, v in out.items()}
        variant = plan.describe()
        plan.close()
        if res is None:
            res = {"metric": "gradient evals/s", "value": round(B / (ms * 1e-3), 1),
                   "unit": "gradient evals/s", "ms_per_step": round(ms, 3),
                   "precision": prec, "kernel_ms": kms,
                   "config": {"workload": "gradient-256-100L-7abs-50kwn", "models": B, "layers": 100,
                              "absorbers": tables.n_abs, "wavenumbers": tables.n_wn,
                              "channels": bins.n, "noise_ppm": 50, "variant": variant}}
            g_main = g
        else:
            res["fp64_forward"] = {"ms_per_step": round(ms, 3), "value": round(B / (ms * 1e-3), 1),
                                   "kernel_ms": kms}
            g_64 = g
    if pool is not None:
        refs, wall, cpu = run_oracle(pool, "gradient", range(B), (obs[0], sigma))
        off = batch.layer_off
        errs, errs64 = [], []
        for b in range(B):
            dT, dv, dR, c2 = refs[b]
            r = np.concatenate([dT, dv, [dR]])
            for gg, lst in ((g_main, errs), (g_64 if args.grad_precision != "fp64" else g_main, errs64)):
                v = np.concatenate([gg["dT"][off[b]:off[b + 1]], gg["dlog10_vmr"][b], [gg["dRp"][b]]])
                lst.append(grad_err(v, r))
        res["error"] = {"max_rel_err_gradient": max(errs), "median_rel_err_gradient": float(np.median(errs)),
                        "models_checked": B}
        if "fp64_forward" in res:
            res["fp64_forward"]["max_rel_err_gradient"] = max(errs64)
        n = pool_size()
        res["cpu_baseline"] = {"value": round(B / wall, 3), "unit": "gradient evals/s", "cores": n,
                               "kind": "oracle", "single_core_value": round(B / cpu, 4),
                               "cpu_model": cpu_model(),
                               "sample": f"all {B} points, numpy FP64 reverse mode, {n} worker "
                                         f"processes of one thread ({wall:.1f} s wall, {cpu:.1f} s "
                                         f"of single-thread work)"}
        log(f"gradient oracle: {B} points in {wall:.1f} s on {n} processes; max err {max(errs):.2e} "
            f"({args.grad_precision}), {max(errs64):.2e} (fp64)")
    bins.close()
    T.close()
    return res


def emission_leg(args, ctx, trx, torch, T, bins, tables, batch, db, pool):
    """Emission spectra (F_p/F_s, 4 Gauss-Legendre angles, a blackbody star
    per model) of the main batch from one graph-captured emission plan, and
    the same with the FP64 path; stratified models against the oracle."""
    B = batch.B
    T_star = _SHARED["T_star"]
    res = {}
    for prec in dict.fromkeys([args.emission_precision, "fp64"]):
        pe = trx.Plan(ctx, T, bins, B_max=B, N_max=200, precision=prec, graph=True, emission=True)
        pe.set_star(T_star, n_mu=4)
        pe.autotune(db)
        ms = time_steps(lambda: pe.launch(db), max(2, args.steps // (1 if prec != "fp64" else 3)), 1)
        nat, binned, st = pe.launch(db, native=True)
        torch.cuda.synchronize()
        assert int((st != 0).sum()) == 0
        kms = kernel_times(ctx, trx, lambda: pe.launch(db), 2, ((trx.KERNEL_FORWARD, "forward"),))
        log(f"emission {prec}: {ms:.3f} ms/step")
        entry = {"ms_per_step": round(ms, 3), "spectra_per_s": round(B / (ms * 1e-3), 1),
                 "kernel_ms": kms, "variant": pe.describe()}
        if pool is not None:
            picks = stratified(batch, 64, 9)
            refs, _, _ = run_oracle(pool, "emission", picks, (4,))
            gn = nat[picks].cpu().numpy()
            gb = binned[picks].cpu().numpy()
            en, eb = [], []
            for i, b in enumerate(picks):
                lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
                en.append(rel_err(gn[i, lo:hi], refs[b][0]))
                eb.append(rel_err(gb[i], refs[b][1]))
            entry["error"] = {"max_rel_err_native": max(en), "median_rel_err_native": float(np.median(en)),
                              "max_rel_err_binned": max(eb), "models_checked": len(picks)}
            log(f"emission {prec} oracle: {len(picks)} models, native {max(en):.2e}, binned {max(eb):.2e}")
        res[prec] = entry
        pe.close()
    ep = args.emission_precision
    out = dict(res[ep])
    out.update({"precision": ep, "n_mu": 4, "star": "blackbody, 4500-6500 K per model"})
    if "fp64" in res and ep != "fp64":
        out["fp64_gpu"] = res["fp64"]
        out["speedup_vs_fp64_batched"] = round(res["fp64"]["ms_per_step"] / res[ep]["ms_per_step"], 2)
    return out


def exp_t_leg(args, ctx, trx, torch, tables, bins_lin, batch, db, ch, pool):
    """The main batch over the same tables in the exponential temperature
    scheme (sigma = a e^{-b/T} between the T nodes): one graph-captured plan
    in the main precision and the FP64 path; stratified models against the
    oracle in that scheme."""
    B = batch.B
    Tx = trx.Tables.from_synth(ctx, tables, "exp")
    bx = trx.Bins(ctx, Tx, ch.lo, ch.hi)
    res = {}
    for prec in dict.fromkeys([args.precision, "fp64"]):
        px = trx.Plan(ctx, Tx, bx, B_max=B, N_max=200, precision=prec, graph=True)
        px.autotune(db)
        ms = time_steps(lambda: px.launch(db), max(2, args.steps // (1 if prec != "fp64" else 3)), 1)
        nat, binned, st = px.launch(db, native=True)
        torch.cuda.synchronize()
        assert int((st != 0).sum()) == 0
        kms = kernel_times(ctx, trx, lambda: px.launch(db), 2, ((trx.KERNEL_FORWARD, "forward"),))
        log(f"exp-T {prec}: {ms:.3f} ms/step")
        entry = {"ms_per_step": round(ms, 3), "spectra_per_s": round(B / (ms * 1e-3), 1),
                 "kernel_ms": kms, "variant": px.describe()}
        if pool is not None and prec != "fp64":
            picks = stratified(batch, 64, 11)
            refs, _, _ = run_oracle(pool, "exp_t", picks)
            gn = nat[picks].cpu().numpy()
            gb = binned[picks].cpu().numpy()
            en, eb = [], []
            for i, b in enumerate(picks):
                lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
                en.append(rel_err(gn[i, lo:hi], refs[b][0]))
                eb.append(rel_err(gb[i], refs[b][1]))
            entry["error"] = {"max_rel_err_native": max(en), "median_rel_err_native": float(np.median(en)),
                              "max_rel_err_binned": max(eb), "models_checked": len(picks)}
            log(f"exp-T {prec} oracle: {len(picks)} models, native {max(en):.2e}, binned {max(eb):.2e}")
        res[prec] = entry
        del nat, binned
        px.close()
    bx.close()
    Tx.close()
    out = dict(res[args.precision])
    out["precision"] = args.precision
    if "fp64" in res and args.precision != "fp64":
        out["fp64_gpu"] = res["fp64"]
        out["speedup_vs_fp64_batched"] = round(res["fp64"]["ms_per_step"] / res[args.precision]["ms_per_step"], 2)
    return out


def two_layer_leg(args, ctx, trx, torch, T, bins, pool):
    """The main batch with two-layer mixing profiles (two switch pressures
    per model, each absorber on one of them or constant: up to three runs of
    one chemistry) through a graph-captured TRX_PLAN_TWO_LAYER plan in the
    main precision; stratified models against the oracle."""
    tb = _SHARED["cfg3_two_layer"]
    db = trx.DeviceBatch.from_synth(tb, max_layers=200)
    p2 = trx.Plan(ctx, T, bins, B_max=tb.B, N_max=200, precision=args.precision, graph=True, two_layer=True)
    p2.autotune(db)
    ms = time_steps(lambda: p2.launch(db), args.steps, args.warmup)
    nat, binned, st = p2.launch(db, native=True)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    kms = kernel_times(ctx, trx, lambda: p2.launch(db), 2, ((trx.KERNEL_FORWARD, "forward"),))
    res = {"ms_per_step": round(ms, 3), "spectra_per_s": round(tb.B / (ms * 1e-3), 1), "kernel_ms": kms,
           "variant": p2.describe(), "precision": args.precision,
           "profiles": "two switch pressures per model, log-uniform in [1e-2, 1e5] Pa; each absorber on "
                       "one of them (top value 0.5-4 dex lower) or constant"}
    log(f"two-layer {args.precision}: {ms:.3f} ms/step")
    if pool is not None:
        picks = stratified(tb, 64, 13)
        refs, _, _ = run_oracle(pool, "two_layer", picks)
        gn = nat[picks].cpu().numpy()
        gb = binned[picks].cpu().numpy()
        en, eb = [], []
        for i, b in enumerate(picks):
            lo, hi = int(tb.wn_lo[b]), int(tb.wn_hi[b])
            en.append(rel_err(gn[i, lo:hi], refs[b][0]))
            eb.append(rel_err(gb[i], refs[b][1]))
        res["error"] = {"max_rel_err_native": max(en), "median_rel_err_native": float(np.median(en)),
                        "max_rel_err_binned": max(eb), "models_checked": len(picks)}
        log(f"two-layer oracle: {len(picks)} models, native {max(en):.2e}, binned {max(eb):.2e}")
    del nat, binned
    p2.close()
    return res


def large_leg(args, ctx, trx, torch):
    """The large workload: 1024 models of 100-200 layers, 10 absorbers with
    CIA and Rayleigh on 40 T x 30 P x 100000-point tables, 100 channels.  The
    split-bf16 forward, and the chi^2 gradients (recompute mode) with the
    split-bf16 and with the FP64 forward, one graph-captured plan each; the
    device memory in use with each gradient plan; the forward of two models
    and the gradient of point 0 against the oracle (in this process, within
    --cpu-seconds)."""
    from synth.workloads import make_config
    t0 = time.time()
    tables, batch, ch = make_config(5)
    B = batch.B
    log(f"large inputs generated in {time.time() - t0:.1f} s: B={B}, W={tables.n_wn}")
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    T = trx.Tables.from_synth(ctx, tables)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=200)
    pf = trx.Plan(ctx, T, bins, B_max=B, N_max=200, precision="bf16x2", graph=True)
    pf.autotune(db)
    ms_f = time_steps(lambda: pf.launch(db), args.steps, args.warmup)
    nat, binned, st = pf.launch(db, native=True)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    log(f"large forward bf16x2: {ms_f:.3f} ms/step")
    obs, sigma = observation(ctx, trx, T, bins, batch, 5, 200, bins.n)
    res = {"forward_ms_per_step": round(ms_f, 3), "forward_spectra_per_s": round(B / (ms_f * 1e-3), 1),
           "forward_precision": "bf16x2", "forward_variant": pf.describe(),
           "config": {"workload": "batched-grad-1024-100to200L-10abs-100000wn", "models": B,
                      "layers": "100-200", "absorbers": tables.n_abs, "wavenumbers": tables.n_wn,
                      "table_grid": [len(tables.T_grid), len(tables.log10P_grid)],
                      "channels": bins.n}}
    import oracle
    from threadpoolctl import threadpool_limits
    t_cpu = 0.0
    if not args.no_cpu:
        order = np.argsort(batch.n_layers * (batch.wn_hi - batch.wn_lo))
        errs = []
        with threadpool_limits(limits=1):
            for b in (int(order[-1]), int(order[0])):
                t1 = time.perf_counter()
                r = oracle.forward_model(batch.model(b), tables, ch)
                t_cpu += time.perf_counter() - t1
                lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
                errs += [rel_err(nat[b, lo:hi].cpu().numpy(), r["depth"]),
                         rel_err(binned[b].cpu().numpy(), r["binned"])]
        res["forward_error"] = {"max_rel_err": max(errs), "models_checked": 2}
        log(f"large forward oracle: 2 models in {t_cpu:.1f} s, max err {max(errs):.2e}")
    del nat
    pf.close()
    for prec in ("bf16x2", "fp64"):
        pg = trx.Plan(ctx, T, bins, B_max=B, N_max=200, precision=prec, graph=True, grad=True)
        ms_g = time_steps(lambda: pg.launch_grad(db, obs, sigma), max(2, args.steps // 3), 1)
        out = pg.launch_grad(db, obs, sigma)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        n_bad = int((out["status"] != 0).sum())
        kms = kernel_times(ctx, trx, lambda: pg.launch_grad(db, obs, sigma), 1,
                           ((trx.KERNEL_GEOMETRY, "geometry"), (trx.KERNEL_FORWARD, "forward"),
                            (trx.KERNEL_ADJOINT, "adjoint_item"),
                            (trx.KERNEL_GEOM_ADJ, "chi2_and_geometry_adjoint")))
        log(f"large gradient ({prec} forward): {ms_g:.3f} ms/step, {n_bad} points flagged")
        gr = {"ms_per_step": round(ms_g, 3), "evals_per_s": round(B / (ms_g * 1e-3), 1),
              "forward_precision": prec, "points_unsupported": n_bad, "kernel_ms": kms,
              "device_memory_gb": round((free0 - free1) / 1e9, 2)}
        if not args.no_cpu and t_cpu < args.cpu_seconds:
            g = {k: v.cpu().numpy() for k, v in out.items()}
            off = batch.layer_off
            with threadpool_limits(limits=1):
                t1 = time.perf_counter()
                ref = oracle.chi2_and_grad(batch.model(0), tables, ch, obs[0], sigma)
                t_cpu += time.perf_counter() - t1
            v = np.concatenate([g["dT"][off[0]:off[1]], g["dlog10_vmr"][0], [g["dRp"][0]]])
            r = np.concatenate([ref["dT"], ref["dlog10_vmr"], [ref["dRp"]]])
            gr["error"] = {"max_rel_err_gradient": grad_err(v, r), "models_checked": 1,
                           "point": "0 (residual at the noise level)"}
            log(f"large gradient oracle ({prec}): point 0, err {gr['error']['max_rel_err_gradient']:.2e}")
        res["gradient_" + prec] = gr
        pg.close()
    bins.close()
    T.close()
    return res


def single_leg(args, ctx, trx, torch):
    """One model per launch, each launch one replay of the plan's graph, back
    to back: the plain model (100 isothermal layers, one absorber, 2000
    points, native depth) in FP64, and the 5-absorber Guillot model on 40000
    points binned to 50 channels in FP32 (P in hi + lo), split-bf16 and
    FP64.  These are single-model latencies: one model does not fill the
    GPU."""
    from synth.workloads import make_config, CONFIG_NAMES
    res = {}
    for cfg, precs in ((1, ("fp64",)), (2, ("fp32", "bf16x2", "fp64"))):
        tables, batch, ch = make_config(cfg)
        T = trx.Tables.from_synth(ctx, tables)
        bins = trx.Bins(ctx, T, ch.lo, ch.hi) if ch is not None else None
        db = trx.DeviceBatch.from_synth(batch, max_layers=100)
        ref = None
        if not args.no_cpu:
            import oracle
            ref = oracle.forward_model(batch.model(0), tables, ch)
        for prec in precs:
            plan = trx.Plan(ctx, T, bins, B_max=1, N_max=100, precision=prec, graph=True)
            plan.autotune(db)
            native = bins is None
            fn = lambda: plan.launch(db, native=native, binned=not native)
            us = time_steps(fn, 200, 20) * 1e3
            nat, binned, st = fn()
            torch.cuda.synchronize()
            assert int(st[0]) == 0
            entry = {"us_per_model": round(us, 2), "spectra_per_s": round(1e6 / us, 1),
                     "variant": plan.describe()}
            if ref is not None:
                if native:
                    entry["max_rel_err_native"] = rel_err(nat[0].cpu().numpy(), ref["depth"])
                else:
                    entry["max_rel_err_binned"] = rel_err(binned[0].cpu().numpy(), ref["binned"])
            res[f"{CONFIG_NAMES[cfg]}:{prec}"] = entry
            log(f"single {CONFIG_NAMES[cfg]} {prec}: {us:.1f} us/model")
            plan.close()
        if bins is not None:
            bins.close()
        T.close()
    return res


def clouds_leg(args, plan, trx, torch, pool):
    """The main batch with a flat-opacity cloud deck on two thirds of the
    models (a third finite decks, a third opaque), through the same plan;
    four models of each kind against the oracle."""
    cb = _SHARED["cfg3_clouds"]
    dbc = trx.DeviceBatch.from_synth(cb, max_layers=200)
    ms = time_steps(lambda: plan.launch(dbc), args.steps, args.warmup)
    _, binned, status = plan.launch(dbc)
    torch.cuda.synchronize()
    assert int((status != 0).sum()) == 0
    res = {"ms_per_step": round(ms, 3), "spectra_per_s": round(cb.B / (ms * 1e-3), 1),
           "decks": "one third none, one third finite (log10 sigma in [-32, -27] m^2), "
                    "one third opaque"}
    if pool is not None:
        picks = list(range(12))
        refs, _, _ = run_oracle(pool, "clouds", picks)
        gb = binned[picks].cpu().numpy()
        errs = [rel_err(gb[i], refs[b][1]) for i, b in enumerate(picks)]
        res.update({"max_rel_err_binned": max(errs), "models_checked": len(picks)})
        log(f"clouds: {ms:.3f} ms/step; max rel err {max(errs):.2e}")
    return res


def retrieval_leg(args, ctx, T, bins, tables, ch, trx, torch):
    """The paper's transit retrieval on synthetic data: 5 log abundances, an
    isothermal T, Rp and the top of an opaque cloud deck, uniform priors; the
    observation is the library's FP64 binned spectrum of the truth (100
    layers, the whole 40000-point grid) plus seeded 50 ppm noise;
    multi-ellipsoid nested sampling with candidates evaluated 2048 per plan
    launch (two plans alternating)."""
    from paper_1912_07759_amd.retrieval import (LikelihoodBudgetExhausted, TransitRetrieval,
                                                nested_sample, posterior)
    from synth.constants import GM_JUP, R_SUN
    from synth.workloads import observation_noise
    N = 100
    truth = np.array([-3.5, -6.0, -5.0, -7.0, -8.0, 1200.0, 1.35, 3.0])
    na = tables.n_abs
    one = trx.DeviceBatch([N], np.full(N, truth[na]), [1e6], [1e-4], truth[None, :na],
                          [truth[na + 1] * TransitRetrieval.R_JUP], [R_SUN], [GM_JUP], [0],
                          [tables.n_wn], max_layers=N, cloud_sigma=[np.inf],
                          cloud_p_top=[10.0 ** truth[na + 2]], cloud_p_bottom=[1e6])
    _, tb, st = trx.forward(ctx, T, one, bins, "fp64", native=False)
    assert int(st[0]) == 0
    noise, sigma = observation_noise(3, 1, len(ch.lo))
    obs = tb[0].cpu().numpy() + noise[0]
    ret = TransitRetrieval(ctx, T, bins, obs, sigma, tables.names, R_SUN, GM_JUP, n_layers=N,
                           B_max=2048, precision=args.precision)
    try:
        # capture both alternating plans' graphs outside the timing
        for _ in range(2):
            ret(np.full((4, len(ret.priors)), 0.5))
        torch.cuda.synchronize()
        ret.n_eval = ret.n_launch = 0
        ret.wait_seconds = 0.0
        try:
            r = nested_sample(ret, len(ret.priors), n_live=200, batch=2048, dlogz=0.5, seed=1)
        except LikelihoodBudgetExhausted as e:
            log(f"retrieval: {e}")
            return {"error": str(e)}
    finally:
        ret.close()
    _, mean, std = posterior(r, ret.priors)
    names = [p.name for p in ret.priors]
    log(f"retrieval: {r['n_eval']} likelihoods in {r['seconds']:.1f} s "
        f"({ret.n_launch} launches, host waited {ret.wait_seconds:.1f} s), logz {r['logz']:.2f}")
    return {"seconds": round(r["seconds"], 2), "likelihood_evals": int(r["n_eval"]),
            "launches": int(ret.n_launch), "host_wait_seconds": round(ret.wait_seconds, 2),
            "likelihoods_per_s": round(r["n_eval"] / r["seconds"], 1),
            "iterations": int(r["n_iter"]), "n_live": 200,
            "logz": round(r["logz"], 3), "logz_err": round(r["logz_err"], 3),
            "truth": dict(zip(names, truth.tolist())),
            "posterior_mean": dict(zip(names, np.round(mean, 4).tolist())),
            "posterior_std": dict(zip(names, np.round(std, 4).tolist())),
            "config": "5 log abundances, isothermal T, Rp, opaque cloud-deck top; 100 layers, "
                      "40000 points, 50 channels, 50 ppm noise"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the batched "
              "path shards by model across GPUs with no exchange, which this benchmark does "
              "not launch.", file=sys.stderr)
        sys.exit(2)
    from synth.workloads import (CONFIG_NAMES, make_config, stellar_temperatures, with_cloud_decks,
                                 with_two_layer_profiles)

    # host inputs, then the oracle's worker pool, before anything touches the GPU
    t0 = time.time()
    tables, batch, ch = make_config(3, B=args.models)
    _SHARED["cfg3"] = (tables, batch, ch)
    _SHARED["cfg3_clouds"] = with_cloud_decks(batch, 5)
    _SHARED["cfg3_two_layer"] = with_two_layer_profiles(batch, 6)
    _SHARED["T_star"] = stellar_temperatures(batch.B)
    if not args.no_grad:
        _SHARED["cfg4"] = make_config(4)
    log(f"inputs generated in {time.time() - t0:.1f} s: B={batch.B}, W={tables.n_wn}")
    pool = None
    if not args.no_cpu:
        import multiprocessing
        from concurrent.futures import ProcessPoolExecutor
        n = pool_size()
        pool = ProcessPoolExecutor(max_workers=n, mp_context=multiprocessing.get_context("fork"))
        list(pool.map(_ping, range(4 * n)))     # every worker forked now

    import torch
    from paper_1912_07759_amd import trx

    ctx = trx.Context(0)
    T = trx.Tables.from_synth(ctx, tables)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=200)
    B = batch.B
    torch.cuda.synchronize()

    # the batched launch: one graph-captured plan, variant autotuned on this batch
    plan = trx.Plan(ctx, T, bins, B_max=B, N_max=200, precision=args.precision, graph=True)
    t1 = time.time()
    if args.variant:
        plan.set_variant(args.variant)
    else:
        plan.autotune(db)
    variant = plan.describe()
    log(f"variant {variant} ({time.time() - t1:.1f} s)")

    def step():
        plan.launch(db)

    ms = time_steps(step, args.steps, args.warmup)
    log(f"{args.precision}: {ms:.3f} ms/step")
    _, binned, status = plan.launch(db)
    torch.cuda.synchronize()
    assert int((status != 0).sum()) == 0
    med, q1, q3 = step_stats(step, args.steps)

    # dominant kernel, timed live with HIP events around each launch on the
    # library's stream (the plan launches its kernels one by one meanwhile)
    kms = kernel_times(ctx, trx, step, args.steps,
                       ((trx.KERNEL_GEOMETRY, "geometry"), (trx.KERNEL_SCHEDULE, "schedule"),
                        (trx.KERNEL_FORWARD, "forward"), (trx.KERNEL_BINNING, "binning")))
    n_l = batch.n_layers.astype(np.float64)
    w_l = (batch.wn_hi - batch.wn_lo).astype(np.float64)
    flops = float(np.sum(n_l * (n_l + 1.0) * w_l))        # triangular dl.kappa, 2 flop/MAC
    achieved = flops / (kms["forward"] * 1e-3) / 1e12
    peak = PEAKS_TFLOPS[args.precision]
    kname = {"fp64": "k_fwd64"}.get(args.precision,
                                    "k_fwd_mfma_persist" if "persistent=1" in variant
                                    else "k_fwd_mfma")
    # the interpolation's compulsory HBM bytes: every FP32 table value once
    # (cross-sections, CIA, Rayleigh), against the forward kernel's time
    esz = 8 if args.precision == "fp64" else 4
    table_bytes = esz * (tables.xsec.size + tables.cia.size
                         + (tables.rayleigh.size if tables.rayleigh is not None else 0))
    interp_gbs = table_bytes / (kms["forward"] * 1e-3) / 1e9
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": traffic_of(kname, args.precision),
                "kernel": kname, "kernel_ms": round(kms["forward"], 4),
                "algorithmic_tflop_per_launch": round(flops / 1e12, 4),
                "interp_hbm": {"compulsory_bytes": table_bytes, "achieved_gbs": round(interp_gbs, 2),
                               "peak_gbs": HBM_PEAK_GBS, "frac": round(interp_gbs / HBM_PEAK_GBS, 5)}}

    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # plain FP64 GPU path on the same batch: batched (one graph) and looped
    # (one model per launch), separating the batching gain from precision
    fp64 = None
    if not args.no_fp64 and args.precision != "fp64":
        p64 = trx.Plan(ctx, T, bins, B_max=B, N_max=200, precision="fp64", graph=True)
        ms64 = time_steps(lambda: p64.launch(db), max(2, args.steps // 3), 1)
        p64.close()
        fp64 = {"batched_ms_per_step": round(ms64, 3),
                "batched_spectra_per_s": round(B / (ms64 * 1e-3), 1),
                "speedup_vs_batched": round(ms64 / ms, 2)}
        log(f"fp64 batched: {ms64:.3f} ms/step")
        if args.fp64_looped > 0:
            M = min(args.fp64_looped, B)
            pick = np.random.default_rng(1).permutation(B)[:M]
            one = trx.Plan(ctx, T, bins, B_max=1, N_max=200, precision="fp64", graph=False,
                           persistent=False)
            views = [db.view(int(b)) for b in pick]
            for v in views[:4]:
                one.launch(v)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for v in views:
                one.launch(v)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t1
            one.close()
            work = float(np.sum(n_l[pick] * w_l[pick]))
            rate = M / sec * (work / M) / float(np.mean(n_l * w_l))
            fp64.update({"looped_spectra_per_s": round(rate, 1),
                         "looped_sample": f"{M} random models, one launch each, rate scaled to "
                                          f"the batch's mean layers x window",
                         "speedup_vs_looped": round(B / (ms * 1e-3) / rate, 2)})
            log(f"fp64 looped: {rate:.1f} spectra/s")

    # oracle leg: the error stamp of a stratified sample of at least 256
    # models (native and binned) and the CPU baseline on the host's cores
    cpu = err = None
    if pool is not None:
        picks = stratified(batch, 256, 0)
        refs, wall, cpu_s = run_oracle(pool, "forward", picks)
        nat, _, _ = plan.launch(db, native=True)
        gn = nat[picks].cpu().numpy()
        del nat
        gb = binned[picks].cpu().numpy()
        en, eb = [], []
        for i, b in enumerate(picks):
            lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
            en.append(rel_err(gn[i, lo:hi], refs[b][0]))
            eb.append(rel_err(gb[i], refs[b][1]))
        work = float(np.sum(n_l[picks] * w_l[picks]))
        scale = (work / len(picks)) / float(np.mean(n_l * w_l))
        n = pool_size()
        cpu = {"value": round(len(picks) / wall * scale, 3), "unit": "spectra/s", "cores": n,
               "kind": "oracle", "single_core_value": round(len(picks) / cpu_s * scale, 4),
               "cpu_model": cpu_model(),
               "sample": f"{len(picks)} of {B} models spread over the work ranks (largest and "
                         f"smallest included), numpy FP64 in {n} worker processes of one thread: "
                         f"{wall:.1f} s wall, {cpu_s:.1f} s of single-thread work; rates scaled "
                         f"to the batch's mean layers x window"}
        err = {"max_rel_err_native": max(en), "max_rel_err_binned": max(eb),
               "median_rel_err_native": float(np.median(en)), "models_checked": len(picks)}
        log(f"oracle: {len(picks)} models in {wall:.1f} s on {n} processes ({cpu_s:.1f} s of work); "
            f"max rel err native {max(en):.2e}, binned {max(eb):.2e}")

    grad = None if args.no_grad else gradient_leg(args, ctx, trx, torch, pool)
    emission = None if args.no_emission else emission_leg(args, ctx, trx, torch, T, bins, tables,
                                                          batch, db, pool)
    clouds = None if args.no_clouds else clouds_leg(args, plan, trx, torch, pool)
    exp_t = None if args.no_exp_t else exp_t_leg(args, ctx, trx, torch, tables, bins, batch, db, ch, pool)
    two_layer = None if args.no_two_layer else two_layer_leg(args, ctx, trx, torch, T, bins, pool)
    single = None if args.no_single else single_leg(args, ctx, trx, torch)
    if pool is not None:
        pool.shutdown()
    retrieval = None if args.no_retrieval else retrieval_leg(args, ctx, T, bins, tables, ch, trx, torch)
    plan.close()
    bins.close()
    T.close()
    large = None if args.no_large else large_leg(args, ctx, trx, torch)

    out = {"metric": "forward spectra/s and gradient evals/s at ≤1e-6 rel err, batched vs "
                     "plain FP64",
           "value": round(B / (ms * 1e-3), 1), "unit": "spectra/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"bf16x2": "bf16", "bf16x3": "bf16", "fp32": "f32", "fp64": "f64"}[args.precision],
           "data": "synthetic",
           "config": {"workload": CONFIG_NAMES[3], "models": B, "layers": "50-200",
                      "wavenumbers": tables.n_wn, "window": "5000-40000", "absorbers": 5,
                      "channels": len(ch.lo), "precision": args.precision,
                      "launch": "hip graph of one plan", "variant": variant},
           "roofline": roofline, "cpu_baseline": cpu, "fp64_gpu": fp64, "error": err,
           "ms_per_step_median": round(med, 3), "ms_per_step_iqr": [round(q1, 3), round(q3, 3)],
           "kernel_ms": {k: round(v, 4) for k, v in kms.items()}, "gradient": grad,
           "emission": emission, "exp_t": exp_t, "two_layer": two_layer, "single_model": single,
           "clouds": clouds,
           "retrieval": retrieval,
           "large": large}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
