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
    p.add_argument("--variant", default=None,
                   help="force a plan variant (e.g. 'persistent=1 group=32') instead of "
                        "the autotuner's choice")
    p.add_argument("--fp64-looped", type=int, default=256, metavar="M",
                   help="time the plain FP64 path one model per launch on M models "
                        "(0: skip); the rate is scaled to the batch")
    p.add_argument("--no-grad", action="store_true",
                   help="skip the gradient leg (chi^2 gradients of the 256-point workload)")
    p.add_argument("--grad-precision", default="fp64", choices=["fp32", "bf16x2", "bf16x3", "fp64"],
                   help="forward pass of the gradient leg (the residual needs its accuracy)")
    p.add_argument("--no-clouds", action="store_true",
                   help="skip the leg with cloud decks on the main batch")
    p.add_argument("--no-retrieval", action="store_true",
                   help="skip the synthetic nested-sampling retrieval")
    p.add_argument("--no-single", action="store_true",
                   help="skip the single-model leg (one model per graph replay)")
    p.add_argument("--large", action="store_true",
                   help="also run the large workload (1024 models of 100-200 layers, 10 "
                        "absorbers, 40 x 30 x 100000 tables): split-bf16 forward and FP64-forward "
                        "gradients, with the device memory in use")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="also run one plain device copy of this many MiB (reference "
                        "for the HBM byte counters of a profiler run)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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


def observation(args, ctx, trx, T, bins, tables, batch, ch, cfg, n_layers):
    """The synthetic observation of a gradient workload: the binned spectrum of
    point 0 plus seeded 50 ppm noise.  With the oracle leg on, that spectrum
    is the oracle's (it is then also an input of the oracle's check); with
    --no-cpu it comes from the library's FP64 path and nothing is checked."""
    from synth.workloads import observation_noise
    if not args.no_cpu:
        import oracle
        truth = oracle.forward_model(batch.model(0), tables, ch)["binned"]
    else:
        one = trx.DeviceBatch.from_synth(batch.subset([0]), max_layers=n_layers)
        _, tb, _ = trx.forward(ctx, T, one, bins, "fp64", native=False)
        truth = tb[0].cpu().numpy()
    noise, sigma = observation_noise(cfg, 1, bins.n)
    return np.tile(truth + noise[0], (batch.B, 1)), sigma


def oracle_grad_check(args, batch, tables, ch, obs, sigma, g, picks):
    """Largest gradient error of the library against the oracle's reference
    gradient over the points `picks` (stopping after --cpu-seconds) and the
    oracle's single-core rate."""
    import oracle
    from threadpoolctl import threadpool_limits
    off = batch.layer_off
    errs, done, t_cpu = [], 0, 0.0
    with threadpool_limits(limits=1):
        for b in picks:
            if done and t_cpu > args.cpu_seconds:
                break
            t1 = time.perf_counter()
            ref = oracle.chi2_and_grad(batch.model(b), tables, ch, obs[b], sigma)
            t_cpu += time.perf_counter() - t1
            done += 1
            v = np.concatenate([g["dT"][off[b]:off[b + 1]], g["dlog10_vmr"][b], [g["dRp"][b]]])
            r = np.concatenate([ref["dT"], ref["dlog10_vmr"], [ref["dRp"]]])
            big = np.abs(r) >= 1e-3 * np.max(np.abs(r))
            errs.append(max(np.linalg.norm(v - r) / np.linalg.norm(r),
                            float(np.max(np.abs(v[big] - r[big]) / np.abs(r[big])))))
    return max(errs), done, t_cpu


def gradient_leg(args, ctx, trx, torch):
    """chi^2 gradients of 256 parameter points (100-layer perturbed Guillot
    profiles, 7 absorbers, 50000-point tables, 100 channels, 50 ppm noise on
    the truth's binned spectrum) from one graph-captured gradient plan."""
    from synth.workloads import make_config
    t0 = time.time()
    tables, batch, ch = make_config(4)
    log(f"gradient inputs generated in {time.time() - t0:.1f} s: B={batch.B}, W={tables.n_wn}")
    T = trx.Tables.from_synth(ctx, tables)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=100)
    B = batch.B
    obs, sigma = observation(args, ctx, trx, T, bins, tables, batch, ch, 4, 100)
    plan = trx.Plan(ctx, T, bins, B_max=B, N_max=100, precision=args.grad_precision, graph=True,
                    grad=True)
    plan.autotune(db)
    ms = time_steps(lambda: plan.launch_grad(db, obs, sigma), args.steps, args.warmup)
    out = plan.launch_grad(db, obs, sigma)
    torch.cuda.synchronize()
    assert int((out["status"] != 0).sum()) == 0
    ctx.profile(True)
    for _ in range(max(2, args.steps // 3)):
        plan.launch_grad(db, obs, sigma)
    kms = {}
    for k, name in ((trx.KERNEL_FORWARD, "forward"), (trx.KERNEL_ADJOINT, "adjoint_item"),
                    (trx.KERNEL_GEOM_ADJ, "chi2_and_geometry_adjoint")):
        tot, n = ctx.profile_read(k)
        kms[name] = round(tot / max(n, 1), 4)
    ctx.profile(False)
    res = {"metric": "gradient evals/s", "value": round(B / (ms * 1e-3), 1),
           "unit": "gradient evals/s", "ms_per_step": round(ms, 3),
           "precision": args.grad_precision, "kernel_ms": kms,
           "config": {"workload": "gradient-256-100L-7abs-50kwn", "models": B, "layers": 100,
                      "absorbers": tables.n_abs, "wavenumbers": tables.n_wn,
                      "channels": bins.n, "noise_ppm": 50, "variant": plan.describe()}}
    log(f"gradient: {ms:.3f} ms/step ({B / (ms * 1e-3):.1f} evals/s)")
    if not args.no_cpu:
        g = {k: v.cpu().numpy() for k, v in out.items()}
        worst, done, t_cpu = oracle_grad_check(args, batch, tables, ch, obs, sigma, g, range(B))
        res["error"] = {"max_rel_err_gradient": worst, "models_checked": done}
        res["cpu_baseline"] = {"value": round(done / t_cpu, 4), "unit": "gradient evals/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"first {done} of {B} points, {t_cpu:.1f} s "
                                         f"single-threaded numpy FP64 reverse mode"}
        log(f"gradient oracle: {done} points in {t_cpu:.1f} s; max err {worst:.2e}")
    plan.close()
    bins.close()
    T.close()
    return res


def large_leg(args, ctx, trx, torch):
    """The large workload: 1024 models of 100-200 layers, 10 absorbers with
    CIA and Rayleigh on 40 T x 30 P x 100000-point tables, 100 channels.  The
    split-bf16 forward, and the chi^2 gradients (recompute mode) with the FP64
    and with the split-bf16 forward, one graph-captured plan each; the device
    memory in use with each gradient plan (tables, model workspaces, partial
    sums and outputs), and the gradient error of sampled points against the
    oracle."""
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
    _, _, st = pf.launch(db)
    torch.cuda.synchronize()
    assert int((st != 0).sum()) == 0
    log(f"large forward bf16x2: {ms_f:.3f} ms/step")
    obs, sigma = observation(args, ctx, trx, T, bins, tables, batch, ch, 5, 200)
    res = {"forward_ms_per_step": round(ms_f, 3), "forward_spectra_per_s": round(B / (ms_f * 1e-3), 1),
           "forward_precision": "bf16x2", "forward_variant": pf.describe(),
           "config": {"workload": "batched-grad-1024-100to200L-10abs-100000wn", "models": B,
                      "layers": "100-200", "absorbers": tables.n_abs, "wavenumbers": tables.n_wn,
                      "table_grid": [len(tables.T_grid), len(tables.log10P_grid)],
                      "channels": bins.n}}
    # gradients with the FP64 forward (the residual at its full accuracy) and
    # with the split-bf16 forward; one plan at a time
    for prec in ("fp64", "bf16x2"):
        pg = trx.Plan(ctx, T, bins, B_max=B, N_max=200, precision=prec, graph=True, grad=True)
        ms_g = time_steps(lambda: pg.launch_grad(db, obs, sigma), max(2, args.steps // 3), 1)
        out = pg.launch_grad(db, obs, sigma)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        n_bad = int((out["status"] != 0).sum())
        ctx.profile(True)
        pg.launch_grad(db, obs, sigma)
        kms = {}
        for k, name in ((trx.KERNEL_GEOMETRY, "geometry"), (trx.KERNEL_FORWARD, "forward"),
                        (trx.KERNEL_ADJOINT, "adjoint_item"),
                        (trx.KERNEL_GEOM_ADJ, "chi2_and_geometry_adjoint")):
            tot, n = ctx.profile_read(k)
            kms[name] = round(tot / max(n, 1), 3)
        ctx.profile(False)
        log(f"large gradient ({prec} forward): {ms_g:.3f} ms/step, {n_bad} points flagged")
        gr = {"ms_per_step": round(ms_g, 3), "evals_per_s": round(B / (ms_g * 1e-3), 1),
              "forward_precision": prec, "points_unsupported": n_bad, "kernel_ms": kms,
              "device_memory_gb": round((free0 - free1) / 1e9, 2)}
        if not args.no_cpu:
            g = {k: v.cpu().numpy() for k, v in out.items()}
            order = np.argsort(batch.n_layers)
            # point 0 (whose residual is the noise), the longest and the shortest
            picks = list(dict.fromkeys([0, int(order[-1]), int(order[0])] + list(range(B))))
            worst, done, t_cpu = oracle_grad_check(args, batch, tables, ch, obs, sigma, g, picks)
            gr["error"] = {"max_rel_err_gradient": worst, "models_checked": done,
                           "oracle_seconds": round(t_cpu, 1)}
            log(f"large gradient oracle: {done} points in {t_cpu:.1f} s; max err {worst:.2e}")
        res["gradient_" + prec] = gr
        pg.close()
    pf.close()
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
                    g = nat[0].cpu().numpy()
                    entry["max_rel_err_native"] = float(np.max(np.abs(g - ref["depth"]) / ref["depth"]))
                else:
                    g = binned[0].cpu().numpy()
                    entry["max_rel_err_binned"] = float(np.max(np.abs(g - ref["binned"]) / ref["binned"]))
            res[f"{CONFIG_NAMES[cfg]}:{prec}"] = entry
            log(f"single {CONFIG_NAMES[cfg]} {prec}: {us:.1f} us/model")
            plan.close()
        if bins is not None:
            bins.close()
        T.close()
    return res


def clouds_leg(args, plan, tables, batch, ch, trx, torch):
    """The main batch with a flat-opacity cloud deck on two thirds of the
    models (a third finite decks, a third opaque), through the same plan;
    sampled models (one of each kind) against the oracle."""
    import oracle
    from synth.workloads import with_cloud_decks
    cb = with_cloud_decks(batch, 5)
    dbc = trx.DeviceBatch.from_synth(cb, max_layers=200)
    ms = time_steps(lambda: plan.launch(dbc), args.steps, args.warmup)
    _, binned, status = plan.launch(dbc)
    torch.cuda.synchronize()
    assert int((status != 0).sum()) == 0
    gb = binned.cpu().numpy()
    errs = []
    for b in (0, 1, 2, 3, 4, 5):
        ref = oracle.forward_model(cb.model(b), tables, ch)["binned"]
        ok = ~np.isnan(ref)
        errs.append(float(np.max(np.abs(gb[b][ok] - ref[ok]) / ref[ok])))
    log(f"clouds: {ms:.3f} ms/step; max rel err {max(errs):.2e}")
    return {"ms_per_step": round(ms, 3), "spectra_per_s": round(batch.B / (ms * 1e-3), 1),
            "decks": "one third none, one third finite (log10 sigma in [-32, -27] m^2), "
                     "one third opaque",
            "max_rel_err_binned": max(errs), "models_checked": len(errs)}


def retrieval_leg(args, ctx, T, bins, tables, ch, trx, torch):
    """The paper's transit retrieval on synthetic data: 5 log abundances, an
    isothermal T, Rp and the top of an opaque cloud deck, uniform priors; the
    observation is the oracle's binned spectrum of the truth (100 layers, the
    whole 40000-point grid) plus seeded 50 ppm noise; single-ellipsoid
    nested sampling with candidates evaluated 2048 per plan launch."""
    import oracle
    from paper_1912_07759_amd.retrieval import TransitRetrieval, nested_sample, posterior
    from synth.constants import GM_JUP, R_SUN
    from synth.workloads import observation_noise
    N = 100
    truth = np.array([-3.5, -6.0, -5.0, -7.0, -8.0, 1200.0, 1.35, 3.0])
    na = tables.n_abs
    m = dict(T=np.full(N, truth[na]), p_bot=1e6, p_top=1e-4, log10_vmr=truth[:na],
             Rp=truth[na + 1] * TransitRetrieval.R_JUP, Rs=R_SUN, GM=GM_JUP, wn_lo=0,
             wn_hi=tables.n_wn, he_h2=0.17, k_B=1.380649e-23, amu=1.66053906660e-27, gravity=0,
             cloud_sigma=np.inf, cloud_p_top=10.0 ** truth[na + 2], cloud_p_bottom=1e6)
    noise, sigma = observation_noise(3, 1, len(ch.lo))
    obs = oracle.forward_model(m, tables, ch)["binned"] + noise[0]
    ret = TransitRetrieval(ctx, T, bins, obs, sigma, tables.names, R_SUN, GM_JUP, n_layers=N,
                           B_max=2048, precision=args.precision)
    ret(np.full((4, len(ret.priors)), 0.5))      # graph capture outside the timing
    torch.cuda.synchronize()
    ret.n_eval = ret.n_launch = 0
    ret.wait_seconds = 0.0
    r = nested_sample(ret, len(ret.priors), n_live=200, batch=2048, dlogz=0.5, seed=1)
    _, mean, std = posterior(r, ret.priors)
    ret.close()
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the batched "
              "path shards by model across GPUs with no exchange, which this benchmark does "
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
    ctx.profile(True)
    for _ in range(args.steps):
        step()
    kms = {}
    for k, name in ((trx.KERNEL_GEOMETRY, "geometry"), (trx.KERNEL_SCHEDULE, "schedule"),
                    (trx.KERNEL_FORWARD, "forward"), (trx.KERNEL_BINNING, "binning")):
        tot, n = ctx.profile_read(k)
        kms[name] = tot / max(n, 1)
    ctx.profile(False)
    n_l = batch.n_layers.astype(np.float64)
    w_l = (batch.wn_hi - batch.wn_lo).astype(np.float64)
    flops = float(np.sum(n_l * (n_l + 1.0) * w_l))        # triangular dl.kappa, 2 flop/MAC
    achieved = flops / (kms["forward"] * 1e-3) / 1e12
    peak = PEAKS_TFLOPS[args.precision]
    kname = {"fp64": "k_fwd64"}.get(args.precision,
                                    "k_fwd_mfma_persist" if "persistent=1" in variant
                                    else "k_fwd_mfma")
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": traffic_of(kname, args.precision),
                "kernel": kname, "kernel_ms": round(kms["forward"], 4),
                "algorithmic_tflop_per_launch": round(flops / 1e12, 4)}

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

    grad = None
    if not args.no_grad:
        grad = gradient_leg(args, ctx, trx, torch)
    single = None if args.no_single else single_leg(args, ctx, trx, torch)
    large = large_leg(args, ctx, trx, torch) if args.large else None

    # oracle leg: CPU baseline rate and the error stamp of sampled models
    cpu = None
    err = None
    if not args.no_cpu:
        import oracle
        from threadpoolctl import threadpool_limits
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

    clouds = None if args.no_clouds else clouds_leg(args, plan, tables, batch, ch, trx, torch)
    retrieval = None
    if not args.no_retrieval:
        try:
            retrieval = retrieval_leg(args, ctx, T, bins, tables, ch, trx, torch)
        except RuntimeError as e:      # the sampler's likelihood budget: report, keep the line
            retrieval = {"error": str(e)}
            log(f"retrieval failed: {e}")

    out = {"metric": "forward spectra/s and gradient evals/s at \u22641e-6 rel err, batched vs "
                     "plain FP64",
           "value": round(B / (ms * 1e-3), 1), "unit": "spectra/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"bf16x2": "bf16", "bf16x3": "bf16", "fp32": "f32", "fp64": "f64"}[args.precision],
           "data": "synthetic",
           "config": {"workload": CONFIG_NAMES[3], "models": B, "layers": "50-200",
                      "wavenumbers": tables.n_wn, "window": "5000-40000", "absorbers": 5,
                      "channels": bins.n, "precision": args.precision,
                      "launch": "hip graph of one plan", "variant": variant},
           "roofline": roofline, "cpu_baseline": cpu, "fp64_gpu": fp64, "error": err,
           "ms_per_step_median": round(med, 3), "ms_per_step_iqr": [round(q1, 3), round(q3, 3)],
           "kernel_ms": {k: round(v, 4) for k, v in kms.items()}, "gradient": grad,
           "single_model": single, "clouds": clouds, "retrieval": retrieval}
    if large is not None:
        out["large"] = large
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
