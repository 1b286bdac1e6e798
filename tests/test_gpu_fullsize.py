"""GPU parity at the full sizes of the benchmark's workloads, in the launch
configuration bench.py times (graph-captured plans, autotuned variant):
sampled models against the oracle one by one, and properties that every
model of the batch must hold whatever its size."""

import numpy as np
import pytest
import torch

import oracle
from synth.workloads import make_config, observation_noise, with_cloud_decks
from parity_util import TOL, binned_rel_err, native_rel_err

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-4


def _picks(batch, k, seed):
    """The models of largest and smallest work (layers x window), then k
    random ones."""
    work = batch.n_layers.astype(np.float64) * (batch.wn_hi - batch.wn_lo)
    order = np.argsort(work)
    rnd = np.random.default_rng(seed).permutation(batch.B)[:k]
    return list(dict.fromkeys([int(order[-1]), int(order[0])] + [int(i) for i in rnd]))


def _bare_disc(batch):
    return (np.asarray(batch.Rp, dtype=np.float64) / np.asarray(batch.Rs, dtype=np.float64)) ** 2 \
        * np.ones(batch.B)


def _grad_err(g, off, b, ref):
    v = np.concatenate([g["dT"][off[b]:off[b + 1]], g["dlog10_vmr"][b], [g["dRp"][b]]])
    r = np.concatenate([ref["dT"], ref["dlog10_vmr"], [ref["dRp"]]])
    big = np.abs(r) >= 1e-3 * np.max(np.abs(r))
    return max(np.linalg.norm(v - r) / np.linalg.norm(r),
               float(np.max(np.abs(v[big] - r[big]) / np.abs(r[big]))))


def _forward_full(ctx, cfg, precision, n_layers, n_check, seed, decks=False):
    """Forward of workload `cfg` at full size through an autotuned graph plan:
    the binned output as timed, then the native grid from the same plan
    (with decks: the benchmark's cloud decks on two thirds of the models)."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(cfg)
    if decks:
        batch = with_cloud_decks(batch, 5)
    T = trx.Tables.from_synth(ctx, tables)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=n_layers)
    plan = trx.Plan(ctx, T, bins, B_max=batch.B, N_max=n_layers, precision=precision, graph=True)
    variant = plan.autotune(db)
    _, binned, st = plan.launch(db)
    binned, st = binned.cpu().numpy().copy(), st.cpu().numpy().copy()
    nat, binned2, _ = plan.launch(db, native=True)
    nat, binned2 = nat.cpu().numpy(), binned2.cpu().numpy()
    plan.close()
    bins.close()
    T.close()
    print(f"workload {cfg}: B={batch.B}, W={tables.n_wn}, variant {variant}")

    # every model: valid, the binned output identical with and without the
    # native grid, finite depths no smaller than the bare disc inside the
    # window (each 1 - e^{-tau} >= 0) and nothing written outside it; the
    # binned channels outside the window are NaN (their pattern is checked
    # against the oracle on the sampled models), every model has some inside
    assert np.all(st == 0), np.flatnonzero(st)
    assert np.array_equal(binned, binned2, equal_nan=True)
    disc = _bare_disc(batch)
    ok = ~np.isnan(binned)
    assert np.all(ok.any(axis=1))
    assert np.all(np.isfinite(binned[ok]))
    assert np.all(binned[ok] >= np.broadcast_to(disc[:, None], binned.shape)[ok] * (1.0 - 1e-12))
    for b in range(batch.B):
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        inside = nat[b, lo:hi]
        assert np.all(np.isfinite(inside)) and np.all(inside >= disc[b] * (1.0 - 1e-12)), b
        assert np.all(np.isnan(nat[b, :lo])) and np.all(np.isnan(nat[b, hi:])), b

    # sampled models against the oracle, element by element
    worst = 0.0
    for b in dict.fromkeys(_picks(batch, n_check, seed) + ([0, 1, 2] if decks else [])):
        ref = oracle.forward_model(batch.model(b), tables, ch)
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        e1 = native_rel_err(nat[b], ref["depth"], lo, hi)
        e2 = binned_rel_err(binned[b], ref["binned"])
        print(f"  model {b} (N={int(batch.n_layers[b])}, window {hi - lo}): native {e1:.2e} binned {e2:.2e}")
        worst = max(worst, e1, e2)
    assert worst <= TOL[precision]
    return tables, batch, ch


def test_batched_4096_full_size(gpu_ctx):
    """The benchmark's batch: 4096 models of 50-200 layers, windows of
    5000-40000 of 40000 points, 5 absorbers with CIA and Rayleigh, 50
    channels, split-bf16."""
    _forward_full(gpu_ctx, 3, "bf16x2", 200, 4, 0)


def test_batched_4096_with_cloud_decks_full_size(gpu_ctx):
    """The benchmark's batch with its cloud decks (a third none, a third
    finite, a third opaque); sampled models of each kind among the checked."""
    _forward_full(gpu_ctx, 3, "bf16x2", 200, 4, 6, decks=True)


def _gradient_full(ctx, cfg, tables, batch, ch, n_layers, n_check, seed, precision="fp64"):
    """chi^2 gradients of workload `cfg` at full size through an autotuned
    graph-captured gradient plan (forward pass in `precision`), against the
    oracle's reference gradient on point 0 (its residual is the noise) and
    sampled points; every point valid with finite outputs.  Returns the
    gradient outputs and the observation."""
    from paper_1912_07759_amd import trx
    T = trx.Tables.from_synth(ctx, tables)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=n_layers)
    truth = oracle.forward_model(batch.model(0), tables, ch)["binned"]
    noise, sigma = observation_noise(cfg, 1, len(ch.lo))
    obs = np.tile(truth + noise[0], (batch.B, 1))
    plan = trx.Plan(ctx, T, bins, B_max=batch.B, N_max=n_layers, precision=precision, graph=True,
                    grad=True)
    plan.autotune(db)
    out = plan.launch_grad(db, obs, sigma)
    g = {k: v.cpu().numpy().copy() for k, v in out.items()}
    plan.close()
    bins.close()
    T.close()
    assert np.all(g["status"] == 0), np.flatnonzero(g["status"])
    for k in ("chi2", "dT", "dlog10_vmr", "dRp"):
        assert np.all(np.isfinite(g[k])), k
    assert np.all(g["chi2"] >= 0.0)
    off = batch.layer_off
    picks = list(dict.fromkeys([0] + [int(i) for i in
                                      np.random.default_rng(seed).permutation(batch.B)[:n_check]]))
    worst = 0.0
    for b in picks:
        ref = oracle.chi2_and_grad(batch.model(b), tables, ch, obs[b], sigma)
        err = _grad_err(g, off, b, ref)
        print(f"  {precision} point {b} (N={int(batch.n_layers[b])}): chi2 {g['chi2'][b]:.6e} "
              f"(oracle {ref['chi2']:.6e}), grad err {err:.2e}")
        assert abs(g["chi2"][b] - ref["chi2"]) <= 1e-5 * ref["chi2"]
        worst = max(worst, err)
    print(f"  {precision}: worst gradient error {worst:.2e} over {len(picks)} points")
    assert worst <= GRAD_TOL, worst
    return g, obs, sigma


@pytest.mark.parametrize("precision", ["fp32", "bf16x2", "fp64"])
def test_gradient_256_full_size(gpu_ctx, precision):
    """The benchmark's gradient workload: 256 points of a 100-layer free
    temperature profile, 7 absorbers, 50000 points, 100 channels, 50 ppm
    noise on the truth's binned spectrum; the forward pass in FP32 (the
    workload's own precision), split-bf16 and FP64; point 0 and 8 random
    points against the oracle's reference gradient."""
    tables, batch, ch = make_config(4)
    _gradient_full(gpu_ctx, 4, tables, batch, ch, 100, 8, 1, precision)


def test_gradient_256_central_differences(gpu_ctx):
    """Central differences of chi^2, every component of 8 points of the
    gradient workload (108 parameters each: 100 temperatures, 7 log10 mixing
    ratios, Rp), from the library's FP64 forward model, against the
    gradients with the FP32 and split-bf16 forwards.  Steps: 1e-4 K (the
    temperatures stay 1e-3 K from the table nodes), 1e-6 dex, 1e-7 Rp; all
    perturbed models run as one batch."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(4)
    truth = oracle.forward_model(batch.model(0), tables, ch)["binned"]
    noise, sigma = observation_noise(4, 1, len(ch.lo))
    obs = truth + noise[0]
    pts = [0] + [int(i) for i in np.random.default_rng(17).permutation(np.arange(1, batch.B))[:7]]
    sub = batch.subset(pts)
    N, na = 100, tables.n_abs
    # perturbed copies: point p, parameter k, sign s
    Ts, vmr, Rp, steps = [], [], [], []
    for p in range(len(pts)):
        for k in range(N + na + 1):
            for sgn in (1.0, -1.0):
                T = sub.T_of(p).copy()
                v = sub.log10_vmr[p].copy()
                R = float(sub.Rp[p])
                if k < N:
                    h = 1e-4
                    T[k] += sgn * h
                elif k < N + na:
                    h = 1e-6
                    v[k - N] += sgn * h
                else:
                    h = 1e-7 * R
                    R += sgn * h
                Ts.append(T)
                vmr.append(v)
                Rp.append(R)
                steps.append(h)
    from synth.workloads import batch_from_models
    fd_batch = batch_from_models(Ts, 1e6, 1e-4, np.array(vmr), np.array(Rp), sub.Rs[0], sub.GM[0], 0,
                                 tables.n_wn)
    Tt = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, Tt, ch.lo, ch.hi)
    try:
        db = trx.DeviceBatch.from_synth(fd_batch, max_layers=N)
        _, binned, st = trx.forward(gpu_ctx, Tt, db, bins, "fp64", native=False)
        binned, st = binned.cpu().numpy(), st.cpu().numpy()
        assert np.all(st == 0)
        c2 = np.sum(((binned - obs[None, :]) / sigma[None, :]) ** 2, axis=1)
        fd = ((c2[0::2] - c2[1::2]) / (2.0 * np.array(steps[0::2]))).reshape(len(pts), N + na + 1)
        dsub = trx.DeviceBatch.from_synth(sub, max_layers=N)
        for mode in ("fp32", "bf16x2"):
            g = trx.chi2_grad(gpu_ctx, Tt, dsub, bins, np.tile(obs, (len(pts), 1)), sigma, mode)
            g = {k: v.cpu().numpy() for k, v in g.items() if v is not None}
            assert np.all(g["status"] == 0)
            worst = 0.0
            for p in range(len(pts)):
                v = np.concatenate([g["dT"][p * N:(p + 1) * N], g["dlog10_vmr"][p], [g["dRp"][p]]])
                r = fd[p]
                big = np.abs(r) >= 1e-3 * np.max(np.abs(r))
                err = max(np.linalg.norm(v - r) / np.linalg.norm(r),
                          float(np.max(np.abs(v[big] - r[big]) / np.abs(r[big]))))
                print(f"  {mode} point {pts[p]}: gradient vs central differences {err:.2e}")
                worst = max(worst, err)
            assert worst <= GRAD_TOL, (mode, worst)
    finally:
        bins.close()
        Tt.close()


def test_large_workload_full_size(gpu_ctx):
    """The large workload: 1024 models of 100-200 layers, 10 absorbers on 40
    x 30 x 100000-point tables, 100 channels; split-bf16 forward of every
    model (sampled ones against the oracle), then gradients with the FP64
    forward on sampled points."""
    tables, batch, ch = _forward_full(gpu_ctx, 5, "bf16x2", 200, 1, 2)
    _gradient_full(gpu_ctx, 5, tables, batch, ch, 200, 1, 3)


def test_emission_4096_full_size(gpu_ctx):
    """The benchmark's batch in emission (a blackbody star of 4500-6500 K per
    model, 4 angles) through an autotuned graph-captured emission plan in
    FP32, in the benchmark's launch configuration (persistent kernel, items
    of several spans, back to back): every model valid with finite outputs
    on its window, sampled models within each point's bound of the oracle."""
    from paper_1912_07759_amd import trx
    from synth.workloads import stellar_temperatures
    from test_gpu_emission import _tol_native
    tables, batch, ch = make_config(3)
    T_star = stellar_temperatures(batch.B)
    T = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, T, ch.lo, ch.hi)
    plan = trx.Plan(gpu_ctx, T, bins, B_max=batch.B, N_max=200, precision="fp32", graph=True,
                    emission=True)
    try:
        plan.set_star(T_star, n_mu=4)
        db = trx.DeviceBatch.from_synth(batch, max_layers=200)
        print("variant", plan.autotune(db))
        for _ in range(3):
            nat, binned, st = plan.launch(db, native=True)
        st = st.cpu().numpy()
        assert np.all(st == 0), np.flatnonzero(st)
        picks = _picks(batch, 3, 4)
        rows = nat[picks].cpu().numpy()
        for i, b in enumerate(picks):
            lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
            ref = oracle.emission_model(batch.model(b), tables, ch, n_mu=4, T_star=float(T_star[b]),
                                        keep=True)
            g = rows[i, lo:hi]
            assert np.all(np.isfinite(g))
            frac = np.max(np.abs(g - ref["fpfs"]) / ref["fpfs"] / _tol_native("fp32", ref, 4))
            print(f"  model {b}: worst point at {frac:.2f} of its bound")
            assert frac <= 1.0
        for b in range(batch.B):
            lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
            assert bool(torch.all(torch.isfinite(nat[b, lo:hi]))), b
    finally:
        plan.close()
        bins.close()
        T.close()
