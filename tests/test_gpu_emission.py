"""GPU parity of the emission forward model (trx_emission and emission
plans) against the FP64 oracle (oracle.emission), element by element on the
native grid and per channel, in every precision."""

import numpy as np
import pytest
import torch

import oracle
from synth.workloads import make_config, with_cloud_decks

pytestmark = pytest.mark.gpu

# Relative error of F_p/F_s against the oracle.  FP64 follows the oracle's
# arithmetic to rounding.  In the fast modes e^{-tau/mu} carries tau's
# relative error eps times tau/mu, so a point's error is bounded by
# 2 eps (1 + tau/mu at which its flux forms) + 1e-6 (the other FP32
# roundings), with the formation depth the flux-weighted tau/mu of the
# oracle's own layer terms: large at short wavelengths, where hot deep
# layers shine through cooler ones (10-20 for the workloads' hot Jupiters,
# up to ~100 for a cool planet around a hot star).  eps = 2^-23 for FP32 and
# split-bf16x3 (FP32 tables, mixing and sums), 2^-16 for split-bf16x2 (16
# bits of the path x weight products).  A binned channel is a weighted mean
# of its points, dominated by the brightest of them where the flux falls
# steeply across the channel (short wavelengths): its bound is the largest
# bound of its points, and no less than 1e-6.
EPS_TAU = {"fp32": 2.0 ** -23, "bf16x2": 2.0 ** -16, "bf16x3": 2.0 ** -23}
TOL_BINNED = {"fp64": 1e-12, "fp32": 1e-6, "bf16x2": 1e-6, "bf16x3": 1e-6}


def _formation_depth(ref, n_mu):
    """Flux-weighted tau/mu per native point of an oracle emission model
    (keep=True): sum over angles and layers of each term's share of the
    flux times the tau/mu at the middle of its layer."""
    tau, B = ref["tau"], ref["B_layer"]
    tau_up = np.vstack([tau[1:], np.zeros((1, tau.shape[1]))])
    mus, ws = oracle.gauss_legendre_mu(n_mu)
    num = np.zeros(tau.shape[1])
    den = np.zeros(tau.shape[1])
    for mu, w in zip(mus, ws):
        E, Eu = np.exp(-tau / mu), np.exp(-tau_up / mu)
        c = 2.0 * w * mu * np.vstack([B[0:1] * E[0:1], B * (Eu - E)])
        d = np.vstack([tau[0:1], 0.5 * (tau + tau_up)]) / mu
        d = np.where(np.isfinite(d), d, 0.0)
        num += np.sum(c * d, axis=0)
        den += np.sum(c, axis=0)
    return num / den


def _tol_native(mode, ref, n_mu):
    if mode == "fp64":
        return 1e-12
    return 2.0 * EPS_TAU[mode] * (1.0 + _formation_depth(ref, n_mu)) + 1e-6


def _rel(g, r):
    g = np.asarray(g)
    assert np.all(np.isfinite(g)), "non-finite emission output"
    return float(np.max(np.abs(g - r) / np.abs(r)))


def _check(ctx, tables, batch, ch, mode, n_mu, T_star, max_layers=None, t_interp="linear"):
    from paper_1912_07759_amd import trx
    Tt = trx.Tables.from_synth(ctx, tables, t_interp)
    bins = trx.Bins(ctx, Tt, ch.lo, ch.hi)
    try:
        db = trx.DeviceBatch.from_synth(batch, max_layers=max_layers)
        nat, binned, st = trx.emission(ctx, Tt, db, bins, mode, n_mu=n_mu, T_star=T_star)
        torch.cuda.synchronize()
        nat, binned, st = nat.cpu().numpy(), binned.cpu().numpy(), st.cpu().numpy()
    finally:
        bins.close()
        Tt.close()
    assert np.all(st == 0), st
    Ts = np.broadcast_to(np.asarray(T_star, dtype=np.float64), (batch.B,))
    worst = 0.0
    for b in range(batch.B):
        ref = oracle.emission_model(dict(batch.model(b), t_interp=t_interp), tables, ch, n_mu=n_mu,
                                    T_star=float(Ts[b]), keep=True)
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        g = nat[b, lo:hi]
        assert np.all(np.isfinite(g)), "non-finite emission output"
        # the largest error as a fraction of each point's own bound
        e1 = float(np.max(np.abs(g - ref["fpfs"]) / np.abs(ref["fpfs"]) / _tol_native(mode, ref, n_mu)))
        ok = ~np.isnan(ref["binned"])
        assert np.array_equal(np.isnan(binned[b]), ~ok)
        e2 = _rel(binned[b][ok], ref["binned"][ok]) if ok.any() else 0.0
        # each channel within the largest bound of its points (at least 1e-6)
        if mode != "fp64" and ok.any():
            tn = _tol_native(mode, ref, n_mu)
            w = oracle.bin_weights(tables.wn, ch.lo, ch.hi, lo, hi)
            tb = np.array([max(TOL_BINNED[mode], np.max(tn[w[c] > 0], initial=0.0)) for c in range(len(ch.lo))])
            eb = np.abs(binned[b][ok] - ref["binned"][ok]) / np.abs(ref["binned"][ok]) / tb[ok]
            assert np.max(eb) <= 1.0, (b, float(np.max(eb)))
        elif ok.any():
            assert e2 <= TOL_BINNED[mode], e2
        assert np.all(np.isnan(nat[b, :lo])) and np.all(np.isnan(nat[b, hi:]))
        print(f"{mode} n_mu={n_mu} model {b} (N={int(batch.n_layers[b])}, window {hi - lo}): "
              f"native {_rel(g, ref['fpfs']):.2e} ({e1:.2f} of its bound) binned {e2:.2e}")
        worst = max(worst, e1)
    return worst


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x2", "bf16x3"])
def test_emission_single_model(gpu_ctx, mode):
    """The 5-absorber 100-layer Guillot model with CIA and Rayleigh on a
    3000-point grid (several spans and a ragged tail), 4 angles, a 5800 K
    star: native and binned against the oracle."""
    tables, batch, ch = make_config(2, n_wn=3000, n_lines=300)
    assert _check(gpu_ctx, tables, batch, ch, mode, 4, 5800.0) <= 1.0


@pytest.mark.parametrize("mode", ["fp64", "bf16x2", "fp32"])
@pytest.mark.parametrize("n_mu", [1, 8])
def test_emission_ragged_batch(gpu_ctx, mode, n_mu):
    """A ragged batch (50-200 layers, windows of the grid) with a star
    temperature per model; 1 and 8 angles."""
    tables, batch, ch = make_config(3, n_wn=2000, n_lines=200, B=10)
    T_star = np.random.default_rng(3).uniform(3500.0, 7500.0, batch.B)
    assert _check(gpu_ctx, tables, batch, ch, mode, n_mu, T_star, max_layers=200) <= 1.0


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x2"])
def test_emission_cloud_decks(gpu_ctx, mode):
    """No deck, finite decks and opaque decks (the deck's vertical optical
    depth joins every layer's; an opaque deck's top layer acts as the
    surface)."""
    tables, batch, ch = make_config(3, n_wn=1500, n_lines=150, B=9)
    batch = with_cloud_decks(batch, 4)
    assert _check(gpu_ctx, tables, batch, ch, mode, 4, 6000.0, max_layers=200) <= 1.0


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x2"])
def test_emission_isothermal_is_planck(gpu_ctx, mode):
    """An isothermal atmosphere emits B(T) whatever its opacity: F_p/F_s =
    B(T)/B(T_star) (Rp/Rs)^2 (Planck's law written out here)."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(3, n_wn=1500, n_lines=150, B=4)
    Tiso = np.array([700.0, 1300.0, 2100.0, 2900.0])
    batch.T = np.concatenate([np.full(int(n), t) for n, t in zip(batch.n_layers, Tiso)])
    Tt = trx.Tables.from_synth(gpu_ctx, tables)
    try:
        db = trx.DeviceBatch.from_synth(batch, max_layers=200)
        nat, _, st = trx.emission(gpu_ctx, Tt, db, None, mode, n_mu=3, T_star=5000.0)
        nat, st = nat.cpu().numpy(), st.cpu().numpy()
    finally:
        Tt.close()
    assert np.all(st == 0)
    c2 = 100.0 * 6.62607015e-34 * 299792458.0 / batch.k_B
    for b in range(batch.B):
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        wn = tables.wn[lo:hi]
        want = np.expm1(c2 * wn / 5000.0) / np.expm1(c2 * wn / Tiso[b]) * (batch.Rp[b] / batch.Rs[b]) ** 2
        e = _rel(nat[b, lo:hi], want)
        print(f"{mode} isothermal {Tiso[b]} K: {e:.2e}")
        assert e <= (1e-13 if mode == "fp64" else 1e-6)   # only the top layer's term: no tau


def test_emission_invalid_inputs(gpu_ctx):
    """A non-positive or NaN star flags its model (NaN outputs, neighbours
    unaffected); bad angle counts and FP64 batches past the layer limit are
    rejected before any work."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(3, n_wn=800, n_lines=60, B=4)
    Tt = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, Tt, ch.lo, ch.hi)
    try:
        db = trx.DeviceBatch.from_synth(batch, max_layers=200)
        nat, binned, st = trx.emission(gpu_ctx, Tt, db, bins, "bf16x2", n_mu=4,
                                       T_star=np.array([5800.0, 0.0, np.nan, 4000.0]))
        st, nat, binned = st.cpu().numpy(), nat.cpu().numpy(), binned.cpu().numpy()
        assert st[0] == 0 and st[3] == 0
        assert st[1] & trx.BAD_PROFILE and st[2] & trx.BAD_PROFILE
        assert np.all(np.isnan(binned[1])) and np.all(np.isnan(binned[2]))
        assert np.all(np.isfinite(binned[0][~np.isnan(binned[0])]))
        for n_mu in (0, 17):
            with pytest.raises(trx.TrxError) as e:
                trx.emission(gpu_ctx, Tt, db, bins, "fp32", n_mu=n_mu)
            assert e.value.code == 1
        db300 = trx.DeviceBatch.from_synth(batch, max_layers=300)
        with pytest.raises(trx.TrxError) as e:
            trx.emission(gpu_ctx, Tt, db300, bins, "fp64")
        assert e.value.code == 4
    finally:
        bins.close()
        Tt.close()


@pytest.mark.parametrize("mode", ["bf16x2", "fp64"])
def test_emission_plan_graph(gpu_ctx, mode):
    """An emission plan replayed from a HIP graph equals trx_emission bit for
    bit, over replays with eager work in between and for a smaller B; a plan
    launched before its star is set is rejected."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(3, n_wn=1500, n_lines=150, B=8)
    T_star = np.linspace(4500.0, 6500.0, batch.B)
    Tt = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, Tt, ch.lo, ch.hi)
    plan = trx.Plan(gpu_ctx, Tt, bins, B_max=batch.B, N_max=200, precision=mode, graph=True,
                    emission=True)
    try:
        db = trx.DeviceBatch.from_synth(batch, max_layers=200)
        with pytest.raises(trx.TrxError):
            plan.launch(db)
        plan.set_star(T_star, n_mu=4)
        ref_nat, ref_bin, _ = trx.emission(gpu_ctx, Tt, db, bins, mode, n_mu=4, T_star=T_star)
        ref_nat, ref_bin = ref_nat.cpu().numpy(), ref_bin.cpu().numpy()
        for r in range(3):
            x = torch.randn(1 << 16, device="cuda").sum()
            nat, binned, st = plan.launch(db, native=True)
            torch.cuda.synchronize()
            assert float(x) == float(x)
            assert np.all(st.cpu().numpy() == 0)
            assert np.array_equal(nat.cpu().numpy(), ref_nat, equal_nan=True)
            assert np.array_equal(binned.cpu().numpy(), ref_bin, equal_nan=True)
        # a batch of one (model 2) on the same graph, its star in slot 0
        plan.set_star([T_star[2]], n_mu=4)
        _, binned, _ = plan.launch(db.view(2))
        torch.cuda.synchronize()
        assert np.array_equal(binned.cpu().numpy()[0], ref_bin[2], equal_nan=True)
    finally:
        plan.close()
        bins.close()
        Tt.close()


@pytest.mark.parametrize("mode", ["fp32", "bf16x2", "fp64"])
def test_emission_faint_planet(gpu_ctx, mode):
    """A cool planet (Guillot profile of 500 K irradiation, 300-650 K) around
    a 7500 K star: at the short-wavelength end of the grid its flux is
    ~1e-50 of the star's (below the FP32 range), and every point must still
    match the oracle (the flux ratio is carried in FP64 range)."""
    from synth.atmosphere import guillot_T, log_midpoint_pressures
    from synth.constants import GM_JUP, R_JUP, R_SUN
    from synth.workloads import Channels, batch_from_models, make_tables
    from synth.atmosphere import log_uniform_channels
    tables = make_tables(2, n_wn=1200, n_lines=120)
    lo, hi = log_uniform_channels(tables.wn, 20)
    ch = Channels(lo, hi)
    Ts = [guillot_T(log_midpoint_pressures(1e6, 1e-4, N), GM_JUP / R_JUP ** 2, 500.0) for N in (80, 150)]
    vmr = np.array([[-4.0, -6.0, -5.0, -7.0, -8.0], [-3.5, -5.0, -6.0, -7.5, -8.5]])
    batch = batch_from_models(Ts, 1e6, 1e-4, vmr, R_JUP, R_SUN, GM_JUP, 0, tables.n_wn)
    ref = oracle.emission_model(batch.model(0), tables, ch, n_mu=4, T_star=7500.0)
    assert np.min(ref["fpfs"]) < 1e-45
    assert _check(gpu_ctx, tables, batch, ch, mode, 4, 7500.0, max_layers=150) <= 1.0
