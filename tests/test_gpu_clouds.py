"""GPU parity of the flat-opacity cloud deck (equation clouds) against the
FP64 oracle: the forward model in every mode (FP64 in its slot form up to
224 layers and its layer form beyond), the optical-depth output, the chi^2
gradient, graph-captured plans, and invalid deck parameters.  Each batch
mixes models without a deck, with finite decks (one over the whole
atmosphere, one between two layer pressures that holds no layer) and with
opaque decks (one reaching the top layer, whose ray has no path)."""

import numpy as np
import pytest

import oracle
from parity_util import TOL, binned_rel_err, native_rel_err
from synth.atmosphere import guillot_T, log_midpoint_pressures, log_uniform_channels
from synth.constants import GM_JUP, R_JUP, R_SUN
from synth.workloads import (Channels, batch_from_models, make_config, make_tables,
                             observation_noise, with_cloud_decks)

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32", "bf16x2", "bf16x3"]
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def tables():
    return make_tables(2, n_wn=700, n_lines=120)


def _channels(t):
    lo, hi = log_uniform_channels(t.wn, 9)
    return Channels(lo, hi)


def _profile(N, T_irr=1200.0):
    return guillot_T(log_midpoint_pressures(1e6, 1e-4, N), GM_JUP / R_JUP ** 2, T_irr)


def _decked_batch(t, Ns):
    """Models of the given layer counts with decks: none, flat mid-level,
    opaque from 1e3 Pa down, flat over everything, opaque reaching the top,
    flat but empty (both bounds between layers 10 and 11), then repeating."""
    n = len(Ns)
    Ts = [_profile(N, 1000.0 + 40.0 * i) for i, N in enumerate(Ns)]
    vmr = np.tile(np.array([-4.0, -5.0, -6.0, -3.5, -7.0]), (n, 1))
    W = t.n_wn
    lo = [(37 * i) % 200 for i in range(n)]
    hi = [W - (53 * i) % 150 for i in range(n)]
    batch = batch_from_models(Ts, 1e6, 1e-4, vmr, R_JUP, R_SUN, GM_JUP, lo, hi)
    sig, pt, pb = np.zeros(n), np.ones(n), np.ones(n)
    for b, N in enumerate(Ns):
        edges = np.logspace(6.0, -4.0, N + 1)
        P = edges[:-1] * np.sqrt(edges[1:] / edges[:-1])
        kind = b % 6
        if kind == 1:
            sig[b], pt[b], pb[b] = 3e-29, 1e2, 1e4
        elif kind == 2:
            sig[b], pt[b], pb[b] = np.inf, 1e3, 1e6
        elif kind == 3:
            sig[b], pt[b], pb[b] = 1e-30, 1e-5, 1e7
        elif kind == 4:
            sig[b], pt[b], pb[b] = np.inf, 1e-5, 1e-2
        elif kind == 5:
            sig[b], pt[b], pb[b] = 1e-27, P[11] * 1.01, P[10] * 0.99
    batch.cloud_sigma, batch.cloud_p_top, batch.cloud_p_bottom = sig, pt, pb
    return batch


def _forward(ctx, t, batch, ch, mode, max_layers, out_tau=None):
    from paper_1912_07759_amd import trx
    T = trx.Tables.from_synth(ctx, t)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=max_layers)
    nat, binned, st = trx.forward(ctx, T, db, bins, mode, out_tau=out_tau)
    ctx.synchronize()
    out = nat.cpu().numpy(), binned.cpu().numpy(), st.cpu().numpy()
    bins.close()
    T.close()
    return out


def _worst(t, batch, ch, nat, binned, st):
    assert np.all(st == 0), st
    worst = 0.0
    for b in range(batch.B):
        ref = oracle.forward_model(batch.model(b), t, ch)
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        worst = max(worst, native_rel_err(nat[b], ref["depth"], lo, hi),
                    binned_rel_err(binned[b], ref["binned"]))
    return worst


@pytest.mark.parametrize("mode", MODES)
def test_cloud_decks_forward(gpu_ctx, tables, mode):
    ch = _channels(tables)
    batch = _decked_batch(tables, [60, 100, 150, 224, 33, 120, 2, 80])
    nat, binned, st = _forward(gpu_ctx, tables, batch, ch, mode, 224)
    worst = _worst(tables, batch, ch, nat, binned, st)
    # the decks raise the spectra (to rounding, where the gas is already
    # opaque) and change them (the empty deck excepted)
    clear = batch.subset(np.arange(batch.B))
    clear.cloud_sigma = None
    clear.cloud_p_top = clear.cloud_p_bottom = None
    nat0, _, _ = _forward(gpu_ctx, tables, clear, ch, mode, 224)
    for b in (1, 2, 3, 4):
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        assert np.all(nat[b, lo:hi] >= nat0[b, lo:hi] * (1.0 - TOL[mode])), b
        assert np.max(nat[b, lo:hi] / nat0[b, lo:hi]) > 1.0 + 100.0 * TOL[mode], b
    b = 5
    assert np.array_equal(nat[b], nat0[b], equal_nan=True)
    print(f"{mode}: cloud decks worst rel err {worst:.2e}")
    assert worst <= TOL[mode]


def test_cloud_decks_fp64_layer_form(gpu_ctx, tables):
    """FP64 models of more than 224 layers run the layer form."""
    ch = _channels(tables)
    batch = _decked_batch(tables, [300, 260, 250, 240, 230, 300])
    nat, binned, st = _forward(gpu_ctx, tables, batch, ch, "fp64", 300)
    worst = _worst(tables, batch, ch, nat, binned, st)
    print(f"fp64 layer form: cloud decks worst rel err {worst:.2e}")
    assert worst <= TOL["fp64"]


@pytest.mark.parametrize("mode", ["fp64", "bf16x2"])
def test_cloud_decks_optical_depth(gpu_ctx, tables, mode):
    """The optical-depth output includes the deck's depth: +inf on the rays
    an opaque deck blocks, the oracle's tau elsewhere."""
    import torch
    ch = _channels(tables)
    batch = _decked_batch(tables, [60, 100, 150, 120, 90, 70])
    tau = torch.full((batch.B, 150, tables.n_wn), float("nan"), dtype=torch.float64, device="cuda")
    _, _, st = _forward(gpu_ctx, tables, batch, ch, mode, 150, out_tau=tau)
    assert np.all(st == 0)
    tau = tau.cpu().numpy()
    tol = {"fp64": 1e-12, "bf16x2": 1e-4}[mode]
    worst = 0.0
    for b in range(batch.B):
        N = int(batch.n_layers[b])
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        ref = oracle.forward_model(batch.model(b), tables, ch, keep=True)["tau"]
        g = tau[b, :N, lo:hi]
        inf = np.isinf(ref)
        assert np.array_equal(np.isinf(g), inf), b
        fin = ~inf
        assert np.all(np.isfinite(g[fin]))
        err = np.abs(g[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1e-300)
        worst = max(worst, float(np.max(err)) if err.size else 0.0)
        assert np.all(np.isnan(tau[b, N:])) and np.all(np.isnan(tau[b, :N, :lo]))
    print(f"{mode}: optical depth with decks worst rel err {worst:.2e}")
    assert worst <= tol


@pytest.fixture(scope="module")
def grad_problem():
    """The reduced gradient workload (100 layers, 7 absorbers, CIA and
    Rayleigh, 100 channels) with decks of every kind: finite, opaque, none."""
    tables, batch, ch = make_config(4, n_wn=2500, n_lines=250, B=6)
    batch = with_cloud_decks(batch, 11, kinds=("flat", "opaque", "none"))
    truth = oracle.forward_model(batch.model(0), tables, ch)["binned"]
    noise, sigma = observation_noise(4, 1, len(ch.lo))
    obs = np.tile(truth + noise[0], (batch.B, 1))
    return tables, batch, ch, obs, sigma


def _grad_err(g, off, b, ref):
    v = np.concatenate([g["dT"][off[b]:off[b + 1]], g["dlog10_vmr"][b], [g["dRp"][b]]])
    assert np.all(np.isfinite(v)), "non-finite gradient"
    r = np.concatenate([ref["dT"], ref["dlog10_vmr"], [ref["dRp"]]])
    big = np.abs(r) >= 1e-3 * np.max(np.abs(r))
    return max(np.linalg.norm(v - r) / np.linalg.norm(r),
               float(np.max(np.abs(v[big] - r[big]) / np.abs(r[big]))))


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
def test_cloud_decks_gradient(gpu_ctx, grad_problem, mode):
    from paper_1912_07759_amd import trx
    tables, batch, ch, obs, sigma = grad_problem
    Tt = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, Tt, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=100)
    out = trx.chi2_grad(gpu_ctx, Tt, db, bins, obs, sigma, mode)
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    bins.close()
    Tt.close()
    assert np.all(g["status"] == 0)
    worst = 0.0
    for b in range(batch.B):
        ref = oracle.chi2_and_grad(batch.model(b), tables, ch, obs[b], sigma)
        assert abs(g["chi2"][b] - ref["chi2"]) <= 1e-5 * ref["chi2"]
        err = _grad_err(g, batch.layer_off, b, ref)
        print(f"{mode} point {b} (deck sigma {batch.cloud_sigma[b]:.1e}): grad err {err:.2e}")
        worst = max(worst, err)
    assert worst <= GRAD_TOL


def test_cloud_decks_plan_graph(gpu_ctx, tables):
    """A graph-captured forward plan with decks reproduces trx_forward over
    replays.  (A plan's own input buffers start without decks: the
    owned-buffer plan test runs them against cloud-free references.)"""
    from paper_1912_07759_amd import trx
    ch = _channels(tables)
    batch = _decked_batch(tables, [60, 100, 150, 120, 90, 70])
    T = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=150)
    nat0, bin0, _ = trx.forward(gpu_ctx, T, db, bins, "bf16x2")
    plan = trx.Plan(gpu_ctx, T, bins, B_max=batch.B, N_max=150, precision="bf16x2", graph=True)
    for _ in range(3):
        nat, binned, st = plan.launch(db, native=True)
        gpu_ctx.synchronize()
        assert np.all(st.cpu().numpy() == 0)
        assert np.array_equal(binned.cpu().numpy(), bin0.cpu().numpy(), equal_nan=True)
        assert np.array_equal(nat.cpu().numpy(), nat0.cpu().numpy(), equal_nan=True)
    plan.close()
    bins.close()
    T.close()


def test_invalid_cloud_decks_are_flagged(gpu_ctx, tables):
    """A negative or NaN cross-section, or a deck pressure that is not
    finite and positive under a nonzero cross-section, flags the model
    TRX_MODEL_BAD_PROFILE; deck pressures under a zero cross-section are
    ignored; the other models of the batch are unaffected."""
    ch = _channels(tables)
    batch = _decked_batch(tables, [60, 60, 60, 60, 60, 60])
    batch.cloud_sigma = np.array([-1e-30, np.nan, 1e-29, 1e-29, 0.0, np.inf])
    batch.cloud_p_top = np.array([1e2, 1e2, 0.0, 1e2, np.nan, np.inf])
    batch.cloud_p_bottom = np.array([1e4, 1e4, 1e4, -5.0, np.nan, 1e4])
    nat, binned, st = _forward(gpu_ctx, tables, batch, ch, "bf16x2", 60)
    assert list(st) == [2, 2, 2, 2, 0, 2]
    ref = oracle.forward_model(batch.model(4), tables, ch)
    lo, hi = int(batch.wn_lo[4]), int(batch.wn_hi[4])
    assert native_rel_err(nat[4], ref["depth"], lo, hi) <= TOL["bf16x2"]
