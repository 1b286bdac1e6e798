"""GPU edge cases of the forward model against the FP64 oracle: the fewest
and the most layers each mode accepts, windows of one point and of the whole
grid, temperatures and pressures outside the tables (each clamp rule),
constant gravity and a model without any opacity.  The batches mix these
cases in one launch (persistent in the matrix-core modes).  A batch of no
models is an invalid argument at every entry point."""

import dataclasses

import numpy as np
import pytest

from synth.atmosphere import guillot_T, log_midpoint_pressures, log_uniform_channels
from synth.constants import GM_JUP, R_JUP, R_SUN
from synth.workloads import Channels, batch_from_models, make_tables
import oracle
from parity_util import TOL, binned_rel_err, native_rel_err, oracle_batch

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32", "bf16x2", "bf16x3"]


@pytest.fixture(scope="module")
def tables():
    return make_tables(2, n_wn=700, n_lines=120)


def _channels(t):
    lo, hi = log_uniform_channels(t.wn, 9)
    return Channels(lo, hi)


def _profile(N, T_irr=1200.0, shift=0.0):
    return guillot_T(log_midpoint_pressures(1e6, 1e-4, N), GM_JUP / R_JUP ** 2, T_irr) + shift


def _run(ctx, t, batch, ch, mode, max_layers):
    from paper_1912_07759_amd import trx
    T = trx.Tables.from_synth(ctx, t)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=max_layers)
    nat, binned, st = trx.forward(ctx, T, db, bins, mode)
    ctx.synchronize()
    out = nat.cpu().numpy(), binned.cpu().numpy(), st.cpu().numpy()
    bins.close()
    T.close()
    return out


def _check(t, batch, ch, mode, nat, binned, st):
    assert np.all(st == 0), st
    idx, ref = oracle_batch(t, batch, ch, mode)
    worst = 0.0
    for b, r in zip(idx, ref):
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        worst = max(worst, native_rel_err(nat[b], r["depth"], lo, hi),
                    binned_rel_err(binned[b], r["binned"]))
    return worst


@pytest.mark.parametrize("mode", MODES)
def test_layer_extremes_and_windows(gpu_ctx, tables, mode):
    """N = 2, 3, 33 and the mode's maximum (224 for the matrix-core modes,
    300 for FP64: two passes of its ray blocks); windows of one point at
    either end of the grid, the whole grid, and a span-ragged middle."""
    t = tables
    W = t.n_wn
    Nmax = 300 if mode == "fp64" else 224
    Ns = [2, 3, 33, Nmax, Nmax, 64]
    win = [(0, 1), (W - 1, W), (0, W), (5, W - 3), (63, 65), (130, 131)]
    Ts = [_profile(N) for N in Ns]
    vmr = np.tile(np.array([-4.0, -5.0, -6.0, -3.5, -7.0]), (len(Ns), 1))
    batch = batch_from_models(Ts, 1e6, 1e-4, vmr, R_JUP, R_SUN, GM_JUP,
                              [w[0] for w in win], [w[1] for w in win])
    ch = _channels(t)
    nat, binned, st = _run(gpu_ctx, t, batch, ch, mode, Nmax)
    worst = _check(t, batch, ch, mode, nat, binned, st)
    print(f"{mode}: layer/window extremes worst rel err {worst:.2e}")
    assert worst <= TOL[mode]


@pytest.mark.parametrize("mode", MODES)
def test_out_of_table_clamps(gpu_ctx, tables, mode):
    """Temperatures below and above the table grid, and pressures below it
    (the top layers at 1e-6 Pa): each clamp case, including T and P both
    below the grid (zero cross-section)."""
    t = tables
    N = 60
    T_hot = np.full(N, 5000.0)                     # above the T grid
    T_cold = np.full(N, 120.0)                     # below the T grid
    T_mix = np.where(np.arange(N) % 2 == 0, 150.0, 4200.0)
    T_grad = np.linspace(4000.0, 100.0, N)         # crosses the grid
    Ts = [T_hot, T_cold, T_mix, T_grad]
    vmr = np.tile(np.array([-3.0, -4.0, -5.0, -6.0, -3.0]), (len(Ts), 1))
    # 1e7 .. 1e-6 Pa extends past both ends of the log10 P grid (-4 .. 6)
    batch = batch_from_models(Ts, 1e7, 1e-6, vmr, R_JUP, R_SUN, GM_JUP, 0, t.n_wn)
    ch = _channels(t)
    nat, binned, st = _run(gpu_ctx, t, batch, ch, mode, N)
    worst = _check(t, batch, ch, mode, nat, binned, st)
    print(f"{mode}: clamp cases worst rel err {worst:.2e}")
    assert worst <= TOL[mode]


@pytest.mark.parametrize("mode", ["fp64", "bf16x2"])
def test_constant_gravity(gpu_ctx, tables, mode):
    t = tables
    Ts = [_profile(80), _profile(120, 1800.0)]
    vmr = np.tile(np.array([-4.0, -5.0, -6.0, -3.5, -7.0]), (2, 1))
    batch = batch_from_models(Ts, 1e6, 1e-4, vmr, R_JUP, R_SUN, GM_JUP, 0, t.n_wn, gravity=1)
    ch = _channels(t)
    nat, binned, st = _run(gpu_ctx, t, batch, ch, mode, 120)
    worst = _check(t, batch, ch, mode, nat, binned, st)
    print(f"{mode}: constant gravity worst rel err {worst:.2e}")
    assert worst <= TOL[mode]


@pytest.mark.parametrize("mode", MODES)
def test_no_opacity_gives_bare_disc(gpu_ctx, tables, mode):
    """Zero cross-sections, no CIA, no Rayleigh: the depth is (Rp/Rs)^2 at
    every point (transit-depth equations with a = 0)."""
    t = dataclasses.replace(tables, xsec=np.zeros_like(tables.xsec),
                            cia=np.zeros((0,) + tables.cia.shape[1:]),
                            cia_pair=np.zeros((0, 2), np.int32), rayleigh=None)
    Ts = [_profile(50), _profile(200)]
    Rp = np.array([0.7, 1.9]) * R_JUP
    vmr = np.full((2, t.n_abs), -3.0)
    batch = batch_from_models(Ts, 1e6, 1e-4, vmr, Rp, R_SUN, GM_JUP, [0, 100], [t.n_wn, 400])
    ch = _channels(t)
    nat, binned, st = _run(gpu_ctx, t, batch, ch, mode, 200)
    assert np.all(st == 0)
    for b in range(2):
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        want = (Rp[b] / R_SUN) ** 2
        assert np.all(nat[b, lo:hi] == want), (mode, b)


@pytest.mark.parametrize("mode", MODES)
def test_many_opacity_slots(gpu_ctx, tables, mode):
    """A three-level zig-zag temperature profile touches ~180 distinct table
    corners and CIA nodes, more than one staging chunk in every mode (128
    slots in the matrix-core modes, 96 in FP64), next to an ordinary model
    with a ragged window."""
    t = tables
    N = 200
    i = np.arange(N)
    zig = np.where(i % 2 == 0, 250.0, 3300.0) + np.linspace(0.0, 900.0, N)
    zig = np.where(i % 4 == 1, 1700.0 + np.linspace(0.0, 900.0, N), zig)
    Ts = [zig, _profile(120)]
    vmr = np.tile(np.array([-4.0, -5.0, -6.0, -3.5, -7.0]), (2, 1))
    batch = batch_from_models(Ts, 1e6, 1e-4, vmr, R_JUP, R_SUN, GM_JUP, [0, 37], [t.n_wn, 650])
    ch = _channels(t)
    nat, binned, st = _run(gpu_ctx, t, batch, ch, mode, N)
    worst = _check(t, batch, ch, mode, nat, binned, st)
    print(f"{mode}: many opacity slots worst rel err {worst:.2e}")
    assert worst <= TOL[mode]


def test_optical_depth_output_long_fp64(gpu_ctx, tables):
    """The optical-depth output of the FP64 layer kernel (models beyond
    TRX_MAX_LAYERS_MFMA layers): 300 layers against the oracle's tau."""
    import torch
    from paper_1912_07759_amd import trx
    t = tables
    batch = batch_from_models([_profile(300)], 1e6, 1e-4, np.array([[-4.0, -5.0, -6.0, -3.5, -7.0]]),
                              R_JUP, R_SUN, GM_JUP, [40], [t.n_wn - 7])
    T = trx.Tables.from_synth(gpu_ctx, t)
    db = trx.DeviceBatch.from_synth(batch, max_layers=300)
    tau = torch.full((1, 300, t.n_wn), float("nan"), dtype=torch.float64, device="cuda")
    _, _, st = trx.forward(gpu_ctx, T, db, None, "fp64", out_tau=tau)
    gpu_ctx.synchronize()
    T.close()
    assert int(st[0]) == 0
    g = tau[0].cpu().numpy()
    ref = oracle.forward_model(batch.model(0), t, None, keep=True)["tau"]
    got = g[:, 40:t.n_wn - 7]
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
    assert np.all(np.isfinite(got)) and not np.any(np.isnan(err))
    assert np.all(np.isnan(g[:, :40])) and np.all(np.isnan(g[:, t.n_wn - 7:]))
    print(f"fp64 300 layers: optical depth worst rel err {err.max():.2e}")
    assert err.max() <= 1e-12


def _no_absorber_tables(t):
    """The same grid with no absorbers: CIA and the H2 and He Rayleigh rows only."""
    return dataclasses.replace(t, xsec=np.zeros((0,) + t.xsec.shape[1:]), abs_mass=np.zeros(0),
                               cia_pair=t.cia_pair - t.n_abs, rayleigh=t.rayleigh[t.n_abs:], names=[])


@pytest.mark.parametrize("mode", MODES)
def test_no_absorbers(gpu_ctx, tables, mode):
    """Tables without absorbers (n_abs = 0; the fill gases' CIA and Rayleigh
    only): forward against the oracle, a full and a partial window."""
    t = _no_absorber_tables(tables)
    Ts = [_profile(60), _profile(150, 1700.0)]
    batch = batch_from_models(Ts, 1e6, 1e-4, np.zeros((2, 0)), R_JUP, R_SUN, GM_JUP, [0, 90], [t.n_wn, 600])
    ch = _channels(t)
    nat, binned, st = _run(gpu_ctx, t, batch, ch, mode, 200)
    worst = _check(t, batch, ch, mode, nat, binned, st)
    print(f"{mode}: no absorbers worst rel err {worst:.2e}")
    assert worst <= TOL[mode]


def test_no_absorbers_gradient(gpu_ctx, tables):
    """chi^2 gradient (FP64 forward) with tables without absorbers: d/dT and
    d/dRp against the oracle's reference gradient; no mixing-ratio outputs."""
    from paper_1912_07759_amd import trx
    t = _no_absorber_tables(tables)
    Ts = [_profile(60), _profile(100, 1500.0)]
    batch = batch_from_models(Ts, 1e6, 1e-4, np.zeros((2, 0)), R_JUP, R_SUN, GM_JUP, 0, t.n_wn)
    ch = _channels(t)
    refs = [oracle.forward_model(batch.model(b), t, ch)["binned"] for b in range(2)]
    sigma = np.full(len(ch.lo), 50e-6)
    obs = np.stack([r * (1.0 + 2e-4 * np.sin(np.arange(len(ch.lo)) + b)) for b, r in enumerate(refs)])
    Tt = trx.Tables.from_synth(gpu_ctx, t)
    bins = trx.Bins(gpu_ctx, Tt, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=100)
    out = trx.chi2_grad(gpu_ctx, Tt, db, bins, obs, sigma, "fp64")
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    bins.close()
    Tt.close()
    assert np.all(g["status"] == 0), g["status"]
    off = batch.layer_off
    for b in range(2):
        ref = oracle.chi2_and_grad(batch.model(b), t, ch, obs[b], sigma)
        assert abs(g["chi2"][b] - ref["chi2"]) <= 1e-5 * ref["chi2"]
        v = np.concatenate([g["dT"][off[b]:off[b + 1]], [g["dRp"][b]]])
        r = np.concatenate([ref["dT"], [ref["dRp"]]])
        assert np.all(np.isfinite(v))
        norm = np.linalg.norm(v - r) / np.linalg.norm(r)
        big = np.abs(r) >= 1e-3 * np.max(np.abs(r))
        comp = float(np.max(np.abs(v[big] - r[big]) / np.abs(r[big])))
        print(f"no absorbers model {b}: grad norm err {norm:.2e} comp err {comp:.2e}")
        assert norm <= 1e-4 and comp <= 1e-4


def test_empty_batch_is_rejected(gpu_ctx, tables):
    """A batch of no models is an invalid argument at every entry point that
    takes one (trx_forward, trx_forward_noalloc, trx_emission, trx_chi2_grad,
    trx_plan_launch): TRX_E_INVALID_ARG with its message, nothing launched,
    and the context works for the next call."""
    import ctypes

    import torch
    from paper_1912_07759_amd import trx
    L = trx.lib()
    Ts = [_profile(40)]
    batch = batch_from_models(Ts, 1e6, 1e-4, np.full((1, tables.n_abs), -4.0), R_JUP, R_SUN, GM_JUP,
                              0, tables.n_wn)
    ch = _channels(tables)
    T = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=40)
    plan = trx.Plan(gpu_ctx, T, bins, B_max=1, N_max=40, precision="fp32")
    try:
        dev = db.T.device
        nat = torch.empty((1, tables.n_wn), dtype=torch.float64, device=dev)
        binned = torch.empty((1, len(ch.lo)), dtype=torch.float64, device=dev)
        st = torch.empty(1, dtype=torch.int32, device=dev)
        f64 = torch.ones(len(ch.lo), dtype=torch.float64, device=dev)
        g = torch.empty(64, dtype=torch.float64, device=dev)
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        empty = db.cstruct(B=0)
        gpu_ctx.bind_stream()
        calls = {
            "trx_forward": lambda: L.trx_forward(gpu_ctx.h, T.h, ctypes.byref(empty), bins.h, trx.FP32,
                                                 p(nat), p(binned), p(st), None),
            "trx_forward_noalloc": lambda: L.trx_forward_noalloc(gpu_ctx.h, T.h, ctypes.byref(empty), bins.h,
                                                                 trx.FP32, p(nat), p(binned), p(st)),
            "trx_emission": lambda: L.trx_emission(gpu_ctx.h, T.h, ctypes.byref(empty), bins.h, trx.FP32, 4,
                                                   p(f64), p(nat), p(binned), p(st)),
            "trx_chi2_grad": lambda: L.trx_chi2_grad(gpu_ctx.h, T.h, ctypes.byref(empty), bins.h, trx.FP64,
                                                     p(binned), p(f64), 1, p(g), p(g), p(g), p(g), p(binned),
                                                     p(st)),
            "trx_plan_launch": lambda: L.trx_plan_launch(plan.h, ctypes.byref(empty), None, p(binned), p(st),
                                                         None, None, None, None, None, None),
        }
        for name, call in calls.items():
            rc = call()
            assert rc == 1, (name, rc)   # TRX_E_INVALID_ARG
            assert "batch.B must be >= 1" in gpu_ctx.last_error(), (name, gpu_ctx.last_error())
        # the same context and handles still run a model of the batch
        _, b1, s1 = trx.forward(gpu_ctx, T, db, bins, "fp32", native=False)
        torch.cuda.synchronize()
        assert int(s1[0]) == 0 and bool(torch.all(torch.isfinite(b1)))
    finally:
        plan.close()
        bins.close()
        T.close()
