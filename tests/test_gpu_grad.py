"""GPU parity of chi^2 and its gradient (a8, through trx_chi2_grad) against
the oracle's FP64 reference gradient and against central differences of the
library's own FP64 forward model; the autograd Function."""

import numpy as np
import pytest
import torch

import oracle
from synth.workloads import make_config, observation_noise

pytestmark = pytest.mark.gpu

# Reading A17: gradient error norm-wise and per component above 1e-3 of
# the largest component, against the FP64 reference.
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def problem():
    """Gradient workload, reduced: 100-layer perturbed Guillot profiles,
    7 absorbers, CIA and Rayleigh, 100 channels, 6 parameter points; the
    observation is the truth (point 0) binned by the oracle plus seeded
    50 ppm noise."""
    tables, batch, ch = make_config(4, n_wn=2500, n_lines=250, B=6)
    truth = oracle.forward_model(batch.model(0), tables, ch)["binned"]
    noise, sigma = observation_noise(4, 1, len(ch.lo))
    obs = np.tile(truth + noise[0], (batch.B, 1))
    return tables, batch, ch, obs, sigma


def _gpu(ctx, tables, batch, ch, obs, sigma, precision, T=None):
    from paper_1912_07759_amd import trx
    Tt = trx.Tables.from_synth(ctx, tables)
    bins = trx.Bins(ctx, Tt, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=100)
    out = trx.chi2_grad(ctx, Tt, db, bins, obs, sigma, precision)
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    bins.close()
    Tt.close()
    return res


def _grad_err(g, ref):
    v = np.concatenate([g["dT"], g["dlog10_vmr"], [g["dRp"]]])
    assert np.all(np.isfinite(v)), "non-finite gradient"
    r = np.concatenate([ref["dT"], ref["dlog10_vmr"], [ref["dRp"]]])
    norm = np.linalg.norm(v - r) / np.linalg.norm(r)
    big = np.abs(r) >= 1e-3 * np.max(np.abs(r))
    comp = np.max(np.abs(v[big] - r[big]) / np.abs(r[big]))
    return norm, comp


@pytest.mark.parametrize("mode", ["fp32", "bf16x2", "fp64"])
def test_gradient_matches_oracle(gpu_ctx, problem, mode):
    tables, batch, ch, obs, sigma = problem
    g = _gpu(gpu_ctx, tables, batch, ch, obs, sigma, mode)
    assert np.all(g["status"] == 0)
    off = batch.layer_off
    worst = 0.0
    for b in range(batch.B):
        ref = oracle.chi2_and_grad(batch.model(b), tables, ch, obs[b], sigma)
        assert abs(g["chi2"][b] - ref["chi2"]) <= 1e-5 * ref["chi2"]
        mine = {"dT": g["dT"][off[b]:off[b + 1]], "dlog10_vmr": g["dlog10_vmr"][b],
                "dRp": g["dRp"][b]}
        norm, comp = _grad_err(mine, ref)
        print(f"{mode} model {b}: chi2 {g['chi2'][b]:.6e} grad norm err {norm:.2e} comp err {comp:.2e}")
        worst = max(worst, norm, comp)
    assert worst <= GRAD_TOL


@pytest.mark.parametrize("mode", ["fp32", "bf16x2", "fp64"])
def test_gradient_deterministic(gpu_ctx, problem, mode):
    """Two runs of the same gradient call give the same bits: every sum of
    the adjoint (span partials, channel cotangents, shell boundaries) runs
    in a fixed order."""
    tables, batch, ch, obs, sigma = problem
    a = _gpu(gpu_ctx, tables, batch, ch, obs, sigma, mode)
    b = _gpu(gpu_ctx, tables, batch, ch, obs, sigma, mode)
    for k in ("chi2", "dT", "dlog10_vmr", "dRp", "status"):
        assert np.array_equal(a[k], b[k]), k


def test_gradient_central_differences(gpu_ctx, problem):
    """Central differences of chi^2 from the library's FP64 forward path
    (step 1e-4 K, 1e-6 dex, 1e-7 Rp) against the FP32 gradient."""
    tables, batch, ch, obs, sigma = problem
    base = _gpu(gpu_ctx, tables, batch, ch, obs, sigma, "fp32")
    b = 1
    off = int(batch.layer_off[b])

    def chi2_at(mod):
        bb = batch.subset([b])
        mod(bb)
        r = _gpu(gpu_ctx, tables, bb, ch, obs[b:b + 1], sigma, "fp64")
        return float(r["chi2"][0])

    checks = []
    for l in (3, 40, 77):
        h = 1e-4
        def up(bb, l=l, s=+1):
            bb.T[l] += s * h
        fd = (chi2_at(lambda bb: up(bb, s=+1)) - chi2_at(lambda bb: up(bb, s=-1))) / (2 * h)
        checks.append(("dT", l, fd, base["dT"][off + l]))
    for i in (0, 3):
        h = 1e-6
        def vm(bb, i=i, s=+1):
            bb.log10_vmr[0, i] += s * h
        fd = (chi2_at(lambda bb: vm(bb, s=+1)) - chi2_at(lambda bb: vm(bb, s=-1))) / (2 * h)
        checks.append(("dvmr", i, fd, base["dlog10_vmr"][b, i]))
    h = 1e-7 * batch.Rp[b]
    def rp(bb, s=+1):
        bb.Rp[0] += s * h
    fd = (chi2_at(lambda bb: rp(bb, s=+1)) - chi2_at(lambda bb: rp(bb, s=-1))) / (2 * h)
    checks.append(("dRp", 0, fd, base["dRp"][b]))
    for name, i, fd, g in checks:
        print(f"{name}[{i}]: central difference {fd:.8e} gradient {g:.8e}")
        assert abs(g - fd) <= 1e-4 * abs(fd) + 1e-9 * max(abs(c[2]) for c in checks)


def test_autograd_function(gpu_ctx, problem):
    from paper_1912_07759_amd import trx
    tables, batch, ch, obs, sigma = problem
    Tt = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, Tt, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=100)
    prob = trx.Chi2Problem(gpu_ctx, Tt, bins, db, obs, sigma, "fp32")
    T = db.T.clone().requires_grad_(True)
    v = db.log10_vmr.clone().requires_grad_(True)
    R = db.Rp.clone().requires_grad_(True)
    c2 = trx.TransitChi2.apply(T, v, R, prob)
    w = torch.arange(1, batch.B + 1, dtype=torch.float64, device=c2.device)
    (c2 * w).sum().backward()
    ref = trx.chi2_grad(gpu_ctx, Tt, db, bins, obs, sigma, "fp32")
    counts = torch.as_tensor(np.diff(batch.layer_off), device=c2.device)
    # a second run of the same call: the gradient is summed in a fixed order,
    # so the Function's outputs equal it bit for bit (times the weights)
    assert torch.equal(c2, ref["chi2"])
    assert torch.equal(T.grad, ref["dT"] * torch.repeat_interleave(w, counts))
    assert torch.equal(v.grad, ref["dlog10_vmr"] * w[:, None])
    assert torch.equal(R.grad, ref["dRp"] * w)
    bins.close()
    Tt.close()


def test_gradient_plan_graph(gpu_ctx, problem):
    """A graph-captured gradient plan reproduces trx_chi2_grad bit for bit,
    over replays with unrelated eager work in between and for a smaller B on
    the same graph."""
    from paper_1912_07759_amd import trx
    tables, batch, ch, obs, sigma = problem
    Tt = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, Tt, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=100)
    ref = {k: v.cpu().numpy() for k, v in
           trx.chi2_grad(gpu_ctx, Tt, db, bins, obs, sigma, "fp32").items() if v is not None}
    plan = trx.Plan(gpu_ctx, Tt, bins, B_max=batch.B, N_max=100, precision="fp32", graph=True,
                    grad=True)

    def check(out, n):
        for k in ("chi2", "dT", "dlog10_vmr", "dRp"):
            got = out[k].cpu().numpy()
            want = ref[k][:n] if k != "dT" else ref[k][:int(batch.layer_off[n])]
            assert np.array_equal(got, want), k
    try:
        for r in range(3):
            x = torch.randn(1 << 18, device="cuda").sum()
            torch.cuda.synchronize()
            out = plan.launch_grad(db, obs, sigma)
            torch.cuda.synchronize()
            assert float(x) == float(x)
            check(out, batch.B)
        sub = db.view(0)
        out = plan.launch_grad(sub, obs[:1], sigma)
        torch.cuda.synchronize()
        check(out, 1)
    finally:
        plan.close()
        bins.close()
        Tt.close()


def test_gradient_long_models_and_slot_limit(gpu_ctx):
    """Models of 40, 150 and 224 layers in one batch (224 takes the kernel
    variant for more than 160 rays) and a model whose zig-zag temperature
    profile touches more than 128 distinct table corners and CIA nodes
    (about 150: two slot chunks) against the oracle's reference gradient,
    next to a model whose scrambled profile touches more than 256 (about
    530): that one is flagged TRX_MODEL_GRAD_UNSUPPORTED with NaN outputs,
    its neighbours unaffected."""
    from paper_1912_07759_amd import trx
    from synth.atmosphere import guillot_T, log_midpoint_pressures, log_uniform_channels
    from synth.constants import GM_JUP, R_JUP, R_SUN
    from synth.workloads import Channels, batch_from_models, make_tables
    tables = make_tables(4, n_wn=700, n_lines=80)
    lo, hi = log_uniform_channels(tables.wn, 24)
    ch = Channels(lo, hi)
    g0 = GM_JUP / R_JUP ** 2
    Ts = [guillot_T(log_midpoint_pressures(1e6, 1e-4, N), g0, Ti)
          for N, Ti in ((40, 900.0), (150, 1500.0), (224, 2100.0))]
    # alternate layers on two branches, 250 -> 1450 K and 3300 -> 2100 K
    ramp = np.linspace(0.0, 1200.0, 120)
    zig = np.where(np.arange(120) % 2 == 0, 250.0 + ramp, 3300.0 - ramp)
    Ts.append(zig)
    # every layer on a different T bracket: 220 K + (7 l mod 29)/28 x 3250 K
    Ts.append(220.0 + (np.arange(200) * 7 % 29) / 28.0 * 3250.0)
    rng = np.random.default_rng(7)
    vmr = rng.uniform(-7.0, -3.0, (len(Ts), tables.n_abs))
    batch = batch_from_models(Ts, 1e6, 1e-4, vmr, R_JUP, R_SUN, GM_JUP, 0, tables.n_wn)
    refs = [oracle.forward_model(batch.model(b), tables, ch)["binned"] for b in range(4)]
    obs = np.stack([r * (1.0 + 2e-4 * np.sin(np.arange(len(ch.lo)) + b)) for b, r in enumerate(refs)]
                   + [refs[0]])
    Tt = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, Tt, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=224)
    out = trx.chi2_grad(gpu_ctx, Tt, db, bins, obs, np.full(len(ch.lo), 50e-6), "fp64")
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    bins.close()
    Tt.close()
    off = batch.layer_off
    assert np.all(g["status"][:4] == 0), g["status"]
    assert g["status"][4] & trx.GRAD_UNSUPPORTED
    assert np.all(np.isnan(g["dT"][off[4]:off[5]])) and np.isnan(g["dRp"][4])
    for b in range(4):
        ref = oracle.chi2_and_grad(batch.model(b), tables, ch, obs[b], np.full(len(ch.lo), 50e-6))
        mine = {"dT": g["dT"][off[b]:off[b + 1]], "dlog10_vmr": g["dlog10_vmr"][b], "dRp": g["dRp"][b]}
        norm, comp = _grad_err(mine, ref)
        print(f"N={len(Ts[b])}: grad norm err {norm:.2e} comp err {comp:.2e}")
        assert norm <= GRAD_TOL and comp <= GRAD_TOL, (b, norm, comp)


def test_gradient_constant_gravity_and_window(gpu_ctx):
    """The constant-gravity altitude recursion (g = GM/Rp^2) and a window
    of 480 of the 700 grid points, whose channels lie inside it: both
    against the oracle's reference gradient."""
    from paper_1912_07759_amd import trx
    from synth.atmosphere import guillot_T, log_midpoint_pressures, log_uniform_channels
    from synth.constants import GM_JUP, R_JUP, R_SUN
    from synth.workloads import Channels, batch_from_models, make_tables
    tables = make_tables(4, n_wn=700, n_lines=80)
    lo, hi = log_uniform_channels(tables.wn[110:590], 16)
    ch = Channels(lo, hi)
    g0 = GM_JUP / R_JUP ** 2
    Ts = [guillot_T(log_midpoint_pressures(1e6, 1e-4, 80), g0, Ti) for Ti in (1100.0, 1700.0)]
    rng = np.random.default_rng(11)
    vmr = rng.uniform(-7.0, -3.0, (2, tables.n_abs))
    sigma = np.full(len(ch.lo), 50e-6)
    for gravity in (0, 1):
        batch = batch_from_models(Ts, 1e6, 1e-4, vmr, R_JUP, R_SUN, GM_JUP, 100, 580, gravity=gravity)
        refs = [oracle.forward_model(batch.model(b), tables, ch)["binned"] for b in range(2)]
        obs = np.stack([r * (1.0 + 3e-4 * np.cos(np.arange(len(ch.lo)) + b)) for b, r in enumerate(refs)])
        Tt = trx.Tables.from_synth(gpu_ctx, tables)
        bins = trx.Bins(gpu_ctx, Tt, ch.lo, ch.hi)
        db = trx.DeviceBatch.from_synth(batch, max_layers=80)
        out = trx.chi2_grad(gpu_ctx, Tt, db, bins, obs, sigma, "fp64")
        g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
        bins.close()
        Tt.close()
        assert np.all(g["status"] == 0), g["status"]
        off = batch.layer_off
        for b in range(2):
            ref = oracle.chi2_and_grad(batch.model(b), tables, ch, obs[b], sigma)
            mine = {"dT": g["dT"][off[b]:off[b + 1]], "dlog10_vmr": g["dlog10_vmr"][b], "dRp": g["dRp"][b]}
            norm, comp = _grad_err(mine, ref)
            print(f"gravity={gravity} model {b}: grad norm err {norm:.2e} comp err {comp:.2e}")
            assert norm <= GRAD_TOL and comp <= GRAD_TOL, (gravity, b, norm, comp)


def test_large_workload_forward_and_gradient(gpu_ctx):
    """The large batched workload's shapes with fewer wavenumbers and models:
    40 T x 30 P tables of 10 absorbers with CIA and Rayleigh, five models of
    100-196 layers, three of them with 104-111 opacity slots (four 32-slot
    blocks in the gradient).  The split-bf16 forward against the oracle's
    depth, then chi^2 and its gradient (recompute mode, FP64 forward) against
    the oracle's reference gradient."""
    from paper_1912_07759_amd import trx
    from parity_util import TOL, binned_rel_err, native_rel_err
    tables, full, ch = make_config(5, n_wn=1200, n_lines=80, B=24)
    batch = full.subset([2, 3, 5, 12, 15])
    refs = [oracle.forward_model(batch.model(b), tables, ch) for b in range(batch.B)]
    Tt = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, Tt, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=200)
    nat, binned, st = trx.forward(gpu_ctx, Tt, db, bins, "bf16x2")
    gpu_ctx.synchronize()
    nat, binned, st = nat.cpu().numpy(), binned.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0), st
    worst = 0.0
    for b, r in enumerate(refs):
        worst = max(worst, native_rel_err(nat[b], r["depth"], 0, tables.n_wn),
                    binned_rel_err(binned[b], r["binned"]))
    print(f"large workload bf16x2 forward: worst rel err {worst:.2e}")
    assert worst <= TOL["bf16x2"]

    sigma = np.full(len(ch.lo), 50e-6)
    obs = np.stack([r["binned"] * (1.0 + 2e-4 * np.sin(np.arange(len(ch.lo)) + b))
                    for b, r in enumerate(refs)])
    out = trx.chi2_grad(gpu_ctx, Tt, db, bins, obs, sigma, "fp64")
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    bins.close()
    Tt.close()
    assert np.all(g["status"] == 0), g["status"]
    off = batch.layer_off
    for b in range(batch.B):
        ref = oracle.chi2_and_grad(batch.model(b), tables, ch, obs[b], sigma)
        assert abs(g["chi2"][b] - ref["chi2"]) <= 1e-5 * ref["chi2"]
        mine = {"dT": g["dT"][off[b]:off[b + 1]], "dlog10_vmr": g["dlog10_vmr"][b], "dRp": g["dRp"][b]}
        norm, comp = _grad_err(mine, ref)
        print(f"large workload model {b} (N={int(batch.n_layers[b])}): grad norm err {norm:.2e} comp err {comp:.2e}")
        assert norm <= GRAD_TOL and comp <= GRAD_TOL, (b, norm, comp)
