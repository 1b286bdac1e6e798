"""GPU parity of the exponential temperature scheme of the cross-sections
(sigma = a e^{-b/T} through the two bracketing grid temperatures, Opacities
section) against the FP64 oracle with t_interp="exp": transmission in every
precision (slot form and the FP64 dense path), ragged batches, tables with
non-positive values (the linear fallback), plans, emission, and the
gradient's refusal."""

import numpy as np
import pytest
import torch

import oracle
from synth.workloads import make_config
from parity_util import TOL, binned_rel_err, native_rel_err

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32", "bf16x2", "bf16x3"]


def _run(ctx, tables, batch, ch, mode, max_layers=None, t_interp="exp"):
    from paper_1912_07759_amd import trx
    T = trx.Tables.from_synth(ctx, tables, t_interp)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    try:
        db = trx.DeviceBatch.from_synth(batch, max_layers=max_layers)
        nat, binned, st = trx.forward(ctx, T, db, bins, mode)
        torch.cuda.synchronize()
        return nat.cpu().numpy(), binned.cpu().numpy(), st.cpu().numpy()
    finally:
        bins.close()
        T.close()


def _worst(tables, batch, ch, nat, binned, models=None):
    worst = 0.0
    for b in (range(batch.B) if models is None else models):
        r = oracle.forward_model(dict(batch.model(b), t_interp="exp"), tables, ch)
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        e1 = native_rel_err(nat[b], r["depth"], lo, hi)
        e2 = binned_rel_err(binned[b], r["binned"])
        assert np.all(np.isnan(nat[b][:lo])) and np.all(np.isnan(nat[b][hi:]))
        worst = max(worst, e1, e2)
    return worst


@pytest.mark.parametrize("mode", MODES)
def test_exp_single_model(gpu_ctx, mode):
    """5 absorbers, CIA and Rayleigh, 100 Guillot layers on a 3000-point
    grid (several spans, a ragged tail), binned to 50 channels."""
    tables, batch, ch = make_config(2, n_wn=3000, n_lines=300)
    nat, binned, st = _run(gpu_ctx, tables, batch, ch, mode)
    assert st[0] == 0
    w = _worst(tables, batch, ch, nat, binned)
    print(f"exp-T single {mode}: worst rel err {w:.3e}")
    assert w <= TOL[mode]


@pytest.mark.parametrize("mode", MODES)
def test_exp_ragged_batch(gpu_ctx, mode):
    """12 models of 50-200 layers (more layer slots than one staging chunk
    of the matrix-core kernel) and ragged windows."""
    tables, batch, ch = make_config(3, n_wn=3000, n_lines=300, B=12)
    nat, binned, st = _run(gpu_ctx, tables, batch, ch, mode, max_layers=200)
    assert np.all(st == 0)
    w = _worst(tables, batch, ch, nat, binned)
    print(f"exp-T ragged {mode}: worst rel err {w:.3e}")
    assert w <= TOL[mode]


def test_exp_differs_from_linear(gpu_ctx):
    """The scheme is applied: between table temperatures the two schemes
    differ far beyond the tolerance, on the GPU as in the oracle."""
    tables, batch, ch = make_config(2, n_wn=1500, n_lines=150)
    a, _, _ = _run(gpu_ctx, tables, batch, ch, "fp32", t_interp="exp")
    b, _, _ = _run(gpu_ctx, tables, batch, ch, "fp32", t_interp="linear")
    d = float(np.max(np.abs(a[0] - b[0]) / np.abs(b[0])))
    r = oracle.forward_model(dict(batch.model(0), t_interp="exp"), tables)["depth"]
    s = oracle.forward_model(batch.model(0), tables)["depth"]
    do = float(np.max(np.abs(r - s) / s))
    print(f"exp vs linear: GPU {d:.2e}, oracle {do:.2e}")
    assert d > 10 * TOL["fp32"] and abs(d - do) <= 2 * TOL["fp32"]


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x2"])
def test_exp_fallback_at_nonpositive_values(gpu_ctx, mode):
    """Zeros at some (T node, P node, wavenumber) points of the tables: the
    brackets touching them fall back to the linear scheme on both sides."""
    tables, batch, ch = make_config(2, n_wn=1500, n_lines=150)
    rng = np.random.default_rng(21)
    x = tables.xsec.copy()
    for i in range(x.shape[0]):
        for iT in range(x.shape[1]):
            x[i, iT, :, rng.integers(0, x.shape[3], 200)] = 0.0
    tables.xsec = x
    nat, binned, st = _run(gpu_ctx, tables, batch, ch, mode)
    assert st[0] == 0
    w = _worst(tables, batch, ch, nat, binned)
    print(f"exp-T fallback {mode}: worst rel err {w:.3e}")
    assert w <= TOL[mode]


def test_exp_fp64_dense_beyond_slot_form(gpu_ctx):
    """Models above the slot form's layer limit take the FP64 dense kernel,
    which forms each layer's exponential-scheme cross-sections itself."""
    tables, batch, ch = make_config(3, n_wn=1000, n_lines=100, B=3, layer_range=(240, 300))
    nat, binned, st = _run(gpu_ctx, tables, batch, ch, "fp64", max_layers=300)
    assert np.all(st == 0)
    w = _worst(tables, batch, ch, nat, binned)
    print(f"exp-T FP64 dense: worst rel err {w:.3e}")
    assert w <= TOL["fp64"]


@pytest.mark.parametrize("flags", ["persistent", "graph"])
def test_exp_plan_matches_eager(gpu_ctx, flags):
    """Plans over exponential-scheme tables give the eager call's bits."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(3, n_wn=2000, n_lines=200, B=10)
    T = trx.Tables.from_synth(gpu_ctx, tables, "exp")
    bins = trx.Bins(gpu_ctx, T, ch.lo, ch.hi)
    try:
        db = trx.DeviceBatch.from_synth(batch, max_layers=200)
        nat, binned, st = trx.forward(gpu_ctx, T, db, bins, "bf16x2")
        p = trx.Plan(gpu_ctx, T, bins, batch.B, 200, "bf16x2",
                     graph=(flags == "graph"), persistent=True)
        try:
            for _ in range(2):
                _, b2, s2 = p.launch(db)
                torch.cuda.synchronize()
                assert torch.equal(s2, st)
                assert torch.equal(torch.nan_to_num(b2, nan=-1.0), torch.nan_to_num(binned, nan=-1.0))
        finally:
            p.close()
        w = _worst(tables, batch, ch, nat.cpu().numpy(), binned.cpu().numpy(), models=[0, 4, 9])
        assert w <= TOL["bf16x2"]
    finally:
        bins.close()
        T.close()


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
def test_exp_emission(gpu_ctx, mode):
    """The emission model over exponential-scheme tables, native and binned
    against the oracle's emission model (per-point bounds of the emission
    tests)."""
    from test_gpu_emission import _check
    tables, batch, ch = make_config(3, n_wn=2000, n_lines=200, B=4)
    assert _check(gpu_ctx, tables, batch, ch, mode, 4, 5800.0, max_layers=200, t_interp="exp") <= 1.0


def test_exp_gradient_refused(gpu_ctx):
    """The gradient of the exponential scheme is not built: the call and a
    gradient plan are refused with TRX_E_UNSUPPORTED."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(2, n_wn=500, n_lines=50)
    T = trx.Tables.from_synth(gpu_ctx, tables, "exp")
    bins = trx.Bins(gpu_ctx, T, ch.lo, ch.hi)
    try:
        db = trx.DeviceBatch.from_synth(batch)
        obs = np.zeros((1, len(ch.lo)))
        sigma = np.full(len(ch.lo), 5e-5)
        with pytest.raises(trx.TrxError) as e:
            trx.chi2_grad(gpu_ctx, T, db, bins, obs, sigma, "fp32")
        assert e.value.code == 4   # TRX_E_UNSUPPORTED
        with pytest.raises(trx.TrxError) as e:
            trx.Plan(gpu_ctx, T, bins, 4, 100, "fp32", grad=True)
        assert e.value.code == 4   # TRX_E_UNSUPPORTED
    finally:
        bins.close()
        T.close()
