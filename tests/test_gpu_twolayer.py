"""GPU parity of two-layer mixing profiles (Chemistry subsection; surface
value at and below a switch pressure, top value above, per-layer fill gases
and mean molecular weight) against the FP64 oracle: every precision, ragged
batches with cloud decks, the exponential temperature scheme, emission,
plans, the flags of models the library refuses, and the gradient's
refusal."""

import numpy as np
import pytest
import torch

import oracle
from synth.workloads import make_config, with_cloud_decks, with_two_layer_profiles
from parity_util import TOL, binned_rel_err, native_rel_err

pytestmark = pytest.mark.gpu

MODES = ["fp64", "fp32", "bf16x2", "bf16x3"]


def _run(ctx, tables, batch, ch, mode, max_layers=None, t_interp="linear"):
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


def _worst(tables, batch, ch, nat, binned, models=None, t_interp="linear"):
    worst = 0.0
    for b in (range(batch.B) if models is None else models):
        r = oracle.forward_model(dict(batch.model(b), t_interp=t_interp), tables, ch)
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        worst = max(worst, native_rel_err(nat[b], r["depth"], lo, hi), binned_rel_err(binned[b], r["binned"]))
        assert np.all(np.isnan(nat[b][:lo])) and np.all(np.isnan(nat[b][hi:]))
    return worst


def _runs(batch, b):
    """Number of runs of one chemistry of model b (distinct switch layers
    inside the model, plus one)."""
    m = batch.model(b)
    _, P = oracle.pressure_grid(m["p_bot"], m["p_top"], len(m["T"]))
    cuts = set()
    for i in range(len(m["log10_vmr"])):
        if m["log10_vmr_top"][i] != m["log10_vmr"][i]:
            l = int(np.sum(P >= m["vmr_switch"][i]))
            if 0 < l < len(P):
                cuts.add(l)
    return len(cuts) + 1


@pytest.mark.parametrize("mode", MODES)
def test_two_layer_single_model(gpu_ctx, mode):
    """5 absorbers, CIA and Rayleigh, 100 Guillot layers on a 3000-point
    grid, three switch pressures (up to four runs), binned."""
    tables, batch, ch = make_config(2, n_wn=3000, n_lines=300)
    tb = with_two_layer_profiles(batch, 7, n_switch=3)
    nat, binned, st = _run(gpu_ctx, tables, tb, ch, mode)
    assert st[0] == 0, st
    w = _worst(tables, tb, ch, nat, binned)
    print(f"two-layer single {mode}: {_runs(tb, 0)} runs, worst rel err {w:.3e}")
    assert w <= TOL[mode]


@pytest.mark.parametrize("mode", MODES)
def test_two_layer_ragged_batch_with_decks(gpu_ctx, mode):
    """16 models of 50-200 layers with ragged windows, two switch pressures
    each, and cloud decks (none, finite, opaque) on top."""
    tables, batch, ch = make_config(3, n_wn=3000, n_lines=300, B=16)
    tb = with_two_layer_profiles(with_cloud_decks(batch, 4), 11)
    nat, binned, st = _run(gpu_ctx, tables, tb, ch, mode, max_layers=200)
    assert np.all(st == 0), st
    w = _worst(tables, tb, ch, nat, binned)
    print(f"two-layer ragged {mode}: runs {[_runs(tb, b) for b in range(tb.B)]}, worst rel err {w:.3e}")
    assert w <= TOL[mode]


@pytest.mark.parametrize("mode", ["fp64", "fp32", "bf16x2"])
def test_two_layer_exp_t(gpu_ctx, mode):
    """Two-layer profiles over tables in the exponential temperature
    scheme (the layer slots padded per run)."""
    tables, batch, ch = make_config(3, n_wn=2000, n_lines=200, B=8)
    tb = with_two_layer_profiles(batch, 5)
    nat, binned, st = _run(gpu_ctx, tables, tb, ch, mode, max_layers=200, t_interp="exp")
    assert np.all(st == 0), st
    w = _worst(tables, tb, ch, nat, binned, t_interp="exp")
    print(f"two-layer exp-T {mode}: worst rel err {w:.3e}")
    assert w <= TOL[mode]


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
def test_two_layer_emission(gpu_ctx, mode):
    """The emission model with two-layer profiles, against the oracle's
    emission model (per-point bounds of the emission tests)."""
    from paper_1912_07759_amd import trx
    from test_gpu_emission import _check
    tables, batch, ch = make_config(3, n_wn=2000, n_lines=200, B=4)
    tb = with_two_layer_profiles(batch, 13)
    assert _check(gpu_ctx, tables, tb, ch, mode, 4, 5800.0, max_layers=200) <= 1.0


@pytest.mark.parametrize("graph", [False, True])
def test_two_layer_plan(gpu_ctx, graph):
    """A TRX_PLAN_TWO_LAYER plan gives the eager call's bits on a two-layer
    batch and the oracle's values on a constant one; a plan without the
    flag refuses a two-layer batch."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(3, n_wn=2000, n_lines=200, B=10)
    tb = with_two_layer_profiles(batch, 17)
    T = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, T, ch.lo, ch.hi)
    try:
        db = trx.DeviceBatch.from_synth(tb, max_layers=200)
        _, binned, st = trx.forward(gpu_ctx, T, db, bins, "bf16x2")
        p = trx.Plan(gpu_ctx, T, bins, tb.B, 200, "bf16x2", graph=graph, two_layer=True)
        try:
            for _ in range(2):
                _, b2, s2 = p.launch(db)
                torch.cuda.synchronize()
                assert torch.equal(s2, st)
                assert torch.equal(torch.nan_to_num(b2, nan=-1.0), torch.nan_to_num(binned, nan=-1.0))
            dc = trx.DeviceBatch.from_synth(batch, max_layers=200)
            _, bc, sc = p.launch(dc)
            torch.cuda.synchronize()
            assert not sc.any()
            bc = bc.cpu().numpy()
            for b in (0, 5):
                r = oracle.forward_model(batch.model(b), tables, ch)
                assert binned_rel_err(bc[b], r["binned"]) <= TOL["bf16x2"]
        finally:
            p.close()
        q = trx.Plan(gpu_ctx, T, bins, tb.B, 200, "bf16x2", graph=graph)
        try:
            with pytest.raises(trx.TrxError) as e:
                q.launch(db)
            assert e.value.code == 1   # TRX_E_INVALID_ARG
        finally:
            q.close()
    finally:
        bins.close()
        T.close()


def test_two_layer_flags(gpu_ctx):
    """Models the library refuses, next to valid ones: more than
    TRX_MAX_REGIMES runs (TRX_MODEL_UNSUPPORTED), a run whose absorbers sum
    to 1 or more, a switch pressure that is not positive, a top value that
    is not finite (TRX_MODEL_BAD_CHEMISTRY); their outputs are NaN."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(3, n_wn=1000, n_lines=100, B=6)
    tb = with_two_layer_profiles(batch, 19)
    na = tb.log10_vmr.shape[1]
    m = tb.model(1)
    _, P = oracle.pressure_grid(m["p_bot"], m["p_top"], len(m["T"]))
    # model 1: five distinct switches inside the model -> six runs
    tb.log10_vmr_top[1] = tb.log10_vmr[1] - 1.0
    tb.vmr_switch[1] = P[np.linspace(5, len(P) - 5, na).astype(int)]
    tb.log10_vmr_top[2, 0] = np.log10(0.7)          # the top run sums above 1
    tb.log10_vmr_top[2, 1] = np.log10(0.4)
    tb.vmr_switch[2, :2] = 1e3
    tb.vmr_switch[3, 0] = -1.0                       # not positive
    tb.log10_vmr_top[4, 2] = np.inf                  # not finite
    nat, binned, st = _run(gpu_ctx, tables, tb, ch, "fp32", max_layers=200)
    assert st[0] == 0 and st[5] == 0
    assert st[1] & trx.UNSUPPORTED
    assert st[2] & trx.BAD_CHEMISTRY and st[3] & trx.BAD_CHEMISTRY and st[4] & trx.BAD_CHEMISTRY
    for b in (1, 2, 3, 4):
        lo, hi = int(tb.wn_lo[b]), int(tb.wn_hi[b])
        assert np.all(np.isnan(nat[b][lo:hi])) and np.all(np.isnan(binned[b]))
    assert _worst(tables, tb, ch, nat, binned, models=[0, 5]) <= TOL["fp32"]


def test_two_layer_gradient_refused(gpu_ctx):
    """The gradient of two-layer profiles is not built: the call and a
    two-layer gradient plan are refused with TRX_E_UNSUPPORTED."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(2, n_wn=500, n_lines=50)
    tb = with_two_layer_profiles(batch, 23)
    T = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, T, ch.lo, ch.hi)
    try:
        db = trx.DeviceBatch.from_synth(tb)
        with pytest.raises(trx.TrxError) as e:
            trx.chi2_grad(gpu_ctx, T, db, bins, np.zeros((1, len(ch.lo))), np.full(len(ch.lo), 5e-5), "fp32")
        assert e.value.code == 4   # TRX_E_UNSUPPORTED
        with pytest.raises(trx.TrxError) as e:
            trx.Plan(gpu_ctx, T, bins, 4, 100, "fp32", grad=True, two_layer=True)
        assert e.value.code == 4
    finally:
        bins.close()
        T.close()
