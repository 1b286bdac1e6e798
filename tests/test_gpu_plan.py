"""GPU tests of the batched plan (a9): graph replays, a B below capacity,
per-model plain launches, the variant autotuner and its cache, all against
the one-shot trx_forward of the same library and against the FP64 oracle."""

import json
import os

import numpy as np
import pytest
import torch

from synth.workloads import make_config
from parity_util import TOL, binned_rel_err, native_rel_err, oracle_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ragged():
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(3, n_wn=3000, n_lines=300, B=12)
    return tables, batch, ch


def _setup(ctx, tables, batch, ch):
    from paper_1912_07759_amd import trx
    T = trx.Tables.from_synth(ctx, tables)
    bins = trx.Bins(ctx, T, ch.lo, ch.hi)
    db = trx.DeviceBatch.from_synth(batch, max_layers=200)
    return T, bins, db


def _np(t):
    return None if t is None else t.detach().cpu().numpy().copy()


def _window_equal(a, b, batch):
    for i in range(a.shape[0]):
        lo, hi = int(batch.wn_lo[i]), int(batch.wn_hi[i])
        assert np.array_equal(a[i, lo:hi], b[i, lo:hi]), f"model {i} differs"


@pytest.mark.parametrize("mode", ["bf16x2", "fp32", "fp64"])
def test_graph_plan_matches_forward_and_oracle(gpu_ctx, ragged, mode):
    """A graph plan gives the bits of trx_forward (same kernels, same
    variant) and stays within the mode's tolerance of the oracle."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = ragged
    T, bins, db = _setup(gpu_ctx, tables, batch, ch)
    ref_nat, ref_bin, ref_st = trx.forward(gpu_ctx, T, db, bins, mode)
    ref_nat, ref_bin, ref_st = _np(ref_nat), _np(ref_bin), _np(ref_st)
    plan = trx.Plan(gpu_ctx, T, bins, B_max=16, N_max=200, precision=mode, graph=True)
    nat, binned, st = plan.launch(db, native=True)
    torch.cuda.synchronize()
    assert np.array_equal(_np(st), ref_st) and not ref_st.any()
    _window_equal(_np(nat), ref_nat, batch)
    assert np.array_equal(_np(binned), ref_bin, equal_nan=True)
    _, ref = oracle_batch(tables, batch, ch, mode, models=[0, 5, 11])
    for k, b in enumerate([0, 5, 11]):
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        e = native_rel_err(_np(nat)[b], ref[k]["depth"], lo, hi)
        e2 = binned_rel_err(_np(binned)[b], ref[k]["binned"])
        print(f"plan {mode} model {b}: native {e:.2e} binned {e2:.2e}")
        assert e <= TOL[mode] and e2 <= TOL[mode]
    plan.close()
    bins.close()
    T.close()


def test_graph_replays_and_smaller_batch(gpu_ctx, ragged):
    """Replays with unrelated eager work in between give identical results;
    a launch with B below the captured count replays the same graph and
    reproduces the first B models."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = ragged
    T, bins, db = _setup(gpu_ctx, tables, batch, ch)
    plan = trx.Plan(gpu_ctx, T, bins, B_max=12, N_max=200, precision="bf16x2", graph=True)
    _, b0, s0 = plan.launch(db)
    first = _np(b0)
    for r in range(3):
        x = torch.randn(1 << 20, device="cuda")
        y = (x * 2).sum()
        torch.cuda.synchronize()
        _, b1, s1 = plan.launch(db)
        torch.cuda.synchronize()
        assert float(y) == float(y)
        assert np.array_equal(_np(b1), first, equal_nan=True), f"replay {r} differs"
        assert not _np(s1).any()
    # same pointers, B = 5: only the count changes
    small_db = _Sub(db, 5)
    _, b2, s2 = plan.launch(small_db)
    torch.cuda.synchronize()
    assert b2.shape[0] == 5
    assert np.array_equal(_np(b2), first[:5], equal_nan=True)
    # and back to the full batch
    _, b3, _ = plan.launch(db)
    torch.cuda.synchronize()
    assert np.array_equal(_np(b3), first, equal_nan=True)
    plan.close()
    bins.close()
    T.close()


class _Sub:
    """The first B models of a DeviceBatch, sharing its device arrays."""

    def __init__(self, db, B):
        self.db, self.B = db, B

    def cstruct(self):
        return self.db.cstruct(B=self.B)


def test_batched_equals_per_model_plain(gpu_ctx, ragged):
    """The batched persistent launch equals one plain launch per model
    (non-persistent kernel, B = 1), model by model."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = ragged
    T, bins, db = _setup(gpu_ctx, tables, batch, ch)
    plan = trx.Plan(gpu_ctx, T, bins, B_max=12, N_max=200, precision="bf16x2", graph=True)
    nat, binned, _ = plan.launch(db, native=True)
    nat, binned = _np(nat), _np(binned)
    single = trx.Plan(gpu_ctx, T, bins, B_max=1, N_max=200, precision="bf16x2", graph=False,
                      persistent=False)
    for b in range(batch.B):
        sb = trx.DeviceBatch.from_synth(batch.subset([b]), max_layers=200)
        n1, b1, s1 = single.launch(sb, native=True)
        torch.cuda.synchronize()
        assert int(_np(s1)[0]) == 0
        lo, hi = int(batch.wn_lo[b]), int(batch.wn_hi[b])
        assert np.array_equal(_np(n1)[0, lo:hi], nat[b, lo:hi]), f"model {b} native differs"
        assert np.array_equal(_np(b1)[0], binned[b], equal_nan=True), f"model {b} binned differs"
    single.close()
    plan.close()
    bins.close()
    T.close()


def test_autotune_and_cache(gpu_ctx, ragged, tmp_path):
    """The autotuner picks a variant, results keep their bits under every
    variant, and a second plan of the same bucket reads the cached choice."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = ragged
    T, bins, db = _setup(gpu_ctx, tables, batch, ch)
    plan = trx.Plan(gpu_ctx, T, bins, B_max=12, N_max=200, precision="bf16x2", graph=True)
    _, ref, _ = plan.launch(db)
    ref = _np(ref)
    cache = str(tmp_path / "tune.json")
    choice = plan.autotune(db, cache)
    print("autotune choice:", choice)
    assert choice.startswith("persistent=")
    data = json.load(open(cache))
    assert list(data.values()) == [choice]
    _, got, _ = plan.launch(db)
    assert np.array_equal(_np(got), ref, equal_nan=True)
    for v in ["persistent=0 group=0 spans=1 rbw=0 occ=3", "persistent=1 group=8 spans=4 rbw=2 occ=3",
              "persistent=1 group=0 spans=2 rbw=0 occ=3"]:
        plan.set_variant(v)
        assert plan.describe() == v
        _, got, _ = plan.launch(db)
        assert np.array_equal(_np(got), ref, equal_nan=True), v
    plan2 = trx.Plan(gpu_ctx, T, bins, B_max=12, N_max=200, precision="bf16x2", graph=True)
    assert plan2.autotune(db, cache) == choice
    plan2.close()
    plan.close()
    bins.close()
    T.close()


@pytest.mark.parametrize("mode", ["bf16x2", "fp32", "fp64"])
def test_tile_variants_keep_bits(gpu_ctx, mode):
    """Models of at most 128 layers: one or two ray blocks per wave, the
    four-workgroup build of the persistent kernel and (FP64) span groups of
    1 to 8 give the same bits; the autotuner searches them and variants
    that do not fit the plan are refused."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(3, n_wn=3000, n_lines=300, B=10, layer_range=(50, 128))
    T, bins, db = _setup(gpu_ctx, tables, batch, ch)
    db = trx.DeviceBatch.from_synth(batch, max_layers=128)
    plan = trx.Plan(gpu_ctx, T, bins, B_max=10, N_max=128, precision=mode, graph=True)
    try:
        _, ref, _ = plan.launch(db)
        ref = _np(ref)
        if mode == "fp64":
            variants = [f"persistent=0 group=0 spans={k} rbw=0 occ=3" for k in (1, 2, 8)]
        else:
            variants = ["persistent=1 group=0 spans=8 rbw=1 occ=3", "persistent=1 group=0 spans=8 rbw=2 occ=3",
                        "persistent=1 group=0 spans=4 rbw=1 occ=4", "persistent=0 group=0 spans=2 rbw=2 occ=3",
                        "persistent=1 group=0 spans=8 rbw=2 occ=4"]
        for v in variants:
            plan.set_variant(v)
            assert plan.describe() == v
            for _ in range(2):
                _, got, st = plan.launch(db)
                assert not _np(st).any()
                assert np.array_equal(_np(got), ref, equal_nan=True), v
        choice = plan.autotune(db)
        print(f"{mode} autotune choice: {choice}")
        _, got, _ = plan.launch(db)
        assert np.array_equal(_np(got), ref, equal_nan=True)
        _, r0 = oracle_batch(tables, batch, ch, mode, models=[0])
        assert binned_rel_err(ref[0], r0[0]["binned"]) <= TOL[mode]
    finally:
        plan.close()
    big = trx.Plan(gpu_ctx, T, bins, B_max=4, N_max=200, precision=mode)
    try:
        for v in ("persistent=1 group=0 spans=8 rbw=1 occ=3", "persistent=0 group=0 spans=8 rbw=2 occ=4"):
            if mode == "fp64" and "persistent=1" in v:
                v = v.replace("persistent=1", "persistent=0")
            with pytest.raises(trx.TrxError):
                big.set_variant(v)
    finally:
        big.close()
        bins.close()
        T.close()


@pytest.mark.parametrize("mode", ["bf16x2", "fp32", "bf16x3"])
def test_two_pass_build_keeps_bits(gpu_ctx, mode):
    """Models of up to 200 layers (seven ray blocks): the four-workgroup
    build, which takes a wave's two ray blocks in two passes over each span
    with one set of accumulators, gives the bits of the default kernel, in
    single-chunk models and in a model of more than 128 slots (restaged
    per pass) alike."""
    from paper_1912_07759_amd import trx
    from synth.constants import GM_JUP, R_JUP, R_SUN
    from synth.workloads import batch_from_models
    tables, batch, ch = make_config(3, n_wn=3000, n_lines=300, B=10, layer_range=(150, 200))
    # a three-level zig-zag temperature profile of 200 layers: some 180
    # table corners and CIA nodes, two staging chunks (restaged per pass)
    i = np.arange(200)
    zig = np.where(i % 2 == 0, 250.0, 3300.0) + np.linspace(0.0, 900.0, 200)
    zig = np.where(i % 4 == 1, 1700.0 + np.linspace(0.0, 900.0, 200), zig)
    zb = batch_from_models([zig], 1e6, 1e-4, np.array([[-4.0, -5.0, -6.0, -3.5, -7.0]]), R_JUP, R_SUN, GM_JUP,
                           [0], [tables.n_wn])
    T, bins, _ = _setup(gpu_ctx, tables, batch, ch)
    db = trx.DeviceBatch.from_synth(batch, max_layers=200)
    dz = trx.DeviceBatch.from_synth(zb, max_layers=200)
    plan = trx.Plan(gpu_ctx, T, bins, B_max=10, N_max=200, precision=mode, graph=True)
    try:
        plan.set_variant("persistent=1 group=0 spans=8 rbw=0 occ=3")
        _, zref, _ = plan.launch(dz)
        zref = _np(zref)
        _, ref, _ = plan.launch(db)
        ref = _np(ref)
        v = "persistent=1 group=0 spans=8 rbw=2 occ=4"
        plan.set_variant(v)
        assert plan.describe() == v
        for _ in range(2):
            _, got, st = plan.launch(db)
            assert not _np(st).any()
            assert np.array_equal(_np(got), ref, equal_nan=True)
            _, got, st = plan.launch(dz)
            assert not _np(st).any()
            assert np.array_equal(_np(got), zref, equal_nan=True)
        _, r0 = oracle_batch(tables, batch, ch, mode, models=[0])
        assert binned_rel_err(ref[0], r0[0]["binned"]) <= TOL[mode]
        _, rz = oracle_batch(tables, zb, ch, mode, models=[0])
        assert binned_rel_err(zref[0], rz[0]["binned"]) <= TOL[mode]
    finally:
        plan.close()
        bins.close()
        T.close()


def test_plan_errors(gpu_ctx, ragged):
    from paper_1912_07759_amd import trx
    tables, batch, ch = ragged
    T, bins, db = _setup(gpu_ctx, tables, batch, ch)
    plan = trx.Plan(gpu_ctx, T, bins, B_max=4, N_max=200, precision="fp32")
    with pytest.raises(trx.TrxError) as e:
        plan.launch(db)  # B = 12 > B_max
    assert e.value.code == 1
    with pytest.raises(trx.TrxError):
        plan.set_variant("persistent=2")
    with pytest.raises(trx.TrxError) as e:
        trx.Plan(gpu_ctx, T, bins, B_max=4, N_max=300, precision="fp32")
    assert e.value.code == 4
    plan.close()
    bins.close()
    T.close()


class _DeviceArray:
    """A device buffer owned by the library, seen by torch without a copy."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False),
                                         "version": 2}


class _OwnBatch:
    def __init__(self, c, B):
        self.c, self.B = c, B

    def cstruct(self):
        return self.c


def test_plan_owned_input_buffers(gpu_ctx, ragged):
    """trx_plan_batch: the plan's own device input buffers (B_max models of
    N_max layers, default constants), filled by the caller with a batch of
    fewer models, give the same result as the caller's own buffers."""
    import ctypes
    from paper_1912_07759_amd import trx
    tables, batch, ch = ragged
    T, bins, db = _setup(gpu_ctx, tables, batch, ch)
    plan = trx.Plan(gpu_ctx, T, bins, B_max=16, N_max=200, precision="bf16x2", graph=True)
    own = trx.BatchC()
    gpu_ctx.check(trx.lib().trx_plan_batch(plan.h, ctypes.byref(own)))
    assert own.B == 16 and own.max_layers == 200 and own.gravity == 0
    assert own.he_h2_ratio == 0.17 and own.k_B == 1.380649e-23 and own.amu_kg == 1.66053906660e-27
    for name, src, ts in (("n_layers", db.n_layers, "<i4"), ("layer_off", db.layer_off, "<i8"),
                          ("T_K", db.T, "<f8"), ("p_bot_Pa", db.p_bot, "<f8"),
                          ("p_top_Pa", db.p_top, "<f8"), ("log10_vmr", db.log10_vmr, "<f8"),
                          ("Rp_m", db.Rp, "<f8"), ("Rs_m", db.Rs, "<f8"), ("GM_m3s2", db.GM, "<f8"),
                          ("wn_lo", db.wn_lo, "<i4"), ("wn_hi", db.wn_hi, "<i4")):
        dst = torch.as_tensor(_DeviceArray(getattr(own, name), src.numel(), ts), device="cuda")
        dst.copy_(src.reshape(-1))
    own.B, own.max_layers = db.B, db.max_layers
    own.he_h2_ratio, own.k_B, own.amu_kg, own.gravity = db.he_h2, db.k_B, db.amu, db.gravity
    nat, binned, st = plan.launch(_OwnBatch(own, db.B), native=True)
    nat, binned, st = nat.cpu().numpy(), binned.cpu().numpy(), st.cpu().numpy()
    ref_nat, ref_binned, ref_st = trx.forward(gpu_ctx, T, db, bins, "bf16x2")
    gpu_ctx.synchronize()
    plan.close()
    bins.close()
    T.close()
    assert np.array_equal(st, ref_st.cpu().numpy()) and np.all(st == 0)
    assert np.array_equal(nat, ref_nat.cpu().numpy(), equal_nan=True)
    assert np.array_equal(binned, ref_binned.cpu().numpy(), equal_nan=True)
