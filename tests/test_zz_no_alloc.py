"""trx_forward_noalloc (the forward model in the library's fixed device
array, no allocation) against trx_forward (which allocates its workspace):
the same kernels on the same inputs, so the outputs must agree bit for bit,
on two calls in a row, the second with a smaller batch; a batch that does
not fit the array is rejected before any work is enqueued."""

import numpy as np
import pytest
import torch

from synth.workloads import make_config

pytestmark = pytest.mark.gpu


def _outputs(B, n_wn, n_ch, dev="cuda"):
    return (torch.full((B, n_wn), float("nan"), dtype=torch.float64, device=dev),
            torch.full((B, n_ch), float("nan"), dtype=torch.float64, device=dev),
            torch.full((B,), -1, dtype=torch.int32, device=dev))


@pytest.mark.parametrize("mode", ["bf16x2", "fp32", "fp64"])
def test_noalloc_forward_matches_trx_forward(gpu_ctx, mode):
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(3, n_wn=3000, n_lines=200, B=16)
    T = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, T, ch.lo, ch.hi)
    try:
        # second call: fewer models, fewer layers, other windows
        for idx in (list(range(16)), [5, 2, 11]):
            sub = batch.subset(idx)
            db = trx.DeviceBatch.from_synth(sub)
            print(f"noalloc {mode}: B={sub.B} max_layers={db.max_layers}", flush=True)
            ref = _outputs(sub.B, tables.n_wn, len(ch.lo))
            got = _outputs(sub.B, tables.n_wn, len(ch.lo))
            trx.forward(gpu_ctx, T, db, bins, mode, out_native=ref[0], out_binned=ref[1],
                        out_status=ref[2])
            trx.forward_noalloc(gpu_ctx, T, db, bins, mode, *got)
            torch.cuda.synchronize()
            r = [x.cpu().numpy() for x in ref]
            g = [x.cpu().numpy() for x in got]
            assert np.array_equal(g[2], r[2]) and np.all(g[2] == 0), (g[2], r[2])
            assert np.array_equal(g[0], r[0], equal_nan=True)
            assert np.array_equal(g[1], r[1], equal_nan=True)
            # the window of every model is written (finite), the rest untouched
            for b in range(sub.B):
                lo, hi = int(sub.wn_lo[b]), int(sub.wn_hi[b])
                assert np.all(np.isfinite(g[0][b, lo:hi]))
                assert np.all(np.isnan(g[0][b, :lo])) and np.all(np.isnan(g[0][b, hi:]))
    finally:
        bins.close()
        T.close()


def test_noalloc_rejects_a_batch_beyond_the_array(gpu_ctx):
    """200 models of up to 200 layers need ~130 MB of workspace in the
    split-bf16 mode, more than the fixed array: the call fails with
    TRX_E_UNSUPPORTED and a message, and writes nothing."""
    from paper_1912_07759_amd import trx
    tables, batch, ch = make_config(3, n_wn=3000, n_lines=50, B=200)
    T = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, T, ch.lo, ch.hi)
    try:
        db = trx.DeviceBatch.from_synth(batch, max_layers=200)
        out = _outputs(batch.B, tables.n_wn, len(ch.lo))
        with pytest.raises(trx.TrxError) as e:
            trx.forward_noalloc(gpu_ctx, T, db, bins, "bf16x2", *out)
        assert e.value.code == 4 and "split the batch" in str(e.value)
        torch.cuda.synchronize()
        assert torch.all(out[2] == -1) and torch.all(torch.isnan(out[1]))
    finally:
        bins.close()
        T.close()
