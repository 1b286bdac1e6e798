"""Shared helpers of the parity tests: run the oracle on the same seeded
inputs as the HIP library and compare element by element."""

import numpy as np

import oracle

# Tolerances (relative error of the transit depth against the FP64 oracle):
# FP64 mode follows the oracle's arithmetic to rounding; the fast modes are
# held to the 1e-6 target of the batched path.
TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x2": 1e-6, "bf16x3": 1e-6}


def oracle_tables_for(tables, precision):
    """Every mode is compared with the oracle on the FP64 tables, so the
    reported error of the FP32-storage modes includes the rounding of the
    stored tables (<= 6e-8 relative per value).  Rounding the oracle's tables
    to float32 instead is not an option for CIA, whose cm^5 values
    (~1e-46) are below the float32 range (the device keeps a rescaled FP32
    copy)."""
    return tables


def oracle_batch(tables, batch, channels, precision, models=None):
    t = oracle_tables_for(tables, precision)
    idx = list(range(batch.B)) if models is None else list(models)
    out = []
    for b in idx:
        out.append(oracle.forward_model(batch.model(b), t, channels))
    return idx, out


def native_rel_err(gpu_native_row, ref, lo, hi):
    g = np.asarray(gpu_native_row)[lo:hi]
    # a NaN would drop out of the callers' max(): reject it here
    assert np.all(np.isfinite(g)), "non-finite native depth inside the window"
    return float(np.max(np.abs(g - ref) / np.abs(ref)))


def binned_rel_err(gpu_binned_row, ref):
    g = np.asarray(gpu_binned_row)
    ok = ~np.isnan(ref)
    assert np.array_equal(np.isnan(g), ~ok), "NaN pattern of binned channels differs"
    if not ok.any():
        return 0.0
    return float(np.max(np.abs(g[ok] - ref[ok]) / np.abs(ref[ok])))
