"""Pins of the oracle's reference gradient: complex-step differentiation of
the oracle forward model (Squire & Trapp 1998; exact to rounding because every
step is analytic inside a fixed bracket) and central finite differences.
CPU only."""

import numpy as np
import pytest

import oracle
from oracle import forward as F
from synth.atmosphere import guillot_T, log_midpoint_pressures, log_uniform_channels
from synth.workloads import Channels, make_config

H_CS = 1e-30


def _setup(N=12, gravity=0, n_wn=300, lo=10, hi=290, n_ch=7):
    tables, batch, _ = make_config(2, n_wn=n_wn, n_lines=60)
    m = batch.model(0)
    m["T"] = (guillot_T(log_midpoint_pressures(1e6, 1e-4, N), 25.0, 1200.0)
              + np.linspace(0.0, 30.0, N) + 0.37)
    m["wn_lo"], m["wn_hi"] = lo, hi
    m["gravity"] = gravity
    clo, chi = log_uniform_channels(tables.wn[lo:hi], n_ch)
    ch = Channels(clo, chi)
    base = F.forward_model(m, tables, ch)["binned"]
    obs = base * (1.0 + 2e-3 * np.sin(np.arange(n_ch) + 0.3))
    sig = np.full(n_ch, 50e-6)
    return tables, m, ch, obs, sig


def _chi2(m, tables, ch, obs, sig):
    b = F.forward_model(m, tables, ch)["binned"]
    r = (b - obs) / sig
    return np.sum(r * r)


def _complex_step(m, tables, ch, obs, sig):
    N = len(m["T"])
    out = {"dT": np.zeros(N), "dlog10_vmr": np.zeros(len(m["log10_vmr"]))}
    for key, n in (("T", N), ("log10_vmr", len(m["log10_vmr"]))):
        for i in range(n):
            mm = dict(m)
            v = np.array(m[key], dtype=complex)
            v[i] += 1j * H_CS
            mm[key] = v
            out["dT" if key == "T" else "dlog10_vmr"][i] = np.imag(_chi2(mm, tables, ch, obs, sig)) / H_CS
    mm = dict(m)
    mm["Rp"] = m["Rp"] + 1j * H_CS
    out["dRp"] = np.imag(_chi2(mm, tables, ch, obs, sig)) / H_CS
    return out


@pytest.mark.parametrize("gravity", [0, 1])
def test_adjoint_matches_complex_step(gravity):
    tables, m, ch, obs, sig = _setup(gravity=gravity)
    g = oracle.chi2_and_grad(m, tables, ch, obs, sig)
    cs = _complex_step(m, tables, ch, obs, sig)
    assert np.isclose(g["chi2"], _chi2(m, tables, ch, obs, sig), rtol=1e-14)
    for k in ("dT", "dlog10_vmr"):
        err = np.max(np.abs(g[k] - cs[k])) / np.max(np.abs(cs[k]))
        assert err < 1e-11, (k, err)
    assert abs(g["dRp"] - cs["dRp"]) / abs(cs["dRp"]) < 1e-11


def test_adjoint_matches_central_differences():
    """FP64 central differences, relative step 1e-6, away from table nodes."""
    tables, m, ch, obs, sig = _setup(N=10)
    g = oracle.chi2_and_grad(m, tables, ch, obs, sig)
    f = lambda mm: _chi2(mm, tables, ch, obs, sig)
    for l in range(10):
        h = 1e-6 * max(abs(m["T"][l]), 1.0)
        mp, mn = dict(m), dict(m)
        mp["T"] = m["T"].copy(); mp["T"][l] += h
        mn["T"] = m["T"].copy(); mn["T"][l] -= h
        fd = (f(mp) - f(mn)) / (2 * h)
        assert abs(fd - g["dT"][l]) <= 1e-5 * np.max(np.abs(g["dT"])), (l, fd, g["dT"][l])
    h = 1e-6 * m["Rp"]
    mp, mn = dict(m), dict(m)
    mp["Rp"] += h
    mn["Rp"] -= h
    fd = (f(mp) - f(mn)) / (2 * h)
    assert abs(fd - g["dRp"]) / abs(g["dRp"]) < 1e-6


def test_adjoint_dot_product_identities():
    """Transpose identities of the linear steps: <dl k, t> = <k, dl^T t> for
    the triangular chord contraction, and the binning transpose."""
    rng = np.random.default_rng(4)
    z = np.concatenate([[0.0], np.cumsum(rng.uniform(3e4, 6e4, 15))])
    dl = F.chord_lengths(z, 7e7)
    k = rng.normal(size=(16, 9))
    t = rng.normal(size=(16, 9))
    assert np.isclose(np.sum((dl @ k) * t), np.sum(k * (dl.T @ t)), rtol=1e-13)
    wn = np.linspace(1000, 2000, 50)
    w = F.bin_weights(wn, np.array([1000.0, 1333.0]), np.array([1333.0, 2000.0]), 0, 50)
    D = rng.normal(size=50)
    c = rng.normal(size=2)
    omega = w / w.sum(axis=1)[:, None]
    assert np.isclose(np.dot(F.bin_spectrum(D, w), c), np.dot(D, omega.T @ c), rtol=1e-13)
