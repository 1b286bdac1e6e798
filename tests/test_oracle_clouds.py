"""Pins of the oracle's flat-opacity cloud deck (equation clouds, Forward
Models section) and of its gradient.  CPU only.

  * a zero cross-section, or a deck between two layer pressures that holds
    no layer, leaves the model bit-identical to the cloud-free one;
  * the paper's remark that deck bounds anywhere between the same two layer
    pressures give identical results (the deck is discretised on P);
  * a deck over the whole atmosphere equals the same opacity routed through
    the Rayleigh path: every species with a flat Rayleigh cross-section
    r = 1e4 sigma cm^2 gives kappa = 1e-4 rho r sum_s chi_s = sigma rho;
  * an opaque deck turns every ray that crosses it (each ray at or below the
    deck's top layer, whatever its bottom) into a full annulus, and leaves
    the other rays' terms as they were: D - D_clear = sum_{j <= top} A_j
    e^{-tau_j} / Rs^2 per point; a large finite cross-section reaches that
    limit;
  * the reverse-mode gradient with a finite and with an opaque deck against
    complex-step differentiation of the forward model.
"""

import dataclasses

import numpy as np
import pytest

import oracle
from oracle import forward as F
from synth.atmosphere import guillot_T, log_midpoint_pressures, log_uniform_channels
from synth.workloads import Channels, batch_from_models, make_config, with_cloud_decks

H_CS = 1e-30


def _model(N=40, n_wn=400, lo=20, hi=380):
    tables, batch, _ = make_config(2, n_wn=n_wn, n_lines=80)
    m = batch.model(0)
    m["T"] = guillot_T(log_midpoint_pressures(1e6, 1e-4, N), 25.0, 1300.0) + np.linspace(0, 40, N)
    m["wn_lo"], m["wn_hi"] = lo, hi
    clo, chi = log_uniform_channels(tables.wn[lo:hi], 9)
    return tables, m, Channels(clo, chi)


def _layer_P(m):
    return F.pressure_grid(m["p_bot"], m["p_top"], len(m["T"]))[1]


def _deck(m, sigma, p_top, p_bottom):
    d = dict(m)
    d.update(cloud_sigma=sigma, cloud_p_top=p_top, cloud_p_bottom=p_bottom)
    return d


def test_zero_sigma_and_empty_deck_change_nothing():
    tables, m, ch = _model()
    P = _layer_P(m)
    ref = F.forward_model(m, tables, ch)
    for d in (_deck(m, 0.0, 1e2, 1e4),
              # both bounds strictly between layers 10 and 11: no layer inside
              _deck(m, 1e-25, P[11] * 1.01, P[10] * 0.99)):
        out = F.forward_model(d, tables, ch)
        assert np.array_equal(out["depth"], ref["depth"])
        assert np.array_equal(out["binned"], ref["binned"])


def test_bounds_between_the_same_layers_give_identical_results():
    tables, m, ch = _model()
    P = _layer_P(m)
    # layers 12..25 (pressure falls with the layer index)
    a = F.forward_model(_deck(m, 3e-29, P[25] * 0.999, P[12] * 1.001), tables, ch)
    b = F.forward_model(_deck(m, 3e-29, P[26] * 1.001, P[11] * 0.999), tables, ch)
    c = F.forward_model(_deck(m, 3e-29, P[12] * 1.001, P[25] * 0.999), tables, ch)   # swapped order
    clear = F.forward_model(m, tables, ch)
    assert np.array_equal(a["depth"], b["depth"]) and np.array_equal(a["depth"], c["depth"])
    assert np.all(a["depth"] >= clear["depth"]) and np.any(a["depth"] > clear["depth"])


def test_full_deck_equals_flat_rayleigh_route():
    tables, m, ch = _model()
    sigma = 7e-30
    W = tables.n_wn
    bare = dataclasses.replace(tables, xsec=np.zeros_like(tables.xsec), cia=np.zeros((0,) + tables.cia.shape[1:]),
                               cia_pair=np.zeros((0, 2), np.int32), rayleigh=None)
    ray = dataclasses.replace(bare, rayleigh=np.full((tables.n_abs + 2, W), 1e4 * sigma))
    d = _deck(m, sigma, m["p_top"], m["p_bot"])
    cloud = F.forward_model(d, bare, ch)["depth"]
    route = F.forward_model(m, ray, ch)["depth"]
    assert np.max(np.abs(cloud - route) / route) < 1e-13
    # and the deck alone is wavenumber independent
    assert np.ptp(cloud) == 0.0


@pytest.mark.parametrize("deck_layers", [(0, 17), (9, 17), (17, 17), (30, 39)])
def test_opaque_deck_fills_every_crossing_ray(deck_layers):
    tables, m, ch = _model()
    P = _layer_P(m)
    kb, kt = deck_layers
    d = _deck(m, np.inf, P[kt] * 0.999, P[kb] * 1.001)
    out = F.forward_model(d, tables, ch, keep=True)
    clear = F.forward_model(m, tables, ch, keep=True)
    A, tau, Rs = clear["A"], clear["tau"], m["Rs"]
    # rays 0..kt cross layer kt (the top ray of a deck that includes the top
    # layer has no path, and keeps its clear term)
    top = kt if kt < len(A) - 1 else kt - 1
    expect = clear["depth"] + np.sum(A[:top + 1, None] * np.exp(-tau[:top + 1]), axis=0) / Rs ** 2
    assert np.max(np.abs(out["depth"] - expect) / expect) < 1e-14
    # the limit of a large finite cross-section
    big = F.forward_model(_deck(m, 1e-15, P[kt] * 0.999, P[kb] * 1.001), tables, ch)
    assert np.max(np.abs(big["depth"] - out["depth"]) / out["depth"]) < 1e-14


def test_opaque_deck_without_gas_is_a_raised_disc():
    """No other opacity: D = (Rp^2 + sum_{j <= top} A_j)/Rs^2 whatever the
    deck's bottom, flat in wavenumber."""
    tables, m, ch = _model()
    bare = dataclasses.replace(tables, xsec=np.zeros_like(tables.xsec), cia=np.zeros((0,) + tables.cia.shape[1:]),
                               cia_pair=np.zeros((0, 2), np.int32), rayleigh=None)
    P = _layer_P(m)
    for kb in (0, 5, 20):
        out = F.forward_model(_deck(m, np.inf, P[20] * 0.999, P[kb] * 1.001), bare, ch, keep=True)
        A = out["A"]
        expect = (m["Rp"] ** 2 + np.sum(A[:21])) / m["Rs"] ** 2
        assert np.all(np.abs(out["depth"] - expect) <= 1e-15 * expect)


def test_with_cloud_decks_kinds():
    T = guillot_T(log_midpoint_pressures(1e6, 1e-4, 30), 25.0, 1300.0)
    batch = batch_from_models([T] * 6, 1e6, 1e-4, np.full((6, 1), -4.0), 7e7, 7e8, 1.2e17, 0, 100)
    cb = with_cloud_decks(batch, 3)
    assert cb.B == 6
    assert list(cb.cloud_sigma[:3] == 0.0) == [True, False, False]
    assert np.isinf(cb.cloud_sigma[2]) and np.isfinite(cb.cloud_sigma[1])
    assert np.all(cb.cloud_p_top[[1, 2]] < cb.cloud_p_bottom[[1, 2]])
    assert cb.subset([1, 2]).model(1)["cloud_sigma"] == np.inf


def _complex_step_grad(m, tables, ch, obs, sig):
    def c2(mm):
        b = F.forward_model(mm, tables, ch)["binned"]
        r = (b - obs) / sig
        return np.sum(r * r)
    N = len(m["T"])
    dT = np.zeros(N)
    for i in range(N):
        mm = dict(m)
        v = np.array(m["T"], dtype=complex)
        v[i] += 1j * H_CS
        mm["T"] = v
        dT[i] = np.imag(c2(mm)) / H_CS
    dv = np.zeros(len(m["log10_vmr"]))
    for i in range(len(dv)):
        mm = dict(m)
        v = np.array(m["log10_vmr"], dtype=complex)
        v[i] += 1j * H_CS
        mm["log10_vmr"] = v
        dv[i] = np.imag(c2(mm)) / H_CS
    mm = dict(m)
    mm["Rp"] = m["Rp"] + 1j * H_CS
    return dT, dv, np.imag(c2(mm)) / H_CS


@pytest.mark.parametrize("sigma", [2e-29, np.inf])
def test_gradient_with_deck_matches_complex_step(sigma):
    tables, m, ch = _model(N=14, n_wn=260, lo=10, hi=250)
    P = _layer_P(m)
    d = _deck(m, sigma, P[9] * 0.999, P[3] * 1.001)
    base = F.forward_model(d, tables, ch)["binned"]
    obs = base * (1.0 + 2e-3 * np.sin(np.arange(len(base)) + 0.3))
    sig = np.full(len(base), 50e-6)
    g = oracle.chi2_and_grad(d, tables, ch, obs, sig)
    dT, dv, dR = _complex_step_grad(d, tables, ch, obs, sig)
    v = np.concatenate([g["dT"], g["dlog10_vmr"], [g["dRp"]]])
    r = np.concatenate([dT, dv, [dR]])
    assert np.linalg.norm(v - r) <= 1e-10 * np.linalg.norm(r)
    # the deck matters to the gradient
    g0 = oracle.chi2_and_grad(m, tables, ch, obs, sig)
    assert np.linalg.norm(g0["dT"] - g["dT"]) > 1e-3 * np.linalg.norm(g["dT"])
