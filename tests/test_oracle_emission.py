"""Pins of the FP64 emission oracle against what the mathematics and the
paper fix (not against the oracle itself).  CPU only."""

import math

import numpy as np
import pytest
from scipy import integrate, optimize, special

from oracle import emission as E
from oracle import forward as F
from synth.atmosphere import guillot_T, log_midpoint_pressures
from synth.constants import (AMU_KG, GM_JUP, HE_H2_RATIO, K_BOLTZMANN, MASSES_AMU, R_JUP,
                             R_SUN)
from synth.workloads import Tables, make_config, with_cloud_decks


def _tables(sigma_cm2, n_wn=5, cia=None):
    """One absorber of constant cross-section (cm^2) on a 5-point grid, no
    Rayleigh; optionally one CIA pair of constant cross-section (cm^5)."""
    wn = np.linspace(800.0, 9000.0, n_wn)
    T = np.linspace(100.0, 4000.0, 3)
    lp = np.linspace(-6.0, 8.0, 3)
    xs = np.full((1, 3, 3, n_wn), sigma_cm2)
    if cia is None:
        c, pair = np.zeros((0, 3, n_wn)), np.zeros((0, 2), np.int32)
    else:
        c, pair = np.full((1, 3, n_wn), cia), np.array([[1, 2]], np.int32)
    return Tables(wn, T, lp, xs, np.array([MASSES_AMU["H2O"]]), MASSES_AMU["H2"],
                  MASSES_AMU["He"], T.copy(), c, pair, None, ["X"])


def _model(T, gravity=0, vmr=-4.0, W=5):
    return dict(T=np.asarray(T, dtype=np.float64), p_bot=1e6, p_top=1e-4,
                log10_vmr=np.array([vmr]), Rp=R_JUP, Rs=R_SUN, GM=GM_JUP, wn_lo=0, wn_hi=W,
                he_h2=HE_H2_RATIO, k_B=K_BOLTZMANN, amu=AMU_KG, gravity=gravity)


def _guillot(N, T_irr=1400.0):
    return guillot_T(log_midpoint_pressures(1e6, 1e-4, N), GM_JUP / R_JUP ** 2, T_irr)


# --------------------------------------------------------------------------
# quadrature and Planck's law
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8])
def test_gauss_legendre_moments(n):
    """int_0^1 mu^k dmu = 1/(k+1) exactly for k <= 2n-1; for k = 2n the
    rule's error is the classical (n!)^4 / ((2n+1) ((2n)!)^2) on [0, 1]."""
    mu, w = E.gauss_legendre_mu(n)
    assert np.all((mu > 0) & (mu < 1)) and np.all(w > 0)
    for k in range(2 * n):
        assert abs(np.sum(w * mu ** k) - 1.0 / (k + 1)) < 1e-14, (n, k)
    err = 1.0 / (2 * n + 1) - np.sum(w * mu ** (2 * n))
    want = math.factorial(n) ** 4 / ((2 * n + 1) * math.factorial(2 * n) ** 2)
    assert abs(err / want - 1.0) < 1e-5, (n, err, want)


def test_planck_integral_and_peak():
    """int B dnu = sigma T^4 / pi with sigma = 2 pi^5 k^4 / (15 h^3 c^2); the
    peak of B per unit wavenumber is at h c nu / k T = 3 + W0(-3 e^-3);
    B -> 2 c k T nu^2 (Rayleigh-Jeans) for h c nu << k T."""
    h, c, k = E.H_PLANCK, E.C_LIGHT, K_BOLTZMANN
    for T in (300.0, 1500.0, 5800.0):
        scale = k * T / (h * c) / 100.0          # wavenumber (cm^-1) of x = 1
        f = lambda wn: E.planck(wn, T, k) * 100.0  # per cm^-1
        tot = sum(integrate.quad(f, a * scale, b * scale, epsabs=0, epsrel=1e-12, limit=400)[0]
                  for a, b in ((1e-9, 1.0), (1.0, 10.0), (10.0, 60.0), (60.0, 200.0)))
        sigma_sb = 2 * np.pi ** 5 * k ** 4 / (15 * h ** 3 * c ** 2)
        assert abs(tot / (sigma_sb * T ** 4 / np.pi) - 1.0) < 1e-9, T
        x_peak = 3.0 + special.lambertw(-3.0 * np.exp(-3.0)).real
        r = optimize.minimize_scalar(lambda x: -E.planck(x * scale, T, k), bounds=(1.0, 5.0),
                                     method="bounded", options={"xatol": 1e-12})
        assert abs(r.x - x_peak) < 1e-6, (T, r.x, x_peak)
        wn = 1e-7 * scale
        rj = 2.0 * c * k * T * (100.0 * wn) ** 2
        assert abs(E.planck(wn, T, k) / rj - 1.0) < 1e-6


# --------------------------------------------------------------------------
# the formal solution
# --------------------------------------------------------------------------
def test_isothermal_atmosphere_emits_planck_at_any_opacity():
    """Every term telescopes to B(T): F_p/F_s = B(T)/B(T*) (Rp/Rs)^2 for any
    opacity (with and without cloud decks) and any number of angles."""
    tables, batch, _ = make_config(2, n_wn=300, n_lines=60)
    m = batch.model(0)
    m["T"] = np.full(len(m["T"]), 1300.0)
    for deck in (None, (1e-28, 1e2, 1e4), (np.inf, 1e3, 1e6)):
        mm = dict(m)
        if deck:
            mm.update(cloud_sigma=deck[0], cloud_p_top=deck[1], cloud_p_bottom=deck[2])
        for n_mu in (1, 4):
            out = E.emission_model(mm, tables, n_mu=n_mu, T_star=5500.0)
            wn = tables.wn[m["wn_lo"]:m["wn_hi"]]
            want = E.planck(wn, 1300.0, K_BOLTZMANN) / E.planck(wn, 5500.0, K_BOLTZMANN) \
                * (R_JUP / R_SUN) ** 2
            assert np.allclose(out["fpfs"], want, rtol=1e-13, atol=0), (deck, n_mu)


def test_transparent_and_opaque_limits():
    """No opacity: the surface (the bottom layer's temperature, E3) shows
    through; an opaque atmosphere shows its top layer."""
    T = _guillot(60)
    wn = np.linspace(800.0, 9000.0, 5)
    ratio = lambda t: E.planck(wn, t, K_BOLTZMANN) / E.planck(wn, 6000.0, K_BOLTZMANN) \
        * (R_JUP / R_SUN) ** 2
    out = E.emission_model(_model(T), _tables(0.0), n_mu=3, T_star=6000.0)
    assert np.allclose(out["fpfs"], ratio(T[0]), rtol=1e-14, atol=0)
    out = E.emission_model(_model(T), _tables(1e10), n_mu=3, T_star=6000.0)
    assert np.allclose(out["fpfs"], ratio(T[-1]), rtol=1e-12, atol=0)


@pytest.mark.parametrize("mu", [0.07, 0.4, 1.0])
def test_linear_source_converges_to_closed_form(mu):
    """With B(t) = a + b t on a uniform optical-depth grid (B of each shell
    at its mid optical depth) the layer formula converges to the exact
    solution a + b mu (1 - e^{-tau_s/mu}) (surface at a + b tau_s), at second
    order (midpoint rule)."""
    a, b, tau_s = 2.0, 3.0, 8.0
    exact = a + b * mu * (1.0 - np.exp(-tau_s / mu))
    errs = []
    for N in (50, 100, 200, 400):
        t = tau_s * (1.0 - np.arange(N) / N)          # tau_l at the bottom of shell l
        t_up = np.append(t[1:], 0.0)
        B = a + b * 0.5 * (t + t_up)
        I = E.emergent_intensity(t[:, None], B[:, None], np.array([a + b * tau_s]), mu)[0]
        errs.append(abs(I - exact) / exact)
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.9 < o < 2.1 for o in orders), (errs, orders)


def test_vertical_optical_depth_converges_to_hydrostatic_column():
    """Constant g: the column density between two levels is Delta P / (mu g)
    whatever the temperatures (hydrostatic equilibrium), so the vertical
    optical depth of a constant cross-section from the top down to z = 0
    tends to chi sigma (P_0 - P_{N-1}) / (mu m g) as the layers get thinner."""
    sigma = 1e-24
    t = _tables(sigma)
    errs = []
    for N in (100, 200, 400, 800, 1600):
        m = _model(_guillot(N), gravity=1)
        out = E.emission_model(m, t, n_mu=1, keep=True)
        chi = 1e-4
        P = out["P"]
        g = GM_JUP / R_JUP ** 2
        col = chi * sigma * 1e-4 * (P[0] - P[-1]) / (out["mu"] * g)
        errs.append((out["tau"][0, 0] - col) / col)
    # the bottom shell holds the density of its lower edge and the altitude
    # step is explicit: a first-order bias with a second-order part that
    # fades under refinement (observed orders 1.7 -> 1.2)
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(e > 0 for e in errs), errs
    assert all(0.9 < o < 2.0 for o in orders), (errs, orders)
    assert all(orders[i] > orders[i + 1] for i in range(len(orders) - 1)), orders
    assert errs[-1] < 1.2e-4, errs


def test_opaque_deck_acts_as_a_surface():
    """An opaque deck whose top is layer l_d hides everything below it: the
    spectrum equals that of the layers above with the deck-top layer as the
    surface (shells l_d .. N-1 of the same atmosphere)."""
    tables, batch, _ = make_config(2, n_wn=300, n_lines=60)
    b = with_cloud_decks(batch, 1, kinds=("opaque",))
    m = b.model(0)
    out = E.emission_model(m, tables, n_mu=4, keep=True)
    _, P = F.pressure_grid(m["p_bot"], m["p_top"], len(m["T"]))
    ld = int(np.flatnonzero(P >= m["cloud_p_top"])[-1])     # the deck's top layer
    full = E.emission_model({k: v for k, v in m.items() if not k.startswith("cloud")}, tables,
                            n_mu=4, keep=True)
    # the gas optical depths above the deck, the deck-top shell as surface
    tau_up = full["tau"][ld + 1:]
    B = full["B_layer"]
    mus, ws = E.gauss_legendre_mu(4)
    flux = 0.0
    for mu, w in zip(mus, ws):
        Eu = np.exp(-np.vstack([tau_up, np.zeros((1, tau_up.shape[1]))]) / mu)
        flux = flux + 2 * w * mu * (B[ld] * Eu[0] + np.sum(B[ld + 1:] * (Eu[1:] - Eu[:-1]), axis=0))
    wn = tables.wn[m["wn_lo"]:m["wn_hi"]]
    want = flux / E.planck(wn, 5800.0, K_BOLTZMANN) * (m["Rp"] / m["Rs"]) ** 2
    assert np.allclose(out["fpfs"], want, rtol=1e-12, atol=0)
