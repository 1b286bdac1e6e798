"""Pins of the FP64 oracle against what the paper and the mathematics fix
(not against the oracle itself).  CPU only."""

import os

import mpmath
import numpy as np
import pytest
from scipy import integrate, special

import oracle
from oracle import forward as F
from synth.constants import (AMU_KG, GM_JUP, HE_H2_RATIO, K_BOLTZMANN, MASSES_AMU,
                             R_JUP, R_SUN)
from synth.workloads import Channels, Tables, make_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _const_tables(sigma_cm2, n_wn=3, nT=3, nP=3, mass=18.01528):
    wn = np.linspace(1000.0, 3000.0, n_wn)
    T = np.linspace(100.0, 4000.0, nT)
    lp = np.linspace(-6.0, 8.0, nP)
    xs = np.full((1, nT, nP, n_wn), sigma_cm2)
    return Tables(wn, T, lp, xs, np.array([mass]), MASSES_AMU["H2"], MASSES_AMU["He"],
                  T.copy(), np.zeros((0, nT, n_wn)), np.zeros((0, 2), np.int32), None, ["X"])


def _model(N=100, T=1500.0, vmr=-4.0, gravity=0, W=3, Rp=R_JUP):
    return dict(T=np.full(N, T), p_bot=1e6, p_top=1e-4, log10_vmr=np.array([vmr]),
                Rp=Rp, Rs=R_SUN, GM=GM_JUP, wn_lo=0, wn_hi=W, he_h2=HE_H2_RATIO,
                k_B=K_BOLTZMANN, amu=AMU_KG, gravity=gravity)


# --------------------------------------------------------------------------
# constants printed in the paper
# --------------------------------------------------------------------------
def test_constants_match_paper_tables():
    """Masses of the paper's mass table and its Jupiter radius
    (tests/golden/paper_constants.txt, with citations)."""
    vals = {}
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    for k in ("H", "He", "H2", "H2O", "CH4"):
        assert MASSES_AMU[k] == vals[k]
    assert R_JUP == vals["R_Jup"]
    assert HE_H2_RATIO == vals["He_H2_ratio"]


# --------------------------------------------------------------------------
# a1: pressure grid and chemistry
# --------------------------------------------------------------------------
def test_pressure_grid_log_spaced_geometric_centres():
    p, P = F.pressure_grid(1e6, 1e-4, 100)
    assert p.shape == (101,) and P.shape == (100,)
    assert np.isclose(p[0], 1e6, rtol=1e-15) and np.isclose(p[-1], 1e-4, rtol=1e-14)
    r = np.log(p[1:] / p[:-1])
    assert np.allclose(r, r[0], rtol=1e-12, atol=0)
    assert np.allclose(P, np.sqrt(p[:-1] * p[1:]), rtol=1e-15)


def test_chemistry_fill_and_mean_molecular_weight():
    """Pure H2/He fill at He/H2 = 0.17 gives mu = (m_H2 + 0.17 m_He)/1.17; one
    absorber takes its share of the volume and the fill keeps the ratio."""
    m = np.array([MASSES_AMU["H2O"]])
    chi, h2, he, mu, ok = F.chemistry(np.array([-30.0]), 0.17, m, MASSES_AMU["H2"],
                                      MASSES_AMU["He"], 1.0)
    assert ok
    assert np.isclose(mu, (MASSES_AMU["H2"] + 0.17 * MASSES_AMU["He"]) / 1.17, rtol=1e-14)
    assert np.isclose(mu, 2.3045, atol=2e-4)
    chi, h2, he, mu, ok = F.chemistry(np.array([np.log10(0.2)]), 0.17, m, MASSES_AMU["H2"],
                                      MASSES_AMU["He"], 1.0)
    assert np.isclose(chi[0] + h2 + he, 1.0, rtol=1e-15)
    assert np.isclose(he / h2, 0.17, rtol=1e-15)
    assert np.isclose(mu, 0.2 * m[0] + 0.8 * (MASSES_AMU["H2"] + 0.17 * MASSES_AMU["He"]) / 1.17,
                      rtol=1e-14)
    assert not F.chemistry(np.array([0.0]), 0.17, m, 2.0, 4.0, 1.0)[4]


# --------------------------------------------------------------------------
# a2: altitude
# --------------------------------------------------------------------------
def test_altitude_constant_gravity_isothermal_closed_form():
    """Isothermal, constant mu and g: z_l = H ln(P_0/P_l) exactly."""
    N, T = 100, 1500.0
    _, P = F.pressure_grid(1e6, 1e-4, N)
    mu = 2.3 * AMU_KG
    z = F.altitude(np.full(N, T), P, mu, R_JUP, GM_JUP, K_BOLTZMANN, gravity=1)
    H = K_BOLTZMANN * T * R_JUP ** 2 / (mu * GM_JUP)
    exact = H * np.log(P[0] / P)
    assert z[0] == 0.0
    assert np.max(np.abs(z[1:] - exact[1:]) / exact[1:]) < 1e-13


def test_altitude_variable_gravity_first_order_convergence():
    """With g = GM/(Rp+z)^2 the exact hydrostatic solution is
    1/Rp - 1/(Rp+z) = k_B T ln(P_0/P)/(mu GM); the explicit recursion
    converges to it at first order in the layer spacing."""
    T, mu = 1500.0, 2.3 * AMU_KG

    def top_err(N):
        _, P = F.pressure_grid(1e6, 1e-4, N)
        z = F.altitude(np.full(N, T), P, mu, R_JUP, GM_JUP, K_BOLTZMANN, gravity=0)
        c = K_BOLTZMANN * T * np.log(P[0] / P[-1]) / (mu * GM_JUP)
        z_ex = 1.0 / (1.0 / R_JUP - c) - R_JUP
        return abs(z[-1] - z_ex) / z_ex

    e = [top_err(N) for N in (100, 200, 400, 800)]
    orders = [np.log2(e[i] / e[i + 1]) for i in range(3)]
    assert all(0.9 < o < 1.1 for o in orders), orders


def test_altitude_non_isothermal_uses_lower_layer_scale_height():
    """Constant g and mu, T linear in x = ln(P_0/P): the exact hydrostatic
    altitude is (k_B/(mu g)) int_0^x T dx'.  A step that takes the scale
    height of the lower layer (the altitude equation's H_{l-1}) is the left
    Riemann sum of that integral, whose error for a linear integrand is
    exactly -(k_B/(mu g)) alpha x_l dx / 2: the upper layer's H gives the
    opposite sign and a centred H gives none."""
    N, mu = 120, 2.3 * AMU_KG
    _, P = F.pressure_grid(1e6, 1e-4, N)
    x = np.log(P[0] / P)
    dx = x[1] - x[0]
    for T0, alpha in ((800.0, 60.0), (2600.0, -55.0)):
        T = T0 + alpha * x
        z = F.altitude(T, P, mu, R_JUP, GM_JUP, K_BOLTZMANN, gravity=1)
        c = K_BOLTZMANN * R_JUP ** 2 / (mu * GM_JUP)
        exact = c * (T0 * x + 0.5 * alpha * x ** 2)
        err = z - exact
        want = -0.5 * c * alpha * x * dx
        assert np.allclose(err[1:], want[1:], rtol=1e-7, atol=0), (T0, alpha)
        assert np.all(np.sign(err[1:]) == -np.sign(alpha))


# --------------------------------------------------------------------------
# a3: geometry
# --------------------------------------------------------------------------
def _random_z(rng, N, H=2e5):
    return np.concatenate([[0.0], np.cumsum(rng.uniform(0.3, 1.7, N - 1) * 0.23 * H)])


def test_chords_match_50_digit_evaluation():
    """Each chord segment evaluated from its definition
    2[sqrt(r_{k+1}^2 - b^2) - sqrt(max(r_k, b)^2 - b^2)] in 50-digit
    arithmetic."""
    mpmath.mp.dps = 50
    rng = np.random.default_rng(7)
    worst = 0.0
    for N in (3, 4, 5, 6):
        z = _random_z(rng, N)
        dl = F.chord_lengths(z, R_JUP)
        zm = [mpmath.mpf(float(v)) for v in z]
        Rp = mpmath.mpf(R_JUP)
        h = [mpmath.mpf(0)] + [(zm[k - 1] + zm[k]) / 2 for k in range(1, N)] + [zm[N - 1]]
        for j in range(N):
            b = Rp + zm[j]
            for k in range(N):
                if k < j:
                    assert dl[j, k] == 0.0
                    continue
                r0, r1 = Rp + h[k], Rp + h[k + 1]
                ref = 2 * (mpmath.sqrt(r1 ** 2 - b ** 2) - mpmath.sqrt(max(r0, b) ** 2 - b ** 2))
                if ref == 0:
                    assert dl[j, k] == 0.0
                else:
                    worst = max(worst, float(abs((dl[j, k] - ref) / ref)))
    assert worst < 1e-13, worst


def test_chord_sum_is_full_chord_and_single_shell():
    rng = np.random.default_rng(3)
    for N in (2, 5, 40):
        z = _random_z(rng, N)
        dl = F.chord_lengths(z, R_JUP)
        rN = R_JUP + z[-1]
        b = R_JUP + z
        full = 2.0 * np.sqrt((rN - b) * (rN + b))
        assert np.allclose(dl.sum(axis=1), full, rtol=1e-12, atol=1e-9)


def test_optical_depth_matches_ray_quadrature():
    """Fine-step quadrature of int kappa(r(s)) ds along each ray through
    shells of random opacity, independent of the chord formula."""
    rng = np.random.default_rng(11)
    N = 5
    z = _random_z(rng, N)
    kappa = rng.uniform(0.1, 2.0, N) * 1e-6
    dl = F.chord_lengths(z, R_JUP)
    tau = F.optical_depth(dl, kappa[:, None])[:, 0]
    h = F.shell_boundaries(z)
    rN = R_JUP + h[-1]
    for j in range(N - 1):
        b = R_JUP + z[j]
        smax = np.sqrt(rN ** 2 - b ** 2)
        n = 2_000_000
        s = (np.arange(n) + 0.5) * (smax / n)
        r = np.sqrt(b * b + s * s)
        shell = np.clip(np.searchsorted(R_JUP + h, r, side="right") - 1, 0, N - 1)
        q = 2.0 * np.sum(kappa[shell]) * (smax / n)
        assert abs(q - tau[j]) / tau[j] < 2e-6, (j, q, tau[j])


def test_annulus_weights_trapezoid():
    rng = np.random.default_rng(5)
    z = _random_z(rng, 30)
    A = F.annulus_weights(z, R_JUP)
    # exact for the linear integrand 2 (Rp + z) over [0, z_top]
    assert np.isclose(A.sum(), (R_JUP + z[-1]) ** 2 - R_JUP ** 2, rtol=1e-13)


# --------------------------------------------------------------------------
# a4: interpolation
# --------------------------------------------------------------------------
def _bilinear_table(nT=6, nP=5, W=4, seed=0):
    rng = np.random.default_rng(seed)
    T = np.sort(rng.uniform(200, 3000, nT))
    lp = np.sort(rng.uniform(-4, 6, nP))
    a, b, c, d = rng.uniform(1, 2, (4, W))
    tab = (a[None, None, :] + b[None, None, :] * T[:, None, None] / 1000
           + c[None, None, :] * lp[None, :, None]
           + d[None, None, :] * (T[:, None, None] / 1000) * lp[None, :, None])
    f = lambda t, x: a + b * t / 1000 + c * x + d * (t / 1000) * x
    return T, lp, tab, f


def test_interpolation_exact_on_bilinear_tables_and_nodes():
    T, lp, tab, f = _bilinear_table()
    rng = np.random.default_rng(1)
    for _ in range(50):
        t = rng.uniform(T[0], T[-1])
        x = rng.uniform(lp[0], lp[-1])
        v = F.interp_xsec(tab, T, lp, t, x)
        assert np.allclose(v, f(t, x), rtol=1e-13)
    for i in range(len(T)):
        for j in range(len(lp)):
            assert np.allclose(F.interp_xsec(tab, T, lp, T[i], lp[j]), tab[i, j], rtol=1e-15)


def test_interpolation_linear_in_P_flag():
    """The paper's literal form (linear in P) reproduces tables linear in P."""
    T = np.array([500.0, 1500.0])
    lp = np.array([0.0, 1.0, 2.0])
    P = 10.0 ** lp
    tab = (3.0 + 2e-3 * T[:, None, None] + 0.5 * P[None, :, None]) * np.ones((1, 1, 2))
    v = F.interp_xsec(tab, T, lp, 900.0, np.log10(37.0), p_interp="linear")
    assert np.allclose(v, 3.0 + 2e-3 * 900.0 + 0.5 * 37.0, rtol=1e-14)
    v_log = F.interp_xsec(tab, T, lp, 900.0, np.log10(37.0), p_interp="log")
    assert not np.allclose(v_log, v, rtol=1e-3)


def test_interpolation_clamp_rules():
    """Opacities section: out-of-range T/P fix to the grid edge; both below
    -> 0; both above -> sigma(Tmax, Pmax)."""
    T, lp, tab, f = _bilinear_table()
    lo_T, hi_T, lo_x, hi_x = T[0] - 50, T[-1] + 50, lp[0] - 1, lp[-1] + 1
    xm = 0.5 * (lp[1] + lp[2])
    Tm = 0.5 * (T[1] + T[2])
    assert np.allclose(F.interp_xsec(tab, T, lp, lo_T, xm), f(T[0], xm), rtol=1e-13)
    assert np.allclose(F.interp_xsec(tab, T, lp, hi_T, xm), f(T[-1], xm), rtol=1e-13)
    assert np.allclose(F.interp_xsec(tab, T, lp, Tm, lo_x), f(Tm, lp[0]), rtol=1e-13)
    assert np.allclose(F.interp_xsec(tab, T, lp, Tm, hi_x), f(Tm, lp[-1]), rtol=1e-13)
    assert np.all(F.interp_xsec(tab, T, lp, lo_T, lo_x) == 0.0)
    assert np.allclose(F.interp_xsec(tab, T, lp, hi_T, hi_x), tab[-1, -1], rtol=1e-15)
    assert np.allclose(F.interp_xsec(tab, T, lp, lo_T, hi_x), tab[0, -1], rtol=1e-15)
    assert np.allclose(F.interp_xsec(tab, T, lp, hi_T, lo_x), tab[-1, 0], rtol=1e-15)
    # alternative reading: P below the grid alone gives zero
    assert np.all(F.interp_xsec(tab, T, lp, Tm, lo_x, zero_rule="p_only") == 0.0)


def test_cia_interpolation_linear_in_T():
    T = np.array([300.0, 800.0, 1900.0, 3000.0])
    tab = (1.0 + 0.002 * T)[:, None] * np.array([1.0, 2.0, 3.0])[None, :]
    for t in (300.0, 555.0, 1900.0, 2999.0):
        assert np.allclose(F.interp_cia(tab, T, t), (1.0 + 0.002 * t) * np.array([1, 2, 3.0]),
                           rtol=1e-14)
    assert np.allclose(F.interp_cia(tab, T, 100.0), tab[0], rtol=1e-15)
    assert np.allclose(F.interp_cia(tab, T, 5000.0), tab[-1], rtol=1e-15)


# --------------------------------------------------------------------------
# a5-a6: whole model closed forms
# --------------------------------------------------------------------------
def test_zero_opacity_gives_geometric_depth():
    t = _const_tables(0.0)
    out = F.forward_model(_model(), t)
    assert np.all(out["depth"] == R_JUP ** 2 / R_SUN ** 2)
    assert np.isclose(out["depth"][0], 0.0100983, rtol=1e-5)


def test_zero_opacity_gradient():
    """dD/dRp = 2 Rp/Rs^2 and dD/dT = 0 with no opacity."""
    t = _const_tables(0.0)
    m = _model(N=12)
    ch = Channels(np.array([900.0]), np.array([3100.0]))
    D = (R_JUP / R_SUN) ** 2
    obs, sig = np.array([D - 1e-4]), np.array([1e-4])
    g = oracle.chi2_and_grad(m, t, ch, obs, sig)
    Dbar = 2 * (D - obs[0]) / sig[0] ** 2
    assert np.isclose(g["dRp"], Dbar * 2 * R_JUP / R_SUN ** 2, rtol=1e-13)
    assert np.all(g["dT"] == 0.0)


def test_opaque_limit_closed_form():
    """kappa -> infinity: every ray below the top is dark and the depth is the
    trapezoid sum of 2(Rp+z) minus the top node, which has zero chord:
    D Rs^2 - Rp^2 = (Rp+z_top)^2 - Rp^2 - (Rp+z_top)(z_top - z_{N-2})."""
    t = _const_tables(1e20)
    out = F.forward_model(_model(), t, keep=True)
    z = out["z"]
    lhs = out["depth"] * R_SUN ** 2 - R_JUP ** 2
    zt = z[-1]
    rhs = (R_JUP + zt) ** 2 - R_JUP ** 2 - (R_JUP + zt) * (zt - z[-2])
    assert np.allclose(lhs, rhs, rtol=1e-10)


def _continuous_depth(N, sigma_m2, chi, T, mu_kg):
    """Continuous isothermal constant-g atmosphere with the discrete model's
    bottom density and top altitude: tau(b) = 2 s n0 b K1(b/H) e^{(Rp-b)/H}
    (from int e^{-sqrt(b^2+s^2)/H} ds = b K1(b/H)), a = 2 int (Rp+z)(1-e^-tau)."""
    _, P = F.pressure_grid(1e6, 1e-4, N)
    H = K_BOLTZMANN * T * R_JUP ** 2 / (mu_kg * GM_JUP)
    n0 = P[0] / (K_BOLTZMANN * T)
    ztop = H * np.log(P[0] / P[-1])

    def tau(z):
        b = R_JUP + z
        return 2.0 * sigma_m2 * chi * n0 * b * special.k1e(b / H) * np.exp(-z / H)

    f = lambda z: 2.0 * (R_JUP + z) * (-np.expm1(-tau(z)))
    a, _ = integrate.quad(f, 0.0, ztop, epsabs=0, epsrel=1e-13, limit=500)
    return (R_JUP ** 2 + a) / R_SUN ** 2, (R_JUP ** 2) / R_SUN ** 2


def test_isothermal_constant_sigma_converges_to_continuous_model():
    T, vmr = 1500.0, -4.0
    sigma_cm2 = 1e-22
    t = _const_tables(sigma_cm2)
    mu = F.chemistry(np.array([vmr]), HE_H2_RATIO, t.abs_mass, t.h2_mass, t.he_mass, AMU_KG)[3]
    errs = []
    for N in (100, 200, 400, 800):
        D = F.forward_model(_model(N=N, T=T, vmr=vmr, gravity=1), t)["depth"][0]
        Dc, D0 = _continuous_depth(N, sigma_cm2 * 1e-4, 10.0 ** vmr, T, mu)
        errs.append(abs(D - Dc) / (Dc - D0))      # error of the atmospheric part
    # observed order ~1.55 (first shell and top-node bias), stable under
    # refinement; at 100 layers the atmospheric part is within ~1.5e-3
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert errs[0] < 3e-3
    assert all(1.3 < o < 2.0 for o in orders), (errs, orders)
    assert max(orders) - min(orders) < 0.1, orders


def _cia_tables(sigma_cm5, pair, n_wn=3, nT=3):
    """One absorber with zero cross-section and one CIA pair (species ids
    ``pair``) whose cross-section sigma_cm5 is the same at every T and
    wavenumber."""
    wn = np.linspace(1000.0, 3000.0, n_wn)
    T = np.linspace(100.0, 4000.0, nT)
    lp = np.linspace(-6.0, 8.0, 3)
    return Tables(wn, T, lp, np.zeros((1, nT, 3, n_wn)), np.array([MASSES_AMU["H2O"]]),
                  MASSES_AMU["H2"], MASSES_AMU["He"], T.copy(),
                  np.full((1, nT, n_wn), sigma_cm5), np.array([pair], np.int32), None, ["X"])


def _continuous_cia_depth(N, kappa0, T, mu_kg):
    """Continuous isothermal constant-g atmosphere whose opacity is
    kappa0 e^{-2z/H}, i.e. rho^2 with rho = rho_0 e^{-z/H} (equation
    cia_opt_dpth): the chord integral is the absorption one with H/2,
    tau(b) = 2 kappa0 b K1(2b/H) e^{2Rp/H}."""
    _, P = F.pressure_grid(1e6, 1e-4, N)
    H = K_BOLTZMANN * T * R_JUP ** 2 / (mu_kg * GM_JUP)
    ztop = H * np.log(P[0] / P[-1])
    Hc = 0.5 * H

    def tau(z):
        b = R_JUP + z
        return 2.0 * kappa0 * b * special.k1e(b / Hc) * np.exp(-z / Hc)

    f = lambda z: 2.0 * (R_JUP + z) * (-np.expm1(-tau(z)))
    a, _ = integrate.quad(f, 0.0, ztop, epsabs=0, epsrel=1e-13, limit=500)
    return (R_JUP ** 2 + a) / R_SUN ** 2, (R_JUP ** 2) / R_SUN ** 2


@pytest.mark.parametrize("pair,vmr", [((1, 1), -30.0), ((1, 2), -30.0), ((0, 1), -1.0)])
def test_isothermal_constant_cia_converges_to_continuous_model(pair, vmr):
    """Equation cia_opt_dpth with one pair of constant cross-section
    sigma_c (cm^5): kappa = 1e-10 sigma_c chi_a chi_b rho^2 (m^-1).  With the
    pair weight of the species ids H2-H2, H2-He or absorber-H2 (a 10 %
    absorber) the discrete model converges to the continuous one, whose
    rho^2 profile has half the scale height.  A wrong unit factor, power of
    rho or pair index moves the depth by percents, far outside the bound."""
    T, sigma_c = 1500.0, 1e-43
    t = _cia_tables(sigma_c, pair)
    chi, h2, he, mu, _ = F.chemistry(np.array([vmr]), HE_H2_RATIO, t.abs_mass, t.h2_mass,
                                     t.he_mass, AMU_KG)
    species = [chi[0], h2, he]
    w = species[pair[0]] * species[pair[1]]
    errs = []
    for N in (100, 200, 400, 800):
        n0 = F.pressure_grid(1e6, 1e-4, N)[1][0] / (K_BOLTZMANN * T)   # rho at z = 0
        kappa0 = 1e-10 * sigma_c * w * n0 ** 2
        m = _model(N=N, T=T, vmr=vmr, gravity=1)
        D = F.forward_model(m, t)["depth"][0]
        Dc, D0 = _continuous_cia_depth(N, kappa0, T, mu)
        errs.append(abs(D - Dc) / (Dc - D0))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert errs[0] < 3.5e-3, errs
    assert all(1.3 < o < 2.0 for o in orders), (errs, orders)
    assert max(orders) - min(orders) < 0.1, orders


# --------------------------------------------------------------------------
# a7: binning
# --------------------------------------------------------------------------
def test_binning_identities():
    wn = np.sort(np.random.default_rng(2).uniform(1000, 2000, 40))
    lo, hi = F.native_bin_edges(wn)
    D = np.random.default_rng(3).uniform(0.01, 0.02, 40)
    # channels equal to the native bins: identity
    w = F.bin_weights(wn, lo, hi, 0, 40)
    assert np.allclose(w, np.eye(40), atol=1e-15)
    assert np.allclose(F.bin_spectrum(D, w), D, rtol=1e-15)
    # constant spectrum stays constant; linear in D
    chl = np.array([lo[0], wn[10], wn[25]])
    chh = np.array([wn[10], wn[25], hi[-1]])
    w = F.bin_weights(wn, chl, chh, 0, 40)
    assert np.allclose(F.bin_spectrum(np.full(40, 0.7), w), 0.7, rtol=1e-15)
    assert np.allclose(F.bin_spectrum(2 * D + 3 * D[::-1], w),
                       2 * F.bin_spectrum(D, w) + 3 * F.bin_spectrum(D[::-1], w), rtol=1e-14)
    # fully inside a channel: w = 1 (Binning subsection); interior partition of unity
    assert np.all(w[1, 11:25] == 1.0)
    assert np.allclose(w.sum(axis=0), 1.0, rtol=1e-14)
    # a channel outside the window is NaN
    w = F.bin_weights(wn, np.array([2500.0]), np.array([2600.0]), 0, 40)
    assert np.isnan(F.bin_spectrum(D, w)[0])


# --------------------------------------------------------------------------
# monotonicity in abundance (geometry frozen)
# --------------------------------------------------------------------------
def test_depth_monotone_in_abundance_with_geometry_frozen():
    tables, batch, _ = make_config(2, n_wn=400, n_lines=60)
    m = batch.model(0)
    base = F.forward_model(m, tables, keep=True)
    for i in range(tables.n_abs):
        chi = base["chi"].copy()
        chi[i] *= 1.5
        k = F.opacity(m["T"], base["P"], chi, base["chi_h2"], base["chi_he"], tables,
                      m["k_B"], 0, tables.n_wn)
        D = F.transit_depth(F.optical_depth(base["dl"], k), base["A"], m["Rp"], m["Rs"])
        assert np.all(D >= base["depth"])
        assert np.all(D > base["depth"])          # every absorber has a 1e-27 floor


def test_paper_magnitude_sanity():
    """Order of magnitude only (parity unpinned): a 1 R_Jup planet with an
    H2/He atmosphere and a trace absorber around a 1 R_Sun star has a depth
    of ~0.0101 plus a few 1e-4 (the paper's library example prints ~0.0106)."""
    tables, batch, _ = make_config(1)
    D = F.forward_model(batch.model(0), tables)["depth"]
    assert 0.0100983 < D.min() and D.max() < 0.0125


# --------------------------------------------------------------------------
# exponential temperature interpolation (reading A25)
# --------------------------------------------------------------------------
def _exp_table(nT=7, nP=5, W=6, seed=4):
    """Tables of the form a(P, w) e^{-b(P, w)/T} at the grid temperatures."""
    rng = np.random.default_rng(seed)
    T = np.sort(rng.uniform(250, 3200, nT))
    lp = np.sort(rng.uniform(-4, 6, nP))
    a = 10.0 ** rng.uniform(-24, -20, (nP, W))
    b = rng.uniform(200.0, 6000.0, (nP, W))
    tab = a[None] * np.exp(-b[None] / T[:, None, None])
    return T, lp, tab, a, b


def test_exp_interpolation_exact_on_exponential_tables():
    """The scheme reproduces a e^{-b/T} exactly between the nodes along T;
    along log10 P it is linear (checked at the P nodes and by linearity)."""
    T, lp, tab, a, b = _exp_table()
    rng = np.random.default_rng(8)
    for _ in range(40):
        t = rng.uniform(T[0], T[-1])
        j = int(rng.integers(0, len(lp)))
        v = F.interp_xsec(tab, T, lp, t, lp[j], t_interp="exp")
        assert np.allclose(v, a[j] * np.exp(-b[j] / t), rtol=1e-12, atol=0)
        x = rng.uniform(lp[0], lp[-1])
        i = int(np.searchsorted(lp, x, side="right")) - 1
        w = (x - lp[i]) / (lp[i + 1] - lp[i])
        want = (1 - w) * a[i] * np.exp(-b[i] / t) + w * a[i + 1] * np.exp(-b[i + 1] / t)
        assert np.allclose(F.interp_xsec(tab, T, lp, t, x, t_interp="exp"), want, rtol=1e-12, atol=0)
    # the linear scheme is not exact on these tables (the two differ between nodes)
    t = 0.5 * (T[2] + T[3])
    assert not np.allclose(F.interp_xsec(tab, T, lp, t, lp[1]), a[1] * np.exp(-b[1] / t), rtol=1e-3,
                           atol=0)


def test_exp_interpolation_nodes_clamps_and_fallback():
    """Node values are returned at the nodes; out-of-range T and P follow the
    clamp rules; where a node value is not positive the linear scheme is
    used (and reproduces linear data there)."""
    T, lp, tab, a, b = _exp_table()
    for i in range(len(T)):
        for j in range(len(lp)):
            # a e^{-b/T} at a node cancels e^{b/T1} e^{-b/T1}: rounding
            # grows with b/T (here up to ~100)
            assert np.allclose(F.interp_xsec(tab, T, lp, T[i], lp[j], t_interp="exp"), tab[i, j],
                               rtol=1e-11, atol=0)
    xm = 0.5 * (lp[1] + lp[2])
    assert np.allclose(F.interp_xsec(tab, T, lp, T[0] - 40, xm, t_interp="exp"),
                       F.interp_xsec(tab, T, lp, T[0], xm, t_interp="exp"), rtol=1e-14, atol=0)
    assert np.allclose(F.interp_xsec(tab, T, lp, T[-1] + 40, xm, t_interp="exp"),
                       F.interp_xsec(tab, T, lp, T[-1], xm, t_interp="exp"), rtol=1e-14, atol=0)
    assert np.all(F.interp_xsec(tab, T, lp, T[0] - 40, lp[0] - 1, t_interp="exp") == 0.0)
    # zeros at one node of a column: that column is linear in T
    lin_T, lin_lp, lin_tab, f = _bilinear_table(nT=len(T), nP=len(lp), W=6)
    mixed = tab.copy()
    mixed[:, :, 2] = lin_tab[:, :, 2]
    mixed[3, :, 2] = 0.0
    t = 0.3 * T[2] + 0.7 * T[3]
    v = F.interp_xsec(mixed, T, lp, t, lp[1], t_interp="exp")
    s1, s2 = mixed[2, 1, 2], mixed[3, 1, 2]
    assert np.isclose(v[2], s1 + (s2 - s1) * (t - T[2]) / (T[3] - T[2]), rtol=1e-14, atol=0)
    assert np.allclose(v[[0, 1, 3, 4, 5]], (a[1] * np.exp(-b[1] / t))[[0, 1, 3, 4, 5]], rtol=1e-12,
                       atol=0)


def test_exp_interpolation_model_equals_linear_at_node_temperatures():
    """An isothermal model at a grid temperature gives the same spectrum in
    both schemes (each layer interpolates at a node), and a model between
    nodes does not."""
    tables, batch, _ = make_config(2, n_wn=300, n_lines=60)
    m = batch.model(0)
    m["T"] = np.full(len(m["T"]), tables.T_grid[7])
    a = F.forward_model(m, tables)["depth"]
    bq = F.forward_model(dict(m, t_interp="exp"), tables)["depth"]
    assert np.allclose(a, bq, rtol=1e-13, atol=0)
    m["T"] = np.full(len(m["T"]), 0.5 * (tables.T_grid[7] + tables.T_grid[8]))
    a = F.forward_model(m, tables)["depth"]
    bq = F.forward_model(dict(m, t_interp="exp"), tables)["depth"]
    assert not np.allclose(a, bq, rtol=1e-9, atol=0)
