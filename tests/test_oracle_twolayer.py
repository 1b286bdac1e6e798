"""Pins of the oracle's two-layer mixing profiles (Chemistry subsection;
reading A26: surface value at and below a switch pressure, top value above,
per-layer fill gases and mean molecular weight): reductions to constant
profiles, the hydrostatic altitude with a mean molecular weight that steps
(closed form), and convergence of a two-layer absorber's transit depth to
the continuous model with the step, by quadrature."""

import numpy as np
from scipy import integrate, special

import oracle
from oracle import forward as F
from synth.constants import (AMU_KG, GM_JUP, HE_H2_RATIO, K_BOLTZMANN, MASSES_AMU, R_JUP,
                             R_SUN)
from synth.workloads import make_config
from test_oracle_pins import _const_tables, _model


def test_two_layer_reduces_to_constant_profiles():
    """Equal surface and top values give the constant profile; a switch
    pressure above every layer's centre gives the top values everywhere,
    one below every layer the surface values."""
    tables, batch, ch = make_config(2, n_wn=400, n_lines=40)
    m = batch.model(0)
    ref = F.forward_model(m, tables, ch)["binned"]
    va = np.asarray(m["log10_vmr"], dtype=np.float64)
    same = F.forward_model(dict(m, log10_vmr_top=va, vmr_switch=np.full(len(va), 50.0)), tables, ch)
    assert np.allclose(same["binned"], ref, rtol=1e-14, atol=0)
    top = va - 1.5
    all_top = F.forward_model(dict(m, log10_vmr_top=top, vmr_switch=np.full(len(va), 2e6)), tables, ch)
    ref_top = F.forward_model(dict(m, log10_vmr=top), tables, ch)
    assert np.allclose(all_top["binned"], ref_top["binned"], rtol=1e-14, atol=0)
    all_surf = F.forward_model(dict(m, log10_vmr_top=top, vmr_switch=np.full(len(va), 1e-5)), tables, ch)
    assert np.allclose(all_surf["binned"], ref, rtol=1e-14, atol=0)
    # a real step differs from both (not necessarily between them: the mean
    # molecular weight, and so the scale height, changes with the step)
    mid = F.forward_model(dict(m, log10_vmr_top=top, vmr_switch=np.full(len(va), 1e2)), tables, ch)
    assert np.max(np.abs(mid["binned"] / ref - 1)) > 1e-5
    assert np.max(np.abs(mid["binned"] / ref_top["binned"] - 1)) > 1e-5


def test_two_layer_altitude_closed_form():
    """Isothermal, constant g, a heavy absorber (44 amu) at 20 % below the
    switch and 1e-6 above: each altitude step uses the lower layer's mean
    molecular weight, so z = H_s ln(P_0/P_l) up to the first layer above the
    switch and continues with H_t above (H = k_B T Rp^2 / (mu GM)); the mean
    molecular weights here are the mixtures' own (absorber plus H2/He in
    the ratio r)."""
    T, N, m_a = 1200.0, 60, 44.0095
    t = _const_tables(1e-25, mass=m_a)
    m = _model(N=N, T=T, vmr=np.log10(0.2), gravity=1)
    p_sw = 30.0
    m.update(log10_vmr_top=np.array([-6.0]), vmr_switch=np.array([p_sw]))
    out = F.forward_model(m, t, keep=True)
    _, P = F.pressure_grid(1e6, 1e-4, N)
    f_h2, f_he = 1.0 / (1.0 + HE_H2_RATIO), HE_H2_RATIO / (1.0 + HE_H2_RATIO)
    fill = f_h2 * MASSES_AMU["H2"] + f_he * MASSES_AMU["He"]
    mu_s = (0.2 * m_a + 0.8 * fill) * AMU_KG
    mu_t = (1e-6 * m_a + (1 - 1e-6) * fill) * AMU_KG
    H_s = K_BOLTZMANN * T * R_JUP ** 2 / (mu_s * GM_JUP)
    H_t = K_BOLTZMANN * T * R_JUP ** 2 / (mu_t * GM_JUP)
    ls = int(np.argmax(P < p_sw))          # first layer above the switch
    assert 0 < ls < N - 1
    z = np.where(np.arange(N) <= ls, H_s * np.log(P[0] / P),
                 H_s * np.log(P[0] / P[ls]) + H_t * np.log(P[ls] / P))
    assert np.allclose(out["z"], z, rtol=1e-12, atol=1e-6)
    assert np.allclose(out["mu"][:ls], mu_s, rtol=1e-14) and np.allclose(out["mu"][ls:], mu_t, rtol=1e-14)


def _continuous_step_depth(N, k_s, k_t, Hc, T, mu_kg, p_sw):
    """Continuous isothermal constant-g atmosphere (rho = rho_0 e^{-z/H},
    z = 0 at the bottom layer's centre pressure P_0, the top at the top
    layer's) whose opacity is k_s e^{-z/Hc} below z_sw = H ln(P_0/p_sw) and
    k_t e^{-z/Hc} above (Hc = H for absorption, H/2 for CIA's rho^2):
    tau(b) = k_t tau_1(b) + (k_s - k_t) tau_below(b), with tau_1 the Bessel-K1
    chord integral of a unit profile, 2 b K1(b/Hc) e^{(Rp - b)/Hc}, and
    tau_below its part below z_sw, 2 b int_0^{acosh(R_sw/b)}
    e^{-(b cosh u - Rp)/Hc} cosh u du (r = b cosh u along the chord)."""
    _, P = F.pressure_grid(1e6, 1e-4, N)
    H = K_BOLTZMANN * T * R_JUP ** 2 / (mu_kg * GM_JUP)
    ztop = H * np.log(P[0] / P[-1])
    z_sw = H * np.log(P[0] / p_sw)
    R_sw = R_JUP + z_sw

    def tau(z):
        b = R_JUP + z
        t1 = 2.0 * b * special.k1e(b / Hc) * np.exp(-z / Hc)
        tb = 0.0
        if b < R_sw:
            g = lambda u: np.exp(-(b * (np.cosh(u) - 1.0) + z) / Hc) * np.cosh(u)
            tb, _ = integrate.quad(g, 0.0, np.arccosh(R_sw / b), epsabs=0, epsrel=1e-12, limit=200)
            tb *= 2.0 * b
        return k_t * t1 + (k_s - k_t) * tb

    f = lambda z: 2.0 * (R_JUP + z) * (-np.expm1(-tau(z)))
    a1, _ = integrate.quad(f, 0.0, z_sw, epsabs=0, epsrel=1e-11, limit=400)
    a2, _ = integrate.quad(f, z_sw, ztop, epsabs=0, epsrel=1e-11, limit=400)
    return (R_JUP ** 2 + a1 + a2) / R_SUN ** 2, R_JUP ** 2 / R_SUN ** 2


def _fill_mass():
    f_h2, f_he = 1.0 / (1.0 + HE_H2_RATIO), HE_H2_RATIO / (1.0 + HE_H2_RATIO)
    return f_h2 * MASSES_AMU["H2"] + f_he * MASSES_AMU["He"]


def test_two_layer_converges_to_continuous_model():
    """A constant-cross-section absorber with a two-layer profile whose
    switch (10 Pa) is a shell boundary of every grid used, and whose mass is
    the fill's mean, so that mu does not change across the step: the
    discrete transit depth converges to the continuous model with the step,
    at the order of the constant-profile pin.  A step placed one layer off,
    or the two values swapped, breaks the order or the bound."""
    T, sigma_cm2 = 1500.0, 1e-22
    fill = _fill_mass()
    t = _const_tables(sigma_cm2, mass=fill)
    chi_s, chi_t, p_sw = 1e-3, 1e-6, 10.0
    mu = fill * AMU_KG
    H = K_BOLTZMANN * T * R_JUP ** 2 / (mu * GM_JUP)
    errs = []
    for N in (100, 200, 400, 800):
        m = _model(N=N, T=T, vmr=np.log10(chi_s), gravity=1)
        m.update(log10_vmr_top=np.array([np.log10(chi_t)]), vmr_switch=np.array([p_sw]))
        D = F.forward_model(m, t)["depth"][0]
        n0 = F.pressure_grid(1e6, 1e-4, N)[1][0] / (K_BOLTZMANN * T)
        k = sigma_cm2 * 1e-4 * n0
        Dc, D0 = _continuous_step_depth(N, k * chi_s, k * chi_t, H, T, mu, p_sw)
        errs.append(abs(D - Dc) / (Dc - D0))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert errs[0] < 3e-3, errs
    assert all(1.3 < o < 2.0 for o in orders), (errs, orders)


def test_two_layer_cia_follows_the_per_layer_fill():
    """An absorber with no cross-section at 30 % below the switch and 1e-6
    above (the switch at 1e4 Pa, a shell boundary of every grid used, deep
    enough for CIA to matter), and one H2-H2 CIA pair of constant
    cross-section: the CIA opacity
    1e-10 sigma_c chi_H2^2 rho^2 steps with the fill gas (chi_H2 = (1 -
    chi)/(1 + r) per layer), and the depth converges to the continuous model
    with that step (rho^2: half the scale height)."""
    from test_oracle_pins import _cia_tables
    T, sigma_c, p_sw = 1500.0, 1e-43, 1e4
    fill = _fill_mass()
    t = _cia_tables(sigma_c, (1, 1))
    t.abs_mass = np.array([fill])
    chi_s, chi_t = 0.3, 1e-6
    h2 = lambda c: (1.0 - c) / (1.0 + HE_H2_RATIO)
    mu = fill * AMU_KG
    H = K_BOLTZMANN * T * R_JUP ** 2 / (mu * GM_JUP)
    errs = []
    for N in (100, 200, 400, 800):
        m = _model(N=N, T=T, vmr=np.log10(chi_s), gravity=1)
        m.update(log10_vmr_top=np.array([np.log10(chi_t)]), vmr_switch=np.array([p_sw]))
        D = F.forward_model(m, t)["depth"][0]
        n0 = F.pressure_grid(1e6, 1e-4, N)[1][0] / (K_BOLTZMANN * T)
        k = 1e-10 * sigma_c * n0 ** 2
        Dc, D0 = _continuous_step_depth(N, k * h2(chi_s) ** 2, k * h2(chi_t) ** 2, 0.5 * H, T, mu, p_sw)
        errs.append(abs(D - Dc) / (Dc - D0))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert errs[0] < 3.5e-3, errs
    assert all(1.3 < o < 2.0 for o in orders), (errs, orders)


def test_two_layer_per_layer_fill_and_validity():
    """The fill gases take the rest of each layer's volume; a model is
    invalid when any layer's absorbers reach 1."""
    P = np.array([1e5, 1e3, 1e1])
    chi = oracle.two_layer_vmr(np.log10([0.3, 0.1]), np.log10([0.01, 0.6]), [1e4, 1e2], P)
    assert np.allclose(chi, [[0.3, 0.1], [0.01, 0.1], [0.01, 0.6]], rtol=1e-15)
    c, h2, he, mu, valid = oracle.chemistry_profile(chi, 0.17, [18.0, 44.0], 2.0, 4.0, 1.0)
    assert valid
    assert np.allclose(h2 + he + chi.sum(1), 1.0, rtol=1e-15)
    assert np.allclose(he / h2, 0.17, rtol=1e-14)
    chi[2, 1] = 0.995
    assert not oracle.chemistry_profile(chi, 0.17, [18.0, 44.0], 2.0, 4.0, 1.0)[4]
