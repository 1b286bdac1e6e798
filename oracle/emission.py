"""FP64 oracle: the emission (eclipse) forward model, step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in
float64.

Paper passages followed (arXiv:1912.07759, Forward Models section):
  * a plane-parallel atmosphere whose emission is integrated layer by layer:
    the intensity leaving the top at cos(angle) mu is the surface's Planck
    intensity attenuated by the total optical depth plus the integral of the
    Planck intensity of the gas along the optical depth;
  * the flux integral over mu by N-point Gauss-Legendre quadrature with the
    weights times the abscissas;
  * F_p / F_s = I / I_s (Rp / Rs)^2.
The atmosphere itself (pressure grid, chemistry, altitudes, opacity, cloud
deck) is the transmission oracle's (``oracle.forward``), with its readings.

Readings taken where the paper is silent, ambiguous or garbled (same list as
the design notes):
  E1  the printed intensity integral lacks the 1/mu of the formal solution
      (with it an isothermal atmosphere emits B(T) at every angle, as it
      must): I(mu) = B(T_s) e^{-tau_s/mu} + int_0^{tau_s} B(T(t)) e^{-t/mu}
      dt/mu.
  E2  discretisation: each shell (the transmission shells, bounded by h_0 = 0,
      midpoints, h_N = z_{N-1}) has its layer's opacity and temperature;
      tau_l is the vertical optical depth from the top down to the bottom of
      shell l, sum_{m >= l} kappa_m (h_{m+1} - h_m); a shell with constant B
      contributes B_l (e^{-tau_{l+1}/mu} - e^{-tau_l/mu}) exactly.
  E3  T_s, "the temperature at maximum atmospheric pressure", is the bottom
      layer's temperature.
  E4  the flux: with N-point Gauss-Legendre nodes mu_i and weights w_i on
      [0, 1] (sum w_i = 1), the disc-integrated intensity is
      2 sum_i w_i mu_i I(mu_i) (the flux 2 pi int I mu dmu over pi), so that
      an isothermal planet at the star's temperature gives (Rp/Rs)^2.
  E5  I_s is the intensity of a blackbody star at T_star; B is Planck's law
      per unit wavenumber, 2 h c^2 nu^3 / (exp(h c nu / k_B T) - 1) with nu
      in m^-1 (h and c exact SI; k_B as passed).

Pins (tests/test_oracle_emission.py): Gauss-Legendre moments are exact to
degree 2N-1 and not beyond; Planck's law integrates to sigma T^4 / pi and
peaks at the Wien constant; an isothermal atmosphere gives B(T)/B(T*)
(Rp/Rs)^2 exactly for any opacity; a transparent one shows the surface; an
opaque one shows its top layer; the formal solution with a source linear in
optical depth converges to a + b mu (1 - e^{-tau_s/mu}); the vertical
optical depth converges to the hydrostatic column chi sigma Delta P /(mu g).
"""

import numpy as np

from .forward import (bin_spectrum, bin_weights, altitude, cloud_opacity, model_chemistry,
                      opacity, pressure_grid, shell_boundaries)

H_PLANCK = 6.62607015e-34   # J s (exact SI)
C_LIGHT = 299792458.0       # m/s (exact SI)


def planck(wn_cm1, T, k_B):
    """Reading E5: Planck intensity per unit wavenumber,
    B = 2 h c^2 nu^3 / (exp(h c nu / (k_B T)) - 1), nu = 100 wn (m^-1),
    in W m^-2 sr^-1 (m^-1)^-1."""
    nu = 100.0 * np.asarray(wn_cm1, dtype=np.float64)
    x = H_PLANCK * C_LIGHT * nu / (k_B * T)
    return 2.0 * H_PLANCK * C_LIGHT ** 2 * nu ** 3 / np.expm1(x)


def gauss_legendre_mu(n):
    """N-point Gauss-Legendre abscissas and weights on [0, 1] (weights sum
    to 1): the nodes of the degree-n Legendre polynomial mapped from
    [-1, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def layer_thickness(z):
    """Reading E2: thickness of each shell, h_{l+1} - h_l."""
    h = shell_boundaries(z)
    return h[1:] - h[:-1]


def vertical_optical_depth(kappa, dz):
    """tau[l, w] = sum_{m >= l} kappa[m, w] dz[m]: from the top of the
    atmosphere down to the bottom of shell l (reading E2)."""
    col = kappa * dz[:, None]
    return np.cumsum(col[::-1], axis=0)[::-1]


def emergent_intensity(tau, B_layer, B_surface, mu):
    """Readings E1, E2: the intensity leaving the top at cos(angle) mu,
    I = B_s e^{-tau_0/mu} + sum_l B_l (e^{-tau_{l+1}/mu} - e^{-tau_l/mu}),
    tau_N = 0 at the top."""
    E = np.exp(-tau / mu)                                   # [N, W]
    E_up = np.vstack([E[1:], np.ones((1, E.shape[1]))])     # e^{-tau_{l+1}/mu}
    return B_surface * E[0] + np.sum(B_layer * (E_up - E), axis=0)


def emission_model(m, tables, channels=None, n_mu=4, T_star=5800.0, keep=False):
    """One model (the same dict as oracle.forward.forward_model) seen in
    emission: F_p/F_s over its window (``fpfs``), binned if channels are
    given (``binned``), and ``valid``.  Reading E4 for the flux, E5 for the
    star, E3 for the surface."""
    T = m["T"]
    N = len(T)
    lo, hi = m["wn_lo"], m["wn_hi"]
    _, P = pressure_grid(m["p_bot"], m["p_top"], N)
    chi, chi_h2, chi_he, mu_kg, valid = model_chemistry(m, tables, P)
    z = altitude(T, P, mu_kg, m["Rp"], m["GM"], m["k_B"], m["gravity"])
    kappa = opacity(T, P, chi, chi_h2, chi_he, tables, m["k_B"], lo, hi,
                    t_interp=m.get("t_interp", "linear"))
    sigma_c = m.get("cloud_sigma", 0.0)
    if sigma_c != 0.0:
        kappa_c, _ = cloud_opacity(P, T, m["k_B"], sigma_c, m["cloud_p_top"], m["cloud_p_bottom"])
        kappa = kappa + kappa_c[:, None]
    dz = layer_thickness(z)
    tau = vertical_optical_depth(kappa, dz)
    wn = tables.wn[lo:hi]
    B_layer = np.stack([planck(wn, T[l], m["k_B"]) for l in range(N)])
    mus, ws = gauss_legendre_mu(n_mu)
    flux = np.zeros(hi - lo)
    for mu, w in zip(mus, ws):
        flux = flux + 2.0 * w * mu * emergent_intensity(tau, B_layer, B_layer[0], mu)
    fpfs = flux / planck(wn, T_star, m["k_B"]) * (m["Rp"] / m["Rs"]) ** 2
    out = {"fpfs": fpfs, "valid": valid}
    if channels is not None:
        wgt = bin_weights(tables.wn, channels.lo, channels.hi, lo, hi)
        out["binned"] = bin_spectrum(fpfs, wgt)
    if keep:
        out.update(z=z, dz=dz, kappa=kappa, tau=tau, B_layer=B_layer, mu=mu_kg, P=P)
    return out
