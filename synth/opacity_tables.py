"""Seeded synthetic opacity tables shaped like the paper's cross-section data.

The paper's benchmarks use ExoMol / HITRAN cross-sections on temperature x
pressure x wavenumber grids (Opacities section; Benchmark section).  Those
files are not available, so every table here is a seeded stand-in with the
same shape and a comparable dynamic range:

* molecular cross-sections: a forest of pressure- and temperature-broadened
  Lorentzian lines on top of a constant floor (cm^2 / molecule);
* collision-induced absorption: smooth bands near the H2 fundamental
  (~4160 cm^-1) and first overtone (~8320 cm^-1) on a weak continuum
  (cm^5 / molecule^2);
* Rayleigh scattering: a nu^4 law per species (cm^2 / molecule).

Nothing here evaluates the forward model.
"""

import numpy as np


def wn_grid_linear(lo_cm1, hi_cm1, n):
    """``n`` equally spaced wavenumbers on [lo, hi] (cm^-1)."""
    return np.linspace(lo_cm1, hi_cm1, n)


def wn_grid_log_wavelength(lam_lo_um, lam_hi_um, n):
    """``n`` wavenumbers, log-uniform in wavelength between the two limits.

    Returned in increasing wavenumber order (cm^-1).
    """
    lam = np.logspace(np.log10(lam_hi_um), np.log10(lam_lo_um), n)
    return 1e4 / lam


def line_forest(rng, wn, T_grid, log10P_grid, n_lines, s_range=(1e-24, 1e-19),
                floor=1e-27, gamma0_range=(0.05, 0.1), beta_range=(-1.0, 1.0),
                half_window_cm1=25.0, half_window_gamma=30.0):
    """Cross-section table ``sigma[nT][nP][nW]`` in cm^2 / molecule.

    sigma(T, P, nu) = floor + sum_l S_l (T/1000)^beta_l * g^2 / ((nu-nu_l)^2 + g^2)
    with g = max(gamma0_l (P/1e5 Pa) (296/T)^0.5, local grid spacing), so
    widths grow with pressure and stay resolved by the grid at low pressure.
    Each line is evaluated within +-min(25 cm^-1, 30 g_max) of its centre.
    """
    wn = np.asarray(wn, dtype=np.float64)
    T = np.asarray(T_grid, dtype=np.float64)
    P = 10.0 ** np.asarray(log10P_grid, dtype=np.float64)
    nT, nP, nW = len(T), len(P), len(wn)
    sigma = np.full((nT, nP, nW), floor, dtype=np.float64)
    nu = rng.uniform(wn[0], wn[-1], n_lines)
    lo, hi = np.log10(s_range[0]), np.log10(s_range[1])
    S = 10.0 ** rng.uniform(lo, hi, n_lines)
    beta = rng.uniform(beta_range[0], beta_range[1], n_lines)
    g0 = rng.uniform(gamma0_range[0], gamma0_range[1], n_lines)
    spacing = np.gradient(wn)
    press_fac = (P / 1e5)[None, :] * np.sqrt(296.0 / T)[:, None]     # [nT, nP]
    for k in range(n_lines):
        dnu = np.interp(nu[k], wn, spacing)
        gam = np.maximum(g0[k] * press_fac, dnu)                     # [nT, nP]
        half = min(half_window_cm1, half_window_gamma * float(gam.max()))
        i0 = int(np.searchsorted(wn, nu[k] - half))
        i1 = int(np.searchsorted(wn, nu[k] + half))
        if i1 <= i0:
            continue
        d2 = (wn[i0:i1] - nu[k]) ** 2                                 # [n]
        g2 = (gam * gam)[:, :, None]
        strength = (S[k] * (T / 1000.0) ** beta[k])[:, None, None]
        sigma[:, :, i0:i1] += strength * g2 / (d2[None, None, :] + g2)
    return sigma


def replicate_forest(rng, base, shift_max=200, scale_range=(0.3, 3.0)):
    """A pseudo-molecule made from an existing table by a seeded wavenumber
    shift (circular, in grid points) and a seeded overall scale.

    The paper builds its molecule-scaling benchmark the same way, by
    replicating cross-sections (Benchmark section, forward-model timings
    versus number of molecules).
    """
    s = int(rng.integers(-shift_max, shift_max + 1))
    f = float(10.0 ** rng.uniform(np.log10(scale_range[0]), np.log10(scale_range[1])))
    return np.roll(base, s, axis=-1) * f


def cia_table(rng, wn, T_grid, peak_range=(1e-46, 1e-45)):
    """Collision-induced absorption ``[nT][nW]`` in cm^5 / molecule^2.

    Gaussian bands at the H2 fundamental and first overtone plus a weak
    continuum; amplitude and width rise with temperature.
    """
    wn = np.asarray(wn, dtype=np.float64)
    T = np.asarray(T_grid, dtype=np.float64)
    lo, hi = np.log10(peak_range[0]), np.log10(peak_range[1])
    peak0 = 10.0 ** rng.uniform(lo, hi)
    alpha = rng.uniform(0.3, 1.0)
    w1 = rng.uniform(300.0, 600.0)
    w2 = rng.uniform(400.0, 800.0)
    r2 = rng.uniform(0.05, 0.2)
    cont = rng.uniform(0.01, 0.05)
    tt = (T / 1000.0)[:, None]
    wid = tt ** 0.3
    amp = peak0 * tt ** alpha
    x = wn[None, :]
    band = (np.exp(-((x - 4160.0) / (w1 * wid)) ** 2)
            + r2 * np.exp(-((x - 8320.0) / (w2 * wid)) ** 2)
            + cont * np.exp(-x / 20000.0))
    return amp * band


def rayleigh_table(rng, wn, n_abs, c_h2=8.14e-45, c_he=5.5e-46,
                   c_abs_range=(1e-45, 1e-44)):
    """Rayleigh cross-sections ``[n_abs + 2][nW]`` = c_s nu^4 (cm^2).

    Row order: absorbers, then H2, then He.  c_H2 is the leading term of the
    Dalgarno & Williams (1962) H2 fit; the absorber coefficients are seeded.
    """
    wn = np.asarray(wn, dtype=np.float64)
    lo, hi = np.log10(c_abs_range[0]), np.log10(c_abs_range[1])
    c = np.concatenate([10.0 ** rng.uniform(lo, hi, n_abs), [c_h2, c_he]])
    return c[:, None] * wn[None, :] ** 4
