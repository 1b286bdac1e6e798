"""Seeded temperature profiles, channel edges and observation noise.

The Guillot (2010, A&A 520, A27, eq. 29) radiative-equilibrium profile is the
paper's ``Guillot2010`` temperature class (Temperature Profiles section,
table of temperature profiles); the paper names its parameters but does not
print the formula, so it is restated here from the original article.  It is
an input generator: the forward model receives the resulting per-layer
temperatures like any free (layer-by-layer) profile.
"""

import numpy as np


def log_midpoint_pressures(p_bot, p_top, n_layers):
    """Pressures at the log-midpoints of ``n_layers`` equal log-P intervals
    between ``p_bot`` and ``p_top`` (bottom first).  Used only to place the
    temperature profile's sample points."""
    t = (np.arange(n_layers) + 0.5) / n_layers
    return 10.0 ** (np.log10(p_bot) + t * (np.log10(p_top) - np.log10(p_bot)))


def guillot_T(P_pa, g_ms2, T_irr, kappa_ir=0.01, gamma=0.05, T_int=100.0, f=0.25):
    """Guillot (2010) eq. 29 temperature at pressures ``P_pa`` (SI units:
    kappa_ir in m^2 kg^-1, g in m s^-2)."""
    P = np.asarray(P_pa, dtype=np.float64)
    tau = kappa_ir * P / g_ms2
    s3 = np.sqrt(3.0)
    t_int4 = 0.75 * T_int ** 4 * (2.0 / 3.0 + tau)
    t_irr4 = 0.75 * T_irr ** 4 * f * (2.0 / 3.0 + 1.0 / (gamma * s3)
                                      + (gamma / s3 - 1.0 / (gamma * s3))
                                      * np.exp(-gamma * tau * s3))
    return (t_int4 + t_irr4) ** 0.25


def smooth_perturbation(rng, n, n_modes=4):
    """A smooth seeded function on n points with max |value| = 1."""
    t = np.linspace(0.0, 1.0, n)
    y = np.zeros(n)
    for m in range(1, n_modes + 1):
        y += rng.normal() / m * np.sin(np.pi * m * t + rng.uniform(0, 2 * np.pi))
    return y / np.max(np.abs(y))


def avoid_nodes(T, T_nodes, min_gap=0.01):
    """Shift any temperature closer than ``min_gap`` K to a table node by
    2*min_gap, so finite differences never straddle a bracket kink."""
    T = np.array(T, dtype=np.float64, copy=True)
    nodes = np.asarray(T_nodes, dtype=np.float64)
    d = T[:, None] - nodes[None, :]
    close = np.abs(d) < min_gap
    rows = np.any(close, axis=1)
    T[rows] += 2.0 * min_gap
    return T


def log_uniform_channels(wn, n_ch):
    """``n_ch`` contiguous channels with log-uniform wavenumber edges spanning
    the grid ``wn``; returns (lo, hi) edge arrays in cm^-1."""
    e = np.logspace(np.log10(wn[0]), np.log10(wn[-1]), n_ch + 1)
    return e[:-1].copy(), e[1:].copy()


def gaussian_noise(rng, n, sigma):
    """Seeded N(0, sigma^2) noise."""
    return rng.normal(0.0, sigma, n)
