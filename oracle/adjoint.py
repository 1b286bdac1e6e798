"""FP64 oracle: reference gradient of chi^2 by hand-written reverse mode.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no gradients; its retrieval layer only evaluates a likelihood
(Optimization section) over parameters that may live in log10 space.  This
module differentiates the forward model of ``oracle.forward`` (same readings)
composed with chi^2 = sum_c ((D_c - O_c)/sigma_c)^2 (reading A14), with
respect to the per-layer temperatures, the log10 mixing ratios of the
absorbers (the log10 parameter space of the Optimization section; the fill
gases respond through the sum constraint) and the planet radius.

It walks the forward steps in reverse: binning, depth, exp and annulus sum,
the chord contraction, the cloud deck's contribution, the opacity (bracket
slopes in T, number density, mixing ratios), the chord geometry, the
altitude recursion and the chemistry.  Derivatives at table nodes and under clamps are one-sided: the
lower-closed bracket's slope, zero under a clamp (reading A16).

Pinned by complex-step differentiation of ``oracle.forward`` (agreement to
~1e-12) and by central finite differences (tests/test_oracle_adjoint.py).
"""

import numpy as np

from .forward import (CM2_TO_M2, CM5_TO_M5, bin_weights, bracket,
                      forward_model, number_density)


def _xsec_value_and_dT(table, T_grid, log10P_grid, T, log10P, zero_rule="both"):
    """Bilinear (T, log10 P) value and its T-derivative at fixed P."""
    iT, Tu, T_lo, T_hi = bracket(T_grid, T)
    iP, xu, P_lo, _ = bracket(log10P_grid, log10P)
    W = table.shape[-1]
    if (zero_rule == "both" and T_lo and P_lo) or (zero_rule == "p_only" and P_lo):
        return np.zeros(W), np.zeros(W)
    T1, T2 = T_grid[iT], T_grid[iT + 1]
    x1, x2 = log10P_grid[iP], log10P_grid[iP + 1]
    wP = (xu - x1) / (x2 - x1)
    m1 = (table[iT + 1, iP] - table[iT, iP]) / (T2 - T1)
    m2 = (table[iT + 1, iP + 1] - table[iT, iP + 1]) / (T2 - T1)
    s1 = table[iT, iP] + m1 * (Tu - T1)
    s2 = table[iT, iP + 1] + m2 * (Tu - T1)
    val = s1 + (s2 - s1) * wP
    inside = not (T_lo or float(np.real(T)) >= T_grid[-1])
    dT = ((1.0 - wP) * m1 + wP * m2) if inside else np.zeros(W)
    return val, dT


def _cia_value_and_dT(table, T_grid, T):
    iT, Tu, T_lo, _ = bracket(T_grid, T)
    T1, T2 = T_grid[iT], T_grid[iT + 1]
    m = (table[iT + 1] - table[iT]) / (T2 - T1)
    val = table[iT] + m * (Tu - T1)
    inside = not (T_lo or float(np.real(T)) >= T_grid[-1])
    return val, (m if inside else np.zeros_like(m))


def chi2_and_grad(m, tables, channels, obs, sigma):
    """chi^2 of one model against ``obs`` (per channel, with ``sigma``) and
    its gradient.  Returns dict(chi2, binned, dT[N], dlog10_vmr[n_abs], dRp).
    """
    f = forward_model(m, tables, channels, keep=True)
    T = np.asarray(m["T"], dtype=np.float64)
    N = len(T)
    lo, hi = m["wn_lo"], m["wn_hi"]
    Rp, Rs, GM, kB = m["Rp"], m["Rs"], m["GM"], m["k_B"]
    P, z, dl, A, kappa, tau = f["P"], f["z"], f["dl"], f["A"], f["kappa"], f["tau"]
    chi, chi_h2, chi_he, mu = f["chi"], f["chi_h2"], f["chi_he"], f["mu"]
    n_abs = tables.n_abs
    chi_s = np.concatenate([chi, [chi_h2, chi_he]])

    # chi^2 and binning
    binned = f["binned"]
    r = (binned - obs) / sigma
    c2 = float(np.sum(r * r))
    Dbar_c = 2.0 * r / sigma
    w = bin_weights(tables.wn, channels.lo, channels.hi, lo, hi)
    omega = w / np.sum(w, axis=1)[:, None]
    Dbar = omega.T @ Dbar_c                                  # [W]

    # depth D = (Rp^2 + a)/Rs^2
    Rp_bar = float(np.sum(Dbar) * 2.0 * Rp / Rs ** 2)
    a_bar = Dbar / Rs ** 2
    e = np.exp(-tau)
    A_bar = (1.0 - e) @ a_bar                                # [N]
    tau_bar = A[:, None] * e * a_bar[None, :]                # [N, W]

    # tau = dl @ kappa (dl upper triangular)
    dl_bar = np.triu(tau_bar @ kappa.T)
    kappa_bar = dl.T @ tau_bar

    # cloud deck: tau += tau_c[:, None], tau_c = dl @ kappa_c, kappa_c =
    # sigma rho on the deck (d rho/dT = -rho/T; the deck's layers are fixed
    # by the pressure grid, so its bounds have no derivative).  An opaque
    # deck has none either: its rays have e^-tau = 0 and the others no path
    # through it.
    kappa_c = f["kappa_c"]
    cT_bar = np.zeros(N)
    if kappa_c is not None and np.isfinite(m["cloud_sigma"]):
        tc_bar = np.sum(tau_bar, axis=1)                     # [N]
        dl_bar += np.triu(np.outer(tc_bar, kappa_c))
        cT_bar = (dl.T @ tc_bar) * (-kappa_c / T)

    # opacity
    n = number_density(P, T, kB)
    lp = np.log10(P)
    T_bar = cT_bar.copy()
    chi_bar = np.zeros(n_abs + 2)
    for l in range(N):
        kb = kappa_bar[l]
        E1 = np.zeros(hi - lo)
        dE1 = np.zeros(hi - lo)
        for i in range(n_abs):
            v, d = _xsec_value_and_dT(tables.xsec[i][:, :, lo:hi], tables.T_grid,
                                      tables.log10P_grid, T[l], lp[l])
            E1 += chi[i] * v
            dE1 += chi[i] * d
            chi_bar[i] += CM2_TO_M2 * n[l] * np.dot(kb, v)
        if tables.rayleigh is not None:
            for s in range(n_abs + 2):
                R = tables.rayleigh[s, lo:hi]
                E1 += chi_s[s] * R
                chi_bar[s] += CM2_TO_M2 * n[l] * np.dot(kb, R)
        E2 = np.zeros(hi - lo)
        dE2 = np.zeros(hi - lo)
        for p in range(tables.cia.shape[0]):
            a, b = tables.cia_pair[p]
            v, d = _cia_value_and_dT(tables.cia[p][:, lo:hi], tables.Tcia_grid, T[l])
            E2 += chi_s[a] * chi_s[b] * v
            dE2 += chi_s[a] * chi_s[b] * d
            proj = CM5_TO_M5 * n[l] ** 2 * np.dot(kb, v)
            chi_bar[a] += proj * chi_s[b]
            chi_bar[b] += proj * chi_s[a]
        dn = -n[l] / T[l]
        dk = (CM2_TO_M2 * (dn * E1 + n[l] * dE1)
              + CM5_TO_M5 * (2.0 * n[l] * dn * E2 + n[l] ** 2 * dE2))
        T_bar[l] += np.dot(kb, dk)

    # geometry: A_j = 2 (Rp + z_j)(h_{j+1} - h_j), dl from q_j(h)
    h = np.zeros(N + 1)
    h[1:N] = 0.5 * (z[:-1] + z[1:])
    h[N] = z[N - 1]
    z_bar = np.zeros(N)
    h_bar = np.zeros(N + 1)
    dh = h[1:] - h[:-1]
    Rp_bar += float(np.sum(A_bar * 2.0 * dh))
    z_bar += A_bar * 2.0 * dh
    h_bar[1:] += A_bar * 2.0 * (Rp + z)
    h_bar[:-1] -= A_bar * 2.0 * (Rp + z)

    def q_adj(j, hk, gbar):
        """Accumulate gbar * d q_j(hk) into z_bar[j], h_bar, Rp_bar."""
        qv = np.sqrt((hk - z[j]) * (2.0 * Rp + hk + z[j]))
        if qv == 0.0:
            return 0.0, 0.0, 0.0      # identically-zero chord of the top ray
        return gbar * (Rp + hk) / qv, -gbar * (Rp + z[j]) / qv, gbar * (hk - z[j]) / qv

    for j in range(N):
        for k in range(j, N):
            g = 2.0 * dl_bar[j, k]
            if g == 0.0:
                continue
            dh_, dz_, dR_ = q_adj(j, h[k + 1], g)
            h_bar[k + 1] += dh_
            z_bar[j] += dz_
            Rp_bar += dR_
            if k > j:
                dh_, dz_, dR_ = q_adj(j, h[k], -g)
                h_bar[k] += dh_
                z_bar[j] += dz_
                Rp_bar += dR_
    # h -> z
    for k in range(1, N):
        z_bar[k - 1] += 0.5 * h_bar[k]
        z_bar[k] += 0.5 * h_bar[k]
    z_bar[N - 1] += h_bar[N]

    # altitude recursion, in reverse
    mu_bar = 0.0
    grav = m["gravity"]
    for l in range(N - 1, 0, -1):
        L = np.log(P[l] / P[l - 1])
        if grav == 0:
            g = GM / (Rp + z[l - 1]) ** 2
            H = kB * T[l - 1] / (mu * g)
            dz_dzprev = 1.0 - L * 2.0 * H / (Rp + z[l - 1])
            dz_dRp = -L * 2.0 * H / (Rp + z[l - 1])
        else:
            g = GM / Rp ** 2
            H = kB * T[l - 1] / (mu * g)
            dz_dzprev = 1.0
            dz_dRp = -L * 2.0 * H / Rp
        T_bar[l - 1] += z_bar[l] * (-L * H / T[l - 1])
        mu_bar += z_bar[l] * (L * H / mu)
        Rp_bar += z_bar[l] * dz_dRp
        z_bar[l - 1] += z_bar[l] * dz_dzprev

    # chemistry: mu = amu * sum chi_s m_s; fill gases
    masses = np.concatenate([tables.abs_mass, [tables.h2_mass, tables.he_mass]])
    chi_bar += mu_bar * m["amu"] * masses
    r_he = m["he_h2"]
    fill_bar = chi_bar[n_abs] + r_he * chi_bar[n_abs + 1]
    chi_abs_bar = chi_bar[:n_abs] - fill_bar / (1.0 + r_he)
    x_bar = chi_abs_bar * chi * np.log(10.0)
    return {"chi2": c2, "binned": binned, "dT": T_bar, "dlog10_vmr": x_bar,
            "dRp": Rp_bar}


def chi2_grad_batch(tables, batch, channels, obs, sigma, models=None):
    idx = range(batch.B) if models is None else models
    return [chi2_and_grad(batch.model(b), tables, channels, obs[b], sigma)
            for b in idx]
