"""FP64 oracle: the transmission forward model, step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in
float64; every arithmetic function also accepts complex128 parameters so that
complex-step differentiation can pin the reference gradient (bracket choices
use real parts only).

Paper passages followed (arXiv:1912.07759):
  * Pressure Profiles subsection: N+1 log-spaced boundary pressures, layer
    centre P_l = p_l sqrt(p_{l+1}/p_l).
  * Chemistry subsection: constant free-chemistry gases; fill gases share the
    remaining volume by ``ratio`` relative to the first fill molecule;
    active and inactive molecules both set the mean molecular weight.
  * Forward Models section, altitude equation: z_0 = 0 at the bottom,
    z_l = z_{l-1} - H_{l-1} ln(P_l / P_{l-1}), H_l = k_B T_l / (mu_l g_l).
  * Forward Models section, transit-depth equations: D = (Rp^2 + a)/Rs^2,
    a = 2 int_0^{z_max} (Rp + z)(1 - exp(-tau(z))) dz.
  * Equations tot_opt_dpth, opt_dpth, cia_opt_dpth and contrib: tau is the
    sum over contributions of int zeta w rho dz' along the line of sight,
    with w = chi for absorption and Rayleigh, w = chi chi' and rho^2 for CIA.
  * Opacities section: linear interpolation in T and in P between the
    bracketing grid points; the out-of-range rules.
  * Binning subsection: overlap weights w_ij, F_j = sum F_i w_ij / sum w_ij.

Readings taken where the paper is silent or ambiguous (same list as the
design notes):
  A1  the P axis is interpolated linearly in log10 P (``p_interp="log"``);
      the literal linear-in-P form is available as ``p_interp="linear"``.
  A3  T and log10 P clamp independently to the grid edges; T below the grid
      AND P below the grid gives zero cross-section (``zero_rule="both"``;
      the alternative "P below the grid alone" is ``zero_rule="p_only"``).
      CIA clamps in T without a zero rule.
  A4  g at a layer is GM/(Rp + z)^2 at that layer's altitude (``gravity=0``);
      ``gravity=1`` uses the constant GM/Rp^2.
  A5  the altitude step uses H of the lower layer (explicit first order).
  A7  rho is the ideal-gas number density P/(k_B T) at the layer centre.
  A8  tables are per molecule in cm^2 (x1e-4 to m^2); CIA in cm^5 (x1e-10).
  A9  rays at the layer-centre altitudes z_j; shells bounded by h_0 = 0,
      h_k = (z_{k-1} + z_k)/2, h_N = z_{N-1}; each shell carries its layer's
      opacity; annulus weights A_j = 2 (Rp + z_j)(h_{j+1} - h_j).
  A12 binning uses the general overlap weight on wavenumber edges; a
      channel with no overlap in the window is NaN.
  A13 native bin edges are midpoints between grid points, end bins mirrored.
  A14 chi^2 = sum_c ((D_c - O_c)/sigma_c)^2.
  A18 Rayleigh applies to every species (absorbers, H2, He); CIA pairs are
      given by species ids (absorbers 0..n_abs-1, then H2, then He).
  A25 the exponential temperature scheme (Opacities section, sigma(T) =
      a e^{-b/T} through the two bracketing grid temperatures, then linear
      along log10 P as in A1) applies to the cross-section tables; CIA stays
      linear in T.  Where a node value is not positive (the logarithm in b is
      undefined) that (P node, wavenumber) falls back to the linear scheme.
      Out-of-range T clamps to the edge node as in A3 (the scheme then
      returns the node value).
  A26 the two-layer mixing profile (Chemistry subsection, its surface and
      top mixing ratios): absorber i has its surface value at the layers
      whose centre pressure is at or above a switch pressure p_i and its top
      value above (lower pressure), a step with no smoothing; the fill gases
      and the mean molecular weight follow per layer, and the altitude step
      uses the lower layer's mu as A5 uses its T.
  A24 the flat-opacity cloud deck (equation clouds) is sigma rho on the
      layers whose centre pressure lies between the two deck pressures
      (bounds included, either order); sigma = +inf is the fully opaque
      deck, whose optical depth is +inf on every ray with a nonzero path
      through it.

Pins (tests/test_oracle_pins.py): zero opacity gives (Rp/Rs)^2 exactly; the
opaque limit equals the closed-form trapezoid sum; the constant-g isothermal
altitude equals H ln(P_0/P_l); with T linear in ln P the altitude's error
is exactly that of a left Riemann sum (the lower layer's H); the isothermal
constant-cross-section model converges to the exact continuous transit depth
(Bessel K1 chord integral), and so does a constant-CIA model (rho^2 halves
the scale height; H2-H2, H2-He and absorber-H2 pairs);
chords match a 50-digit mpmath evaluation and a fine-step quadrature of
int kappa ds along the ray; the chord sum equals the full chord; bilinear
interpolation is exact on T-logP-bilinear tables and at nodes; each clamp
case; binning identities; monotonicity in abundance with geometry frozen.
"""

import numpy as np

CM2_TO_M2 = 1e-4      # cross-section cm^2 -> m^2 (reading A8)
CM5_TO_M5 = 1e-10     # CIA cm^5 -> m^5 (reading A8)


# --------------------------------------------------------------------------
# Profiles and chemistry
# --------------------------------------------------------------------------
def pressure_grid(p_bot, p_top, n_layers):
    """Pressure Profiles subsection: ``n_layers + 1`` boundary pressures
    equally spaced in log between p_bot (bottom, p_0) and p_top, and the
    geometric layer centres P_l = p_l sqrt(p_{l+1} / p_l)."""
    p = 10.0 ** np.linspace(np.log10(p_bot), np.log10(p_top), n_layers + 1)
    P = p[:-1] * np.sqrt(p[1:] / p[:-1])
    return p, P


def chemistry(log10_vmr, he_h2, abs_mass, h2_mass, he_mass, amu):
    """Chemistry subsection (free chemistry, constant gases, fill gases).

    chi_i = 10**log10_vmr_i for the absorbers.  The fill gases H2 and He take
    the remaining volume 1 - sum chi_i with He/H2 = ``he_h2`` (reading A6).
    The mean molecular weight sums over every species, active or inactive.
    Returns (chi_abs, chi_h2, chi_he, mu_kg, valid).
    """
    chi = 10.0 ** np.asarray(log10_vmr)
    S = np.sum(chi)
    chi_h2 = (1.0 - S) / (1.0 + he_h2)
    chi_he = he_h2 * chi_h2
    mu_amu = np.sum(chi * np.asarray(abs_mass)) + chi_h2 * h2_mass + chi_he * he_mass
    valid = bool(np.real(S) < 1.0)
    return chi, chi_h2, chi_he, mu_amu * amu, valid


def two_layer_vmr(log10_surface, log10_top, p_switch, P):
    """Reading A26: chi[l, i] = 10**log10_surface[i] at the layers with
    P_l >= p_switch[i], 10**log10_top[i] above."""
    deep = np.asarray(P)[:, None] >= np.asarray(p_switch, dtype=np.float64)[None, :]
    return np.where(deep, 10.0 ** np.asarray(log10_surface)[None, :],
                    10.0 ** np.asarray(log10_top)[None, :])


def chemistry_profile(chi, he_h2, abs_mass, h2_mass, he_mass, amu):
    """The chemistry of ``chemistry`` layer by layer for absorber profiles
    chi[l, i]: per-layer fill gases and mean molecular weight.  Returns
    (chi, chi_h2[N], chi_he[N], mu_kg[N], valid), valid when every layer's
    absorbers sum below 1."""
    S = np.sum(chi, axis=1)
    chi_h2 = (1.0 - S) / (1.0 + he_h2)
    chi_he = he_h2 * chi_h2
    mu_amu = chi @ np.asarray(abs_mass, dtype=np.float64) + chi_h2 * h2_mass + chi_he * he_mass
    valid = bool(np.all(np.real(S) < 1.0))
    return chi, chi_h2, chi_he, mu_amu * amu, valid


def model_chemistry(m, tables, P):
    """The chemistry of model dict m at layer centres P: constant profiles
    (log10_vmr) or, when m has log10_vmr_top and vmr_switch (Pa), the
    two-layer profiles of reading A26."""
    if m.get("log10_vmr_top") is not None:
        chi = two_layer_vmr(m["log10_vmr"], m["log10_vmr_top"], m["vmr_switch"], P)
        return chemistry_profile(chi, m["he_h2"], tables.abs_mass, tables.h2_mass, tables.he_mass,
                                 m["amu"])
    return chemistry(m["log10_vmr"], m["he_h2"], tables.abs_mass, tables.h2_mass, tables.he_mass,
                     m["amu"])


def altitude(T, P, mu_kg, Rp, GM, k_B, gravity=0):
    """Forward Models section, altitude equation.

    z_0 = 0 (bottom of the atmosphere, where Rp is defined); for l >= 1,
    z_l = z_{l-1} - H_{l-1} ln(P_l / P_{l-1}) with H = k_B T / (mu g).
    Reading A4: g_{l-1} = GM / (Rp + z_{l-1})^2 (gravity=0) or GM/Rp^2.
    Reading A5: the lower layer's H is used for each step (mu_kg a scalar
    or per layer, reading A26).
    """
    N = len(T)
    z = np.zeros(N, dtype=np.result_type(T, Rp, mu_kg, 0.0))
    mu = np.broadcast_to(np.asarray(mu_kg), (N,))
    for l in range(1, N):
        if gravity == 0:
            g = GM / (Rp + z[l - 1]) ** 2
        else:
            g = GM / Rp ** 2
        H = k_B * T[l - 1] / (mu[l - 1] * g)
        z[l] = z[l - 1] - H * np.log(P[l] / P[l - 1])
    return z


def number_density(P, T, k_B):
    """Reading A7: ideal-gas number density rho = P / (k_B T) (m^-3)."""
    return P / (k_B * T)


# --------------------------------------------------------------------------
# Geometry (reading A9)
# --------------------------------------------------------------------------
def shell_boundaries(z):
    """Shell boundaries h_0 = 0, h_k = (z_{k-1} + z_k)/2, h_N = z_{N-1}."""
    N = len(z)
    h = np.zeros(N + 1, dtype=z.dtype)
    h[1:N] = 0.5 * (z[:-1] + z[1:])
    h[N] = z[N - 1]
    return h


def chord_lengths(z, Rp):
    """Path length dl[j, k] of ray j (impact parameter b_j = Rp + z_j)
    through shell k (radii Rp + h_k .. Rp + h_{k+1}), for k >= j:

        dl[j, k] = 2 [ sqrt(r_{k+1}^2 - b^2) - sqrt(max(r_k, b)^2 - b^2) ].

    r^2 - b^2 is formed as (h - z_j)(2 Rp + h + z_j) so that no large radii
    are squared and subtracted.  Entries with k < j are zero.
    """
    N = len(z)
    h = shell_boundaries(z)
    dl = np.zeros((N, N), dtype=np.result_type(z, Rp))
    for j in range(N):
        def q(hk):
            return np.sqrt((hk - z[j]) * (2.0 * Rp + hk + z[j]))
        for k in range(j, N):
            outer = q(h[k + 1])                   # zero for the top ray: h_N = z_{N-1}
            inner = 0.0 if k == j else q(h[k])    # max(r_k, b_j) = b_j at k == j
            dl[j, k] = 2.0 * (outer - inner)
    return dl


def annulus_weights(z, Rp):
    """Reading A9: a = 2 int (Rp + z)(1 - e^-tau) dz evaluated on the nodes
    z_j with cell widths h_{j+1} - h_j (the trapezoid rule on a uniform
    grid): A_j = 2 (Rp + z_j)(h_{j+1} - h_j)."""
    h = shell_boundaries(z)
    return 2.0 * (Rp + z) * (h[1:] - h[:-1])


# --------------------------------------------------------------------------
# Opacity (Opacities section; equations opt_dpth, cia_opt_dpth, contrib)
# --------------------------------------------------------------------------
def bracket(grid, x):
    """Lower-closed bracket of x on an increasing grid with edge clamping.

    Returns (i, x_used, below, above): grid[i] <= x_used <= grid[i+1];
    x_used is x itself inside the grid and the nearest edge outside it
    (Opacities section: values outside the range are fixed to the minimum or
    maximum).  x == grid[-1] uses the last interval.  Uses Re(x) only.
    """
    xr = float(np.real(x))
    n = len(grid)
    if xr < grid[0]:
        return 0, grid[0], True, False
    if xr >= grid[n - 1]:
        return n - 2, grid[n - 1], False, xr > grid[n - 1]
    i = int(np.searchsorted(grid, xr, side="right")) - 1
    return i, x, False, False


def interp_xsec(table, T_grid, log10P_grid, T, log10P, p_interp="log",
                zero_rule="both", t_interp="linear"):
    """Opacities section, linear scheme: sigma(T) = sigma(T1) + m (T - T1)
    with m = (sigma(T2) - sigma(T1)) / (T2 - T1), then the same form along P
    (reading A1: along log10 P, or along P itself with p_interp="linear").
    t_interp="exp": the exponential scheme along T (reading A25),
    sigma(T) = a e^{-b/T}, b = (1/T2 - 1/T1)^{-1} ln(sigma(T1)/sigma(T2)),
    a = sigma(T1) e^{b/T1}.

    table: [nT, nP, W].  Out-of-range rules (reading A3): T and P clamp to
    the grid edges; T below AND P below the grid gives zero.
    """
    iT, Tu, T_lo, _ = bracket(T_grid, T)
    iP, xu, P_lo, _ = bracket(log10P_grid, log10P)
    if zero_rule == "both" and T_lo and P_lo:
        return np.zeros(table.shape[-1])
    if zero_rule == "p_only" and P_lo:
        return np.zeros(table.shape[-1])
    T1, T2 = T_grid[iT], T_grid[iT + 1]

    def along_T(j):
        s1, s2 = table[iT, j], table[iT + 1, j]
        m = (s2 - s1) / (T2 - T1)
        lin = s1 + m * (Tu - T1)
        if t_interp == "linear":
            return lin
        ok = (s1 > 0) & (s2 > 0)
        r1 = np.where(ok, s1, 1.0)
        r2 = np.where(ok, s2, 1.0)
        b = np.log(r1 / r2) / (1.0 / T2 - 1.0 / T1)
        a = r1 * np.exp(b / T1)
        return np.where(ok, a * np.exp(-b / Tu), lin)

    s_p1, s_p2 = along_T(iP), along_T(iP + 1)
    if p_interp == "log":
        x1, x2, x = log10P_grid[iP], log10P_grid[iP + 1], xu
    else:
        x1, x2 = 10.0 ** log10P_grid[iP], 10.0 ** log10P_grid[iP + 1]
        x = 10.0 ** xu
    m = (s_p2 - s_p1) / (x2 - x1)
    return s_p1 + m * (x - x1)


def interp_cia(table, T_grid, T):
    """CIA cross-section at temperature T: linear in T between the
    bracketing nodes, clamped to the grid edges.  table: [nTc, W]."""
    iT, Tu, _, _ = bracket(T_grid, T)
    T1, T2 = T_grid[iT], T_grid[iT + 1]
    s1, s2 = table[iT], table[iT + 1]
    return s1 + (s2 - s1) / (T2 - T1) * (Tu - T1)


def opacity(T, P, chi_abs, chi_h2, chi_he, tables, k_B, lo, hi,
            p_interp="log", zero_rule="both", t_interp="linear"):
    """Absorption coefficient kappa[l, w] (m^-1) of each layer over the
    window [lo, hi): the integrands of equations opt_dpth (absorption),
    cia_opt_dpth (CIA) and contrib (Rayleigh with w = chi), summed over
    contributions before the path integral:

        kappa = 1e-4 rho [sum_i chi_i sigma_i(T,P) + sum_s chi_s sigma_R,s]
              + 1e-10 rho^2 sum_pairs chi_a chi_b sigma_ab(T).

    chi_abs is [n_abs] (constant profiles) or [N, n_abs] with chi_h2 and
    chi_he per layer (reading A26).
    """
    N = len(T)
    n = number_density(P, T, k_B)
    per_layer = np.ndim(chi_abs) == 2
    W = hi - lo
    kappa = np.zeros((N, W), dtype=np.result_type(T, chi_abs, 0.0))
    lp = np.log10(P)
    chi_all = chi_abs
    for l in range(N):
        if per_layer:
            chi_abs = chi_all[l]
            chi_s = list(chi_abs) + [chi_h2[l], chi_he[l]]
        else:
            chi_s = list(chi_abs) + [chi_h2, chi_he]
        acc = np.zeros(W, dtype=kappa.dtype)
        for i in range(tables.n_abs):
            acc = acc + chi_abs[i] * interp_xsec(tables.xsec[i][:, :, lo:hi],
                                                 tables.T_grid, tables.log10P_grid,
                                                 T[l], lp[l], p_interp, zero_rule, t_interp)
        if tables.rayleigh is not None:
            for s in range(tables.n_abs + 2):
                acc = acc + chi_s[s] * tables.rayleigh[s, lo:hi]
        k_l = CM2_TO_M2 * n[l] * acc
        for p in range(tables.cia.shape[0]):
            a, b = tables.cia_pair[p]
            k_l = k_l + CM5_TO_M5 * n[l] ** 2 * chi_s[a] * chi_s[b] * interp_cia(
                tables.cia[p][:, lo:hi], tables.Tcia_grid, T[l])
        kappa[l] = k_l
    return kappa


def cloud_opacity(P, T, k_B, sigma, p_top, p_bottom):
    """Equation clouds: a flat (wavenumber-independent) cross-section sigma
    (m^2) on the layers inside the deck and zero outside, entering the path
    integral with the number density like absorption (w = 1), so the deck
    adds kappa_c[l] = sigma rho_l (m^-1).  Reading A24: the deck is
    discretised on the layer-centre pressures and takes the layers with
    min(p_top, p_bottom) <= P_l <= max(p_top, p_bottom) (the equation and
    the text name the two bounds in opposite orders).  sigma = +inf is the
    fully opaque deck of the Retrievals section.
    """
    lo_p, hi_p = min(p_top, p_bottom), max(p_top, p_bottom)
    deck = (np.real(P) >= lo_p) & (np.real(P) <= hi_p)
    if np.isinf(sigma):
        return np.where(deck, np.inf, 0.0), deck
    n = number_density(P, T, k_B)
    return np.where(deck, sigma * n, 0.0 * n), deck


def cloud_optical_depth(dl, kappa_c, deck, sigma):
    """The deck's own line-of-sight integral per ray, tau_c[j] =
    sum_{k >= j} dl[j, k] kappa_c[k] (equation tot_opt_dpth sums the
    contributions' integrals).  For sigma = +inf this is the limit: +inf
    for a ray with a nonzero path through the deck, zero otherwise."""
    if np.isinf(sigma):
        col = np.real(dl) @ deck.astype(np.float64)
        return np.where(col > 0.0, np.inf, 0.0)
    return dl @ kappa_c


def optical_depth(dl, kappa):
    """tau[j, w] = sum_{k >= j} dl[j, k] kappa[k, w]: the line-of-sight
    integral of equation opt_dpth for the ray at altitude z_j, with each
    shell carrying its layer's opacity (reading A10)."""
    return dl @ kappa


def transit_depth(tau, A, Rp, Rs):
    """Forward Models section: D = (Rp^2 + a)/Rs^2 with
    a = sum_j A_j (1 - exp(-tau_j)), 1 - exp(-tau) taken as -expm1(-tau)."""
    a = np.sum(A[:, None] * (-np.expm1(-tau)), axis=0)
    return (Rp ** 2 + a) / Rs ** 2


# --------------------------------------------------------------------------
# Binning subsection
# --------------------------------------------------------------------------
def native_bin_edges(wn):
    """Reading A13: native bin edges at midpoints, end bins mirrored."""
    wn = np.asarray(wn, dtype=np.float64)
    mid = 0.5 * (wn[:-1] + wn[1:])
    lo = np.concatenate([[wn[0] - (mid[0] - wn[0])], mid])
    hi = np.concatenate([mid, [wn[-1] + (wn[-1] - mid[-1])]])
    return lo, hi


def bin_weights(wn, ch_lo, ch_hi, lo, hi):
    """Binning subsection overlap weights w[c, i] for native points i in the
    window [lo, hi): (min(c+, i+) - max(c-, i-)) / (i+ - i-), zero when the
    bins do not overlap (reading A12)."""
    e_lo, e_hi = native_bin_edges(wn)
    e_lo, e_hi = e_lo[lo:hi], e_hi[lo:hi]
    ov = (np.minimum(np.asarray(ch_hi)[:, None], e_hi[None, :])
          - np.maximum(np.asarray(ch_lo)[:, None], e_lo[None, :]))
    return np.maximum(ov, 0.0) / (e_hi - e_lo)[None, :]


def bin_spectrum(D, w):
    """F_c = sum_i F_i w_ci / sum_i w_ci; NaN for a channel with no
    overlap (reading A12)."""
    s = np.sum(w, axis=1)
    num = w @ D
    out = np.full(w.shape[0], np.nan, dtype=np.result_type(D, 0.0))
    ok = s > 0
    out[ok] = num[ok] / s[ok]
    return out


# --------------------------------------------------------------------------
# Whole model
# --------------------------------------------------------------------------
def forward_model(m, tables, channels=None, p_interp="log", zero_rule="both",
                  keep=False):
    """One model: dict ``m`` with T (per layer, bottom first), p_bot, p_top,
    log10_vmr, Rp, Rs, GM, wn_lo, wn_hi, he_h2, k_B, amu, gravity, and
    optionally a cloud deck: cloud_sigma (m^2, +inf for opaque; absent or 0
    for none), cloud_p_top, cloud_p_bottom (Pa); optionally t_interp
    ("linear", the default, or "exp": reading A25); optionally two-layer
    profiles: log10_vmr_top and vmr_switch (Pa) per absorber (reading A26).

    Returns a dict with the native depth over the window (``depth``), the
    binned depth (``binned``, if channels are given) and ``valid``.  With
    keep=True the intermediates (z, dl, A, kappa, tau) are returned too.
    """
    T = m["T"]
    N = len(T)
    lo, hi = m["wn_lo"], m["wn_hi"]
    _, P = pressure_grid(m["p_bot"], m["p_top"], N)
    chi, chi_h2, chi_he, mu, valid = model_chemistry(m, tables, P)
    z = altitude(T, P, mu, m["Rp"], m["GM"], m["k_B"], m["gravity"])
    dl = chord_lengths(z, m["Rp"])
    A = annulus_weights(z, m["Rp"])
    kappa = opacity(T, P, chi, chi_h2, chi_he, tables, m["k_B"], lo, hi,
                    p_interp, zero_rule, m.get("t_interp", "linear"))
    tau = optical_depth(dl, kappa)
    sigma_c = m.get("cloud_sigma", 0.0)
    if sigma_c != 0.0:
        kappa_c, deck = cloud_opacity(P, T, m["k_B"], sigma_c, m["cloud_p_top"],
                                      m["cloud_p_bottom"])
        tau_c = cloud_optical_depth(dl, kappa_c, deck, sigma_c)
        tau = tau + tau_c[:, None]
    else:
        kappa_c = tau_c = None
    D = transit_depth(tau, A, m["Rp"], m["Rs"])
    out = {"depth": D, "valid": valid}
    if channels is not None:
        w = bin_weights(tables.wn, channels.lo, channels.hi, lo, hi)
        out["binned"] = bin_spectrum(D, w)
    if keep:
        out.update(z=z, dl=dl, A=A, kappa=kappa, tau=tau, P=P, mu=mu,
                   chi=chi, chi_h2=chi_h2, chi_he=chi_he, kappa_c=kappa_c,
                   tau_c=tau_c)
    return out


def forward_batch(tables, batch, channels=None, models=None):
    """Run forward_model over (a subset of) a synth.Batch."""
    idx = range(batch.B) if models is None else models
    return [forward_model(batch.model(b), tables, channels) for b in idx]


def chi2(binned, obs, sigma):
    """Reading A14: chi^2 = sum_c ((D_c - O_c) / sigma_c)^2."""
    r = (binned - obs) / sigma
    return np.sum(r * r)
