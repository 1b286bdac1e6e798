"""The five benchmark workloads as seeded synthetic inputs.

Each workload mirrors one benchmark configuration of this project (plain
FP64 single model; single FP32 model; batched live-point set; adjoint batch;
large batched forward + gradient).  Shapes follow the paper's own workloads:
100-layer atmospheres between 1e6 and 1e-4 Pa, H2/He fill with He/H2 = 0.17,
1 R_Jup planet around a 1 R_Sun star, cross-section grids of ~20-40
temperatures x 20-30 pressures, and R ~ 10^4 wavenumber grids over
0.3-15 um (Benchmark section).

Random streams: ``SeedSequence(config_index).spawn(4)`` gives independent
generators for tables, parameters, windows and noise.

``make_config(i, **shrink)`` accepts overrides (fewer wavenumbers, lines,
models, ...) so tests can build the same recipe at sizes a CPU finishes in
seconds.
"""

from dataclasses import dataclass, field, replace
from functools import lru_cache

import numpy as np

from .constants import (ABSORBERS, AMU_KG, GM_JUP, HE_H2_RATIO, K_BOLTZMANN,
                        MASSES_AMU, R_JUP, R_SUN)
from .atmosphere import (avoid_nodes, guillot_T, log_midpoint_pressures,
                         log_uniform_channels, smooth_perturbation)
from .opacity_tables import (cia_table, line_forest, rayleigh_table,
                             replicate_forest, wn_grid_linear,
                             wn_grid_log_wavelength)

CONFIG_NAMES = {
    1: "plain-fp64-1abs-100L-2000wn",
    2: "single-fp32-5abs-100L-40000wn-50ch",
    3: "batched-4096-ragged-50to200L-5to40kwn",
    4: "adjoint-256-100L-7abs-50000wn-100ch",
    5: "batched-grad-1024-100to200L-10abs-100000wn",
}


@dataclass
class Tables:
    """Opacity inputs on one shared wavenumber grid (all float64, host)."""
    wn: np.ndarray                 # [W] cm^-1, increasing
    T_grid: np.ndarray             # [nT] K, increasing
    log10P_grid: np.ndarray        # [nP] log10(Pa), increasing
    xsec: np.ndarray               # [n_abs, nT, nP, W] cm^2
    abs_mass: np.ndarray           # [n_abs] amu
    h2_mass: float
    he_mass: float
    Tcia_grid: np.ndarray          # [nTc] K
    cia: np.ndarray                # [n_cia, nTc, W] cm^5 (n_cia may be 0)
    cia_pair: np.ndarray           # [n_cia, 2] int32 species ids
    rayleigh: object               # [n_abs + 2, W] cm^2 or None
    names: list = field(default_factory=list)

    @property
    def n_abs(self):
        return self.xsec.shape[0]

    @property
    def n_wn(self):
        return self.wn.shape[0]

    def as_float32_rounded(self):
        """The same tables after rounding every value to float32 and back
        (what a float32-storage device path actually reads)."""
        f = lambda a: None if a is None else a.astype(np.float32).astype(np.float64)
        return Tables(self.wn, self.T_grid, self.log10P_grid, f(self.xsec),
                      self.abs_mass, self.h2_mass, self.he_mass, self.Tcia_grid,
                      f(self.cia), self.cia_pair, f(self.rayleigh), list(self.names))


@dataclass
class Batch:
    """B models, ragged in layers; host numpy arrays."""
    n_layers: np.ndarray           # [B] int32
    layer_off: np.ndarray          # [B+1] int64
    T: np.ndarray                  # [layer_off[-1]] K, bottom first
    p_bot: np.ndarray              # [B] Pa
    p_top: np.ndarray              # [B] Pa
    log10_vmr: np.ndarray          # [B, n_abs]
    Rp: np.ndarray                 # [B] m
    Rs: np.ndarray                 # [B] m
    GM: np.ndarray                 # [B] m^3 s^-2
    wn_lo: np.ndarray              # [B] int32, window start (inclusive)
    wn_hi: np.ndarray              # [B] int32, window end (exclusive)
    he_h2: float = HE_H2_RATIO
    k_B: float = K_BOLTZMANN
    amu: float = AMU_KG
    gravity: int = 0               # 0: g = GM/(Rp+z)^2, 1: g = GM/Rp^2
    # optional flat-opacity cloud deck per model ([B] each, or None for no
    # decks): cross-section in m^2 (0: none, +inf: opaque) and the deck's
    # bounding pressures in Pa
    cloud_sigma: np.ndarray = None
    cloud_p_top: np.ndarray = None
    cloud_p_bottom: np.ndarray = None
    # optional two-layer profiles ([B, n_abs] each, or None): top values
    # (log10) and switch pressures (Pa); log10_vmr holds the surface values
    log10_vmr_top: np.ndarray = None
    vmr_switch: np.ndarray = None

    @property
    def B(self):
        return int(self.n_layers.shape[0])

    def T_of(self, b):
        return self.T[self.layer_off[b]:self.layer_off[b + 1]]

    def model(self, b):
        """Per-model view as a dict (the oracle's input form)."""
        d = dict(T=self.T_of(b).copy(), p_bot=float(self.p_bot[b]),
                    p_top=float(self.p_top[b]), log10_vmr=self.log10_vmr[b].copy(),
                    Rp=float(self.Rp[b]), Rs=float(self.Rs[b]), GM=float(self.GM[b]),
                    wn_lo=int(self.wn_lo[b]), wn_hi=int(self.wn_hi[b]),
                    he_h2=self.he_h2, k_B=self.k_B, amu=self.amu,
                    gravity=self.gravity)
        if self.cloud_sigma is not None:
            d.update(cloud_sigma=float(self.cloud_sigma[b]),
                     cloud_p_top=float(self.cloud_p_top[b]),
                     cloud_p_bottom=float(self.cloud_p_bottom[b]))
        if self.log10_vmr_top is not None:
            d.update(log10_vmr_top=self.log10_vmr_top[b].copy(), vmr_switch=self.vmr_switch[b].copy())
        return d

    def subset(self, idx):
        idx = np.asarray(idx)
        Ts = [self.T_of(int(b)) for b in idx]
        nl = np.array([len(t) for t in Ts], dtype=np.int32)
        off = np.zeros(len(idx) + 1, dtype=np.int64)
        off[1:] = np.cumsum(nl)
        return Batch(nl, off, np.concatenate(Ts) if Ts else np.zeros(0),
                     self.p_bot[idx].copy(), self.p_top[idx].copy(),
                     self.log10_vmr[idx].copy(), self.Rp[idx].copy(),
                     self.Rs[idx].copy(), self.GM[idx].copy(),
                     self.wn_lo[idx].copy(), self.wn_hi[idx].copy(),
                     self.he_h2, self.k_B, self.amu, self.gravity,
                     *(None if c is None else c[idx].copy()
                       for c in (self.cloud_sigma, self.cloud_p_top, self.cloud_p_bottom,
                                 self.log10_vmr_top, self.vmr_switch)))


def with_cloud_decks(batch, seed, kinds=("none", "flat", "opaque")):
    """A copy of ``batch`` with a cloud deck per model, model b of kind
    kinds[b % len(kinds)]: "none" (sigma 0), "flat" (a deck of 2-20 % of the
    atmosphere's log-pressure span at a random height, log10 sigma uniform in
    [-32, -27] m^2, so that its optical depth along a chord spans ~0.01-1e4),
    "opaque" (sigma +inf from a cloud-top pressure log-uniform over the
    upper 80 % of the span down to the bottom boundary: the fully opaque deck
    whose top pressure the paper's transit retrieval fits)."""
    rng = np.random.default_rng(seed)
    B = batch.B
    sig = np.zeros(B)
    pt = np.ones(B)
    pb = np.ones(B)
    for b in range(B):
        kind = kinds[b % len(kinds)]
        xb, xt = np.log10(batch.p_bot[b]), np.log10(batch.p_top[b])
        if kind == "flat":
            width = rng.uniform(0.02, 0.2) * (xb - xt)
            x1 = rng.uniform(xt, xb - width)
            pt[b], pb[b] = 10.0 ** x1, 10.0 ** (x1 + width)
            sig[b] = 10.0 ** rng.uniform(-32.0, -27.0)
        elif kind == "opaque":
            pt[b] = 10.0 ** rng.uniform(xt, xt + 0.8 * (xb - xt))
            pb[b] = batch.p_bot[b]
            sig[b] = np.inf
    out = batch.subset(np.arange(B))
    out.cloud_sigma, out.cloud_p_top, out.cloud_p_bottom = sig, pt, pb
    return out


@dataclass
class Channels:
    lo: np.ndarray                 # [C] cm^-1
    hi: np.ndarray                 # [C] cm^-1

    @property
    def n(self):
        return int(self.lo.shape[0])


def with_two_layer_profiles(batch, seed, n_switch=2, drop=(0.5, 4.0)):
    """A copy of ``batch`` whose absorbers have two-layer profiles: per
    model, n_switch switch pressures log-uniform in [1e-2, 1e5] Pa, each
    absorber on one of them or constant (equal top and surface values), its
    top value lower than its surface value by a drop in log10 uniform in
    ``drop``.  The layers then fall into at most n_switch + 1 runs."""
    rng = np.random.default_rng(seed)
    B, na = batch.log10_vmr.shape
    sw = 10.0 ** rng.uniform(-2.0, 5.0, (B, n_switch))
    pick = rng.integers(0, n_switch + 1, (B, na))       # n_switch: constant
    top = batch.log10_vmr - rng.uniform(drop[0], drop[1], (B, na))
    top = np.where(pick == n_switch, batch.log10_vmr, top)
    p_sw = np.take_along_axis(np.concatenate([sw, np.ones((B, 1))], axis=1), pick, axis=1)
    out = replace(batch)
    out.log10_vmr_top, out.vmr_switch = top, p_sw
    return out


def batch_from_models(T_list, p_bot, p_top, log10_vmr, Rp, Rs, GM, wn_lo, wn_hi,
                      gravity=0):
    nl = np.array([len(t) for t in T_list], dtype=np.int32)
    off = np.zeros(len(T_list) + 1, dtype=np.int64)
    off[1:] = np.cumsum(nl)
    B = len(T_list)
    bc = lambda v, dt=np.float64: np.broadcast_to(np.asarray(v, dtype=dt), (B,)).copy()
    return Batch(nl, off, np.concatenate([np.asarray(t, np.float64) for t in T_list]),
                 bc(p_bot), bc(p_top), np.asarray(log10_vmr, np.float64).reshape(B, -1).copy(),
                 bc(Rp), bc(Rs), bc(GM), bc(wn_lo, np.int32), bc(wn_hi, np.int32),
                 gravity=gravity)


def _streams(cfg_index):
    ss = np.random.SeedSequence(cfg_index)
    return [np.random.default_rng(s) for s in ss.spawn(4)]


@lru_cache(maxsize=8)
def _tables_cached(key):
    (kind, n_wn, nT, nP, T_lo, T_hi, n_abs, n_lines, with_cia, seed, wn_kind) = key
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(4)[0])
    if wn_kind == "linear":
        wn = wn_grid_linear(1000.0, 10000.0, n_wn)
    else:
        wn = wn_grid_log_wavelength(0.3, 15.0, n_wn)
    T_grid = np.linspace(T_lo, T_hi, nT)
    logP = np.linspace(-4.0, 6.0, nP)
    n_gen = min(n_abs, 5)
    forests = [line_forest(rng, wn, T_grid, logP, n_lines) for _ in range(n_gen)]
    for _ in range(n_abs - n_gen):
        forests.append(replicate_forest(rng, forests[len(forests) % n_gen]))
    xsec = np.stack(forests) if forests else np.zeros((0, nT, nP, n_wn))
    names = ABSORBERS[:n_abs]
    mass = np.array([MASSES_AMU[m] for m in names])
    if with_cia:
        cia = np.stack([cia_table(rng, wn, T_grid), cia_table(rng, wn, T_grid)])
        pair = np.array([[n_abs, n_abs], [n_abs, n_abs + 1]], dtype=np.int32)
        ray = rayleigh_table(rng, wn, n_abs)
    else:
        cia = np.zeros((0, nT, n_wn))
        pair = np.zeros((0, 2), dtype=np.int32)
        ray = None
    return Tables(wn, T_grid, logP, xsec, mass, MASSES_AMU["H2"], MASSES_AMU["He"],
                  T_grid.copy(), cia, pair, ray, names)


def make_tables(cfg_index, n_wn=None, n_lines=None, nT=None, nP=None):
    """Tables for a workload, optionally shrunk (fewer wavenumbers/lines)."""
    d = {1: dict(n_wn=2000, nT=20, nP=20, T=(300.0, 3000.0), n_abs=1, n_lines=200,
                 cia=False, wn="linear"),
         2: dict(n_wn=40000, nT=30, nP=22, T=(200.0, 3500.0), n_abs=5, n_lines=5000,
                 cia=True, wn="log"),
         4: dict(n_wn=50000, nT=30, nP=22, T=(200.0, 3500.0), n_abs=7, n_lines=5000,
                 cia=True, wn="log"),
         5: dict(n_wn=100000, nT=40, nP=30, T=(200.0, 3500.0), n_abs=10, n_lines=5000,
                 cia=True, wn="log")}
    base = {3: 2}.get(cfg_index, cfg_index)
    c = d[base]
    key = ("x", n_wn or c["n_wn"], nT or c["nT"], nP or c["nP"], c["T"][0], c["T"][1],
           c["n_abs"], n_lines or c["n_lines"], c["cia"], base, c["wn"])
    return _tables_cached(key)


def make_config(cfg_index, n_wn=None, n_lines=None, B=None, layer_range=None,
                nT=None, nP=None):
    """Build (tables, batch, channels-or-None) for workload ``cfg_index``.

    Overrides shrink the workload for tests; the defaults are the full
    benchmark sizes.
    """
    tables = make_tables(cfg_index, n_wn=n_wn, n_lines=n_lines, nT=nT, nP=nP)
    W = tables.n_wn
    _, r_par, r_win, _ = _streams(cfg_index)
    n_abs = tables.n_abs
    if cfg_index == 1:
        N = 100
        T = [np.full(N, 1500.0)]
        batch = batch_from_models(T, 1e6, 1e-4, np.full((1, 1), -4.0), R_JUP, R_SUN,
                                  GM_JUP, 0, W)
        return tables, batch, None
    if cfg_index == 2:
        N = 100
        g = GM_JUP / R_JUP ** 2
        T = guillot_T(log_midpoint_pressures(1e6, 1e-4, N), g, 1200.0)
        vmr = r_par.uniform(-8.0, -2.0, (1, n_abs))
        batch = batch_from_models([T], 1e6, 1e-4, vmr, R_JUP, R_SUN, GM_JUP, 0, W)
        lo, hi = log_uniform_channels(tables.wn, 50)
        return tables, batch, Channels(lo, hi)
    if cfg_index == 3:
        B = B or 4096
        lmin, lmax = layer_range or (50, 200)
        T_irr = r_par.uniform(500.0, 2500.0, B)
        vmr = r_par.uniform(-12.0, -1.0, (B, n_abs))
        Rp = r_par.uniform(0.5, 2.0, B) * R_JUP
        N = r_par.integers(lmin, lmax + 1, B)
        wmin = max(1, (W * 5000) // 40000)
        wlen = r_win.integers(wmin, W + 1, B)
        wlo = np.array([r_win.integers(0, W - L + 1) for L in wlen])
        Ts = [guillot_T(log_midpoint_pressures(1e6, 1e-4, int(N[b])),
                        GM_JUP / Rp[b] ** 2, T_irr[b]) for b in range(B)]
        batch = batch_from_models(Ts, 1e6, 1e-4, vmr, Rp, R_SUN, GM_JUP, wlo, wlo + wlen)
        lo, hi = log_uniform_channels(tables.wn, 50)
        return tables, batch, Channels(lo, hi)
    if cfg_index == 4:
        B = B or 256
        N = 100
        g = GM_JUP / R_JUP ** 2
        T0 = guillot_T(log_midpoint_pressures(1e6, 1e-4, N), g, 1200.0)
        T0 = T0 * (1.0 + 0.05 * smooth_perturbation(r_par, N))
        vmr0 = r_par.uniform(-8.0, -3.0, n_abs)
        Ts, vmr, Rp = [], [], []
        for b in range(B):
            if b == 0:
                Ts.append(avoid_nodes(T0, tables.T_grid))
                vmr.append(vmr0.copy())
                Rp.append(R_JUP)
            else:
                Ts.append(avoid_nodes(T0 + r_par.normal(0.0, 20.0, N), tables.T_grid))
                vmr.append(vmr0 + r_par.normal(0.0, 0.1, n_abs))
                Rp.append(R_JUP * (1.0 + 0.01 * r_par.normal()))
        batch = batch_from_models(Ts, 1e6, 1e-4, np.array(vmr), np.array(Rp), R_SUN,
                                  GM_JUP, 0, W)
        lo, hi = log_uniform_channels(tables.wn, 100)
        return tables, batch, Channels(lo, hi)
    if cfg_index == 5:
        B = B or 1024
        lmin, lmax = layer_range or (100, 200)
        T_irr = r_par.uniform(500.0, 2500.0, B)
        vmr = np.empty((B, n_abs))
        for b in range(B):
            while True:
                v = r_par.uniform(-12.0, -2.0, n_abs)
                if np.sum(10.0 ** v) < 1.0:
                    vmr[b] = v
                    break
        Rp = r_par.uniform(0.5, 2.0, B) * R_JUP
        N = r_par.integers(lmin, lmax + 1, B)
        Ts = [avoid_nodes(guillot_T(log_midpoint_pressures(1e6, 1e-4, int(N[b])),
                                    GM_JUP / Rp[b] ** 2, T_irr[b]), tables.T_grid)
              for b in range(B)]
        batch = batch_from_models(Ts, 1e6, 1e-4, vmr, Rp, R_SUN, GM_JUP, 0, W)
        lo, hi = log_uniform_channels(tables.wn, 100)
        return tables, batch, Channels(lo, hi)
    raise ValueError(f"unknown workload {cfg_index}")


def stellar_temperatures(B, seed=58):
    """Seeded blackbody temperatures of the stars of an emission batch,
    uniform in [4500, 6500] K (the paper's host stars are Sun-like)."""
    return np.random.default_rng(seed).uniform(4500.0, 6500.0, B)


def observation_noise(cfg_index, n_models, n_ch, sigma_ppm=50.0):
    """Seeded N(0, sigma^2) noise [n_models, n_ch] and the per-channel sigma
    for a workload's synthetic observation (50 ppm by default)."""
    r_noise = _streams(cfg_index)[3]
    s = sigma_ppm * 1e-6
    return r_noise.normal(0.0, s, (n_models, n_ch)), np.full(n_ch, s)
