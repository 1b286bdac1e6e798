"""Python binding of libtrx (ctypes): argument marshalling only.

Every step of the forward model and its gradient runs in the HIP library;
this module converts arrays to device tensors, fills the C structs of
``include/trx.h`` and calls the entry points of the same names.  PyTorch is
used for device memory and the current stream.  If ``libtrx.so`` has not
been built the import of the library fails loudly: there is no fallback.
"""

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrx.so")

FP64, FP32, BF16_SPLIT2, BF16_SPLIT3 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x2": BF16_SPLIT2, "bf16x3": BF16_SPLIT3}

MODEL_OK, BAD_CHEMISTRY, BAD_PROFILE, BAD_WINDOW, NONFINITE, GRAD_UNSUPPORTED, UNSUPPORTED = \
    0, 1, 2, 4, 8, 16, 32
PLAN_GRAPH, PLAN_PERSISTENT, PLAN_GRAD, PLAN_EMISSION, PLAN_TWO_LAYER = 1, 2, 4, 8, 16

STATUS_NAMES = {0: "TRX_OK", 1: "TRX_E_INVALID_ARG", 2: "TRX_E_OUT_OF_MEMORY",
                3: "TRX_E_DEVICE", 4: "TRX_E_UNSUPPORTED"}

EXPORTS = ["trx_create", "trx_destroy", "trx_last_error", "trx_set_stream",
           "trx_synchronize", "trx_tables_create", "trx_tables_destroy",
           "trx_bins_create", "trx_bins_destroy", "trx_forward", "trx_forward_noalloc",
           "trx_emission", "trx_plan_set_star", "trx_chi2_grad",
           "trx_plan_create", "trx_plan_destroy", "trx_plan_batch", "trx_plan_launch",
           "trx_autotune", "trx_plan_set_variant", "trx_plan_describe", "trx_profile",
           "trx_profile_read"]

KERNEL_GEOMETRY, KERNEL_FORWARD, KERNEL_BINNING, KERNEL_ADJOINT, KERNEL_GEOM_ADJ, \
    KERNEL_SCHEDULE = range(6)

_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double


class TrxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class TablesDesc(ctypes.Structure):
    _fields_ = [("n_wn", _I), ("wn_cm1", _P), ("n_T", _I), ("T_K", _P),
                ("n_P", _I), ("log10P_Pa", _P), ("n_abs", _I), ("xsec_cm2", _P),
                ("abs_mass_amu", _P), ("h2_mass_amu", _D), ("he_mass_amu", _D),
                ("n_cia", _I), ("n_Tcia", _I), ("Tcia_K", _P), ("cia_cm5", _P),
                ("cia_pair", _P), ("rayleigh_cm2", _P), ("t_interp", _I)]


class BatchC(ctypes.Structure):
    _fields_ = [("B", _I), ("max_layers", _I), ("n_layers", _P), ("layer_off", _P),
                ("T_K", _P), ("p_bot_Pa", _P), ("p_top_Pa", _P), ("log10_vmr", _P),
                ("Rp_m", _P), ("Rs_m", _P), ("GM_m3s2", _P), ("wn_lo", _P),
                ("wn_hi", _P), ("he_h2_ratio", _D), ("k_B", _D), ("amu_kg", _D),
                ("gravity", _I), ("cloud_sigma_m2", _P), ("cloud_p_top_Pa", _P),
                ("cloud_p_bottom_Pa", _P), ("log10_vmr_top", _P), ("vmr_switch_Pa", _P)]


_lib = None


def lib():
    """The loaded libtrx (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1912_07759_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name in EXPORTS:
            getattr(L, name).restype = ctypes.c_int
        L.trx_last_error.restype = ctypes.c_char_p
        L.trx_plan_describe.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _hptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Context:
    """A libtrx context on one HIP device; calls use torch's current stream."""

    def __init__(self, device=0):
        self.device = device
        h = ctypes.c_void_p()
        rc = lib().trx_create(int(device), ctypes.byref(h))
        if rc != 0:
            raise TrxError(rc, "trx_create failed")
        self.h = h

    def check(self, rc):
        if rc != 0:
            raise TrxError(rc, lib().trx_last_error(self.h).decode())

    def bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.check(lib().trx_set_stream(self.h, ctypes.c_void_p(s)))

    def synchronize(self):
        self.check(lib().trx_synchronize(self.h))

    def profile(self, enable=True):
        self.check(lib().trx_profile(self.h, int(bool(enable))))

    def profile_read(self, kernel):
        """(total GPU ms, launches) of one kernel class since profile(True)."""
        ms = ctypes.c_double()
        n = ctypes.c_int32()
        self.check(lib().trx_profile_read(self.h, int(kernel), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def last_error(self):
        return lib().trx_last_error(self.h).decode()

    def close(self):
        if self.h:
            lib().trx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


T_INTERP = {"linear": 0, "exp": 1}


class Tables:
    """Device copy of opacity tables (host float64 arrays in).  t_interp:
    "linear" or "exp", the cross-sections' scheme in temperature."""

    def __init__(self, ctx, wn, T_grid, log10P_grid, xsec, abs_mass, h2_mass, he_mass,
                 Tcia_grid=None, cia=None, cia_pair=None, rayleigh=None, t_interp="linear"):
        self.ctx = ctx
        c = lambda a, dt=np.float64: None if a is None else np.ascontiguousarray(a, dtype=dt)
        self._keep = [c(wn), c(T_grid), c(log10P_grid), c(xsec), c(abs_mass),
                      c(Tcia_grid), c(cia), c(cia_pair, np.int32), c(rayleigh)]
        wn, T_grid, log10P_grid, xsec, abs_mass, Tcia_grid, cia, cia_pair, rayleigh = self._keep
        n_cia = 0 if cia is None else int(cia.shape[0])
        d = TablesDesc(len(wn), _hptr(wn), len(T_grid), _hptr(T_grid), len(log10P_grid),
                       _hptr(log10P_grid), int(xsec.shape[0]), _hptr(xsec), _hptr(abs_mass),
                       float(h2_mass), float(he_mass), n_cia,
                       0 if Tcia_grid is None else len(Tcia_grid), _hptr(Tcia_grid),
                       _hptr(cia) if n_cia else None, _hptr(cia_pair) if n_cia else None,
                       _hptr(rayleigh), T_INTERP[t_interp])
        h = ctypes.c_void_p()
        ctx.check(lib().trx_tables_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.n_wn = len(wn)
        self.n_abs = int(xsec.shape[0])
        self.t_interp = t_interp
        self._keep = None

    @classmethod
    def from_synth(cls, ctx, t, t_interp="linear"):
        return cls(ctx, t.wn, t.T_grid, t.log10P_grid, t.xsec, t.abs_mass, t.h2_mass,
                   t.he_mass, t.Tcia_grid if t.cia.shape[0] else None,
                   t.cia if t.cia.shape[0] else None,
                   t.cia_pair if t.cia.shape[0] else None, t.rayleigh, t_interp)

    def close(self):
        if self.h:
            lib().trx_tables_destroy(self.h)
            self.h = None


class Bins:
    """Channels [lo, hi) in cm^-1 for a set of tables."""

    def __init__(self, ctx, tables, lo, hi):
        self.ctx = ctx
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        h = ctypes.c_void_p()
        ctx.check(lib().trx_bins_create(ctx.h, tables.h, int(len(lo)), _hptr(lo), _hptr(hi),
                                        ctypes.byref(h)))
        self.h = h
        self.n = len(lo)

    def close(self):
        if self.h:
            lib().trx_bins_destroy(self.h)
            self.h = None


class DeviceBatch:
    """B models on the device.  Arrays may be numpy or torch; they are copied
    to ``device`` with the dtypes of ``include/trx.h``."""

    def __init__(self, n_layers, T, p_bot, p_top, log10_vmr, Rp, Rs, GM, wn_lo, wn_hi,
                 he_h2=0.17, k_B=1.380649e-23, amu=1.66053906660e-27, gravity=0,
                 device="cuda", max_layers=None, cloud_sigma=None, cloud_p_top=None,
                 cloud_p_bottom=None, log10_vmr_top=None, vmr_switch=None):
        dev = torch.device(device)
        t = lambda a, dt: torch.as_tensor(np.asarray(a) if not torch.is_tensor(a) else a,
                                          dtype=dt).to(dev).contiguous()
        self.n_layers = t(n_layers, torch.int32)
        nl = self.n_layers.to("cpu").to(torch.int64)
        off = torch.zeros(nl.numel() + 1, dtype=torch.int64)
        off[1:] = torch.cumsum(nl, 0)
        self.layer_off = off.to(dev)
        self.T = t(T, torch.float64)
        self.p_bot, self.p_top = t(p_bot, torch.float64), t(p_top, torch.float64)
        self.log10_vmr = t(log10_vmr, torch.float64)
        self.Rp, self.Rs, self.GM = t(Rp, torch.float64), t(Rs, torch.float64), t(GM, torch.float64)
        self.wn_lo, self.wn_hi = t(wn_lo, torch.int32), t(wn_hi, torch.int32)
        self.he_h2, self.k_B, self.amu, self.gravity = he_h2, k_B, amu, gravity
        self.B = int(self.n_layers.numel())
        # optional cloud decks: all three per-model arrays, or none
        if (cloud_sigma is None) != (cloud_p_top is None) or (cloud_sigma is None) != (cloud_p_bottom is None):
            raise ValueError("cloud deck arrays: all three or none")
        self.cloud = None if cloud_sigma is None else tuple(
            t(v, torch.float64) for v in (cloud_sigma, cloud_p_top, cloud_p_bottom))
        # optional two-layer profiles: top values and switch pressures, or none
        if (log10_vmr_top is None) != (vmr_switch is None):
            raise ValueError("two-layer arrays: both or neither")
        self.two_layer = None if log10_vmr_top is None else (
            t(log10_vmr_top, torch.float64), t(vmr_switch, torch.float64))
        self.max_layers = int(max_layers if max_layers is not None else max(2, int(nl.max())))

    @classmethod
    def from_synth(cls, b, device="cuda", max_layers=None):
        return cls(b.n_layers, b.T, b.p_bot, b.p_top, b.log10_vmr, b.Rp, b.Rs, b.GM,
                   b.wn_lo, b.wn_hi, b.he_h2, b.k_B, b.amu, b.gravity, device, max_layers,
                   getattr(b, "cloud_sigma", None), getattr(b, "cloud_p_top", None),
                   getattr(b, "cloud_p_bottom", None), getattr(b, "log10_vmr_top", None),
                   getattr(b, "vmr_switch", None))

    @property
    def n_abs(self):
        return int(self.log10_vmr.shape[1]) if self.log10_vmr.dim() == 2 else 0

    def view(self, b):
        """Model b alone, sharing this batch's device arrays."""
        return _ModelView(self, b)

    def cstruct(self, B=None):
        return BatchC(self.B if B is None else B, self.max_layers, _ptr(self.n_layers),
                      _ptr(self.layer_off), _ptr(self.T), _ptr(self.p_bot), _ptr(self.p_top),
                      _ptr(self.log10_vmr), _ptr(self.Rp), _ptr(self.Rs), _ptr(self.GM),
                      _ptr(self.wn_lo), _ptr(self.wn_hi), float(self.he_h2), float(self.k_B),
                      float(self.amu), int(self.gravity),
                      *((None, None, None) if self.cloud is None else (_ptr(c) for c in self.cloud)),
                      *((None, None) if self.two_layer is None else (_ptr(c) for c in self.two_layer)))


class _ModelView:
    """Model b of a DeviceBatch as a batch of one (pointer offsets into the
    parent's device arrays; layer offsets stay absolute)."""

    def __init__(self, db, b):
        self.db, self.b, self.B = db, int(b), 1

    def cstruct(self):
        d, b = self.db, self.b
        at = lambda t, k: ctypes.c_void_p(t.data_ptr() + k * t.element_size())
        return BatchC(1, d.max_layers, at(d.n_layers, b), at(d.layer_off, b), _ptr(d.T),
                      at(d.p_bot, b), at(d.p_top, b), at(d.log10_vmr, b * d.n_abs),
                      at(d.Rp, b), at(d.Rs, b), at(d.GM, b), at(d.wn_lo, b), at(d.wn_hi, b),
                      float(d.he_h2), float(d.k_B), float(d.amu), int(d.gravity),
                      *((None, None, None) if d.cloud is None else (at(c, b) for c in d.cloud)),
                      *((None, None) if d.two_layer is None else (at(c, b * d.n_abs) for c in d.two_layer)))


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def forward(ctx, tables, batch, bins=None, precision=FP64, native=True, binned=True,
            out_native=None, out_binned=None, out_status=None, out_tau=None):
    """trx_forward.  Returns (depth_native [B, n_wn] or None,
    depth_binned [B, n_ch] or None, model_status [B]).  With out_tau (a
    float64 device tensor [B, max_layers, n_wn]) the optical depth of every
    ray j < N inside each model's window is written there as well."""
    dev = batch.T.device
    B = batch.B
    if native and out_native is None:
        out_native = torch.full((B, tables.n_wn), float("nan"), dtype=torch.float64, device=dev)
    if not native:
        out_native = None
    if binned and bins is not None and out_binned is None:
        out_binned = torch.empty((B, bins.n), dtype=torch.float64, device=dev)
    if bins is None or not binned:
        out_binned = None
    if out_status is None:
        out_status = torch.empty(B, dtype=torch.int32, device=dev)
    ctx.bind_stream()
    bc = batch.cstruct()
    ctx.check(lib().trx_forward(ctx.h, tables.h, ctypes.byref(bc),
                                bins.h if bins is not None else None, _prec(precision),
                                _ptr(out_native), _ptr(out_binned), _ptr(out_status),
                                _ptr(out_tau)))
    return out_native, out_binned, out_status


def emission(ctx, tables, batch, bins=None, precision=FP64, n_mu=4, T_star=5800.0, native=True,
             binned=True):
    """trx_emission.  T_star: a scalar or [B] stellar temperatures.  Returns
    (fpfs_native [B, n_wn] or None, fpfs_binned [B, n_ch] or None,
    model_status [B])."""
    dev = batch.T.device
    B = batch.B
    ts = torch.as_tensor(np.broadcast_to(np.asarray(T_star, dtype=np.float64), (B,)).copy()
                         if not torch.is_tensor(T_star) else T_star, dtype=torch.float64).to(dev)
    out_native = torch.full((B, tables.n_wn), float("nan"), dtype=torch.float64, device=dev) \
        if native else None
    out_binned = torch.empty((B, bins.n), dtype=torch.float64, device=dev) \
        if (binned and bins is not None) else None
    out_status = torch.empty(B, dtype=torch.int32, device=dev)
    ctx.bind_stream()
    bc = batch.cstruct()
    ctx.check(lib().trx_emission(ctx.h, tables.h, ctypes.byref(bc),
                                 bins.h if bins is not None else None, _prec(precision), int(n_mu),
                                 _ptr(ts), _ptr(out_native), _ptr(out_binned), _ptr(out_status)))
    ctx._keep_star = ts
    return out_native, out_binned, out_status


def forward_noalloc(ctx, tables, batch, bins, precision, out_native, out_binned, out_status):
    """trx_forward_noalloc: the forward model in the library's fixed device
    array (no device memory is allocated by the library).  The outputs are
    caller tensors as for trx_forward (out_native / out_binned may be None);
    returns them."""
    ctx.bind_stream()
    bc = batch.cstruct()
    ctx.check(lib().trx_forward_noalloc(ctx.h, tables.h, ctypes.byref(bc),
                                        bins.h if bins is not None else None, _prec(precision),
                                        _ptr(out_native), _ptr(out_binned), _ptr(out_status)))
    return out_native, out_binned, out_status


def chi2_grad(ctx, tables, batch, bins, obs, sigma, precision=FP32, recompute=True,
              binned=False):
    """trx_chi2_grad.  Returns dict(chi2 [B], dT [sum N], dlog10_vmr [B, n_abs],
    dRp [B], status [B], binned [B, n_ch] or None)."""
    dev = batch.T.device
    B = batch.B
    obs = torch.as_tensor(obs, dtype=torch.float64).to(dev).contiguous()
    sigma = torch.as_tensor(sigma, dtype=torch.float64).to(dev).contiguous()
    out = {"chi2": torch.empty(B, dtype=torch.float64, device=dev),
           "dT": torch.empty(batch.T.numel(), dtype=torch.float64, device=dev),
           "dlog10_vmr": torch.empty((B, tables.n_abs), dtype=torch.float64, device=dev),
           "dRp": torch.empty(B, dtype=torch.float64, device=dev),
           "status": torch.empty(B, dtype=torch.int32, device=dev),
           "binned": torch.empty((B, bins.n), dtype=torch.float64, device=dev) if binned else None}
    ctx.bind_stream()
    bc = batch.cstruct()
    ctx.check(lib().trx_chi2_grad(ctx.h, tables.h, ctypes.byref(bc), bins.h, _prec(precision),
                                  _ptr(obs), _ptr(sigma), int(bool(recompute)), _ptr(out["chi2"]),
                                  _ptr(out["dT"]), _ptr(out["dlog10_vmr"]), _ptr(out["dRp"]),
                                  _ptr(out["binned"]), _ptr(out["status"])))
    return out


class Chi2Problem:
    """Everything of a chi^2 evaluation except the differentiated parameters:
    the context, tables, channels, a DeviceBatch giving the layer counts,
    pressures, radii, windows and constants, the observation and sigma."""

    def __init__(self, ctx, tables, bins, batch, obs, sigma, precision=FP32):
        self.ctx, self.tables, self.bins, self.batch = ctx, tables, bins, batch
        dev = batch.T.device
        self.obs = torch.as_tensor(obs, dtype=torch.float64).to(dev).contiguous()
        self.sigma = torch.as_tensor(sigma, dtype=torch.float64).to(dev).contiguous()
        self.precision = precision

    def with_params(self, T, log10_vmr, Rp):
        """A DeviceBatch sharing this problem's arrays but the given
        parameter tensors (float64, on the device)."""
        b = object.__new__(DeviceBatch)
        b.__dict__.update(self.batch.__dict__)
        b.T = T.detach().to(torch.float64).contiguous()
        b.log10_vmr = log10_vmr.detach().to(torch.float64).contiguous()
        b.Rp = Rp.detach().to(torch.float64).contiguous()
        return b


class TransitChi2(torch.autograd.Function):
    """chi^2 per model as a differentiable function of the per-layer
    temperatures T [sum N], the log10 mixing ratios [B, n_abs] and Rp [B].

    The value and the gradient come from one trx_chi2_grad call (recompute
    mode: no opacity or optical depth is kept); only the gradient vectors
    are saved for backward."""

    @staticmethod
    def forward(ctx, T, log10_vmr, Rp, problem):
        b = problem.with_params(T, log10_vmr, Rp)
        out = chi2_grad(problem.ctx, problem.tables, b, problem.bins, problem.obs,
                        problem.sigma, problem.precision)
        bad = out["status"] != 0
        if bool(bad.any()):
            out["chi2"] = torch.where(bad, torch.full_like(out["chi2"], float("nan")), out["chi2"])
        ctx.save_for_backward(out["dT"], out["dlog10_vmr"], out["dRp"], problem.batch.layer_off)
        return out["chi2"]

    @staticmethod
    def backward(ctx, g):
        dT, dv, dR, off = ctx.saved_tensors
        g = g.to(torch.float64)
        counts = (off[1:] - off[:-1]).to(torch.int64)
        gT = dT * torch.repeat_interleave(g, counts)
        return gT, dv * g[:, None], dR * g, None


class Plan:
    """trx_plan_*: a batched launch for up to B_max models of at most N_max
    layers, replayed from a HIP graph when ``graph`` is set.

    Outputs default to plan-owned tensors of B_max rows (the first B rows are
    returned), so that repeated launches keep the output pointers a graph
    was captured with."""

    def __init__(self, ctx, tables, bins, B_max, N_max, precision=FP32, graph=True,
                 persistent=True, grad=False, emission=False, two_layer=False):
        self.ctx, self.tables, self.bins = ctx, tables, bins
        self.B_max, self.N_max = int(B_max), int(N_max)
        flags = (PLAN_GRAPH if graph else 0) | (PLAN_PERSISTENT if persistent else 0) | \
            (PLAN_GRAD if grad else 0) | (PLAN_EMISSION if emission else 0) | \
            (PLAN_TWO_LAYER if two_layer else 0)
        h = ctypes.c_void_p()
        ctx.check(lib().trx_plan_create(ctx.h, tables.h, bins.h if bins is not None else None,
                                        self.B_max, self.N_max, _prec(precision), flags,
                                        ctypes.byref(h)))
        self.h = h
        dev = torch.device("cuda", ctx.device)
        self.out_status = torch.empty(self.B_max, dtype=torch.int32, device=dev)
        self.out_binned = None if bins is None else torch.empty(
            (self.B_max, bins.n), dtype=torch.float64, device=dev)
        self.out_native = None
        self.grad = bool(grad)
        if self.grad:
            f64 = dict(dtype=torch.float64, device=dev)
            self.obs = torch.zeros((self.B_max, bins.n), **f64)
            self.sigma = torch.ones(bins.n, **f64)
            self.out_chi2 = torch.empty(self.B_max, **f64)
            self.out_dT = torch.empty(self.B_max * self.N_max, **f64)
            self.out_dvmr = torch.empty((self.B_max, max(tables.n_abs, 1)), **f64)
            self.out_dRp = torch.empty(self.B_max, **f64)

    def set_star(self, T_star, n_mu=4):
        """trx_plan_set_star of an emission plan: T_star (scalar or [<= B_max])
        is copied into a plan-owned device tensor of B_max entries."""
        dev = self.out_status.device
        t = torch.as_tensor(T_star, dtype=torch.float64).flatten()
        if not hasattr(self, "T_star"):
            self.T_star = torch.full((self.B_max,), 5800.0, dtype=torch.float64, device=dev)
        if t.numel() == 1:
            self.T_star.fill_(float(t[0]))
        else:
            self.T_star[:t.numel()].copy_(t)
        self.ctx.check(lib().trx_plan_set_star(self.h, _ptr(self.T_star), int(n_mu)))

    def launch_grad(self, batch, obs, sigma):
        """trx_plan_launch of a gradient plan: chi^2 against obs [B, n_ch]
        with sigma [n_ch] and its gradient.  obs and sigma are copied into
        plan-owned tensors (stable pointers for the graph).  Returns dict
        (chi2, dT [sum N], dlog10_vmr [B, n_abs], dRp, binned, status)."""
        B = batch.B
        self.obs[:B].copy_(torch.as_tensor(obs, dtype=torch.float64).reshape(B, -1))
        self.sigma.copy_(torch.as_tensor(sigma, dtype=torch.float64))
        self.ctx.bind_stream()
        bc = batch.cstruct()
        self.ctx.check(lib().trx_plan_launch(
            self.h, ctypes.byref(bc), None, _ptr(self.out_binned), _ptr(self.out_status),
            _ptr(self.obs), _ptr(self.sigma), _ptr(self.out_chi2), _ptr(self.out_dT),
            _ptr(self.out_dvmr), _ptr(self.out_dRp)))
        # dT is indexed by the batch's (absolute) layer offsets
        nT = int(batch.T.numel()) if hasattr(batch, "T") else int(batch.db.layer_off[batch.b + 1])
        return {"chi2": self.out_chi2[:B], "dT": self.out_dT[:nT],
                "dlog10_vmr": self.out_dvmr[:B, :self.tables.n_abs], "dRp": self.out_dRp[:B],
                "binned": self.out_binned[:B], "status": self.out_status[:B]}

    def launch(self, batch, native=False, binned=True, out_native=None, out_binned=None,
               out_status=None):
        """trx_plan_launch on ``batch`` (a DeviceBatch).  Returns (depth_native
        or None, depth_binned or None, model_status), each with B rows."""
        B = batch.B
        if native and out_native is None:
            if self.out_native is None:
                self.out_native = torch.full((self.B_max, self.tables.n_wn), float("nan"),
                                             dtype=torch.float64, device=self.out_status.device)
            out_native = self.out_native
        if not native:
            out_native = None
        if binned and out_binned is None:
            out_binned = self.out_binned
        if not binned:
            out_binned = None
        if out_status is None:
            out_status = self.out_status
        self.ctx.bind_stream()
        bc = batch.cstruct()
        self.ctx.check(lib().trx_plan_launch(self.h, ctypes.byref(bc), _ptr(out_native),
                                             _ptr(out_binned), _ptr(out_status), None, None,
                                             None, None, None, None))
        cut = lambda t: None if t is None else t[:B]
        return cut(out_native), cut(out_binned), out_status[:B]

    def autotune(self, batch, cache_json=None):
        self.ctx.bind_stream()
        bc = batch.cstruct()
        path = None if cache_json is None else os.fsencode(cache_json)
        self.ctx.check(lib().trx_autotune(self.h, ctypes.byref(bc), path))
        return self.describe()

    def set_variant(self, variant):
        self.ctx.check(lib().trx_plan_set_variant(self.h, variant.encode()))

    def describe(self):
        return lib().trx_plan_describe(self.h).decode()

    def close(self):
        if self.h:
            lib().trx_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
