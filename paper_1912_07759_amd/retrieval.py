"""A synthetic transmission retrieval driven by the batched forward plan.

The paper's transmission retrieval (Retrievals section, prior table) fits
five absorber abundances in log10 space, an isothermal temperature, the
planet radius and the pressure of a fully opaque cloud deck, all with
uniform priors whose bounds are given in linear space (Optimization
section); a model the forward model rejects gets the lowest possible
log-likelihood (Model Rejection subsection).  Its samplers are nested
samplers (MultiNest, Nestle, PolyChord, ...), which are not part of this
library; `nested_sample` is a plain single-ellipsoid nested sampler
(Skilling's algorithm with the bounding-ellipsoid proposal of the Nestle /
MultiNest family) written for batched likelihoods: candidates are drawn
from the current ellipsoid a batch at a time, evaluated in one launch of
the plan, and consumed in order by the usual rejection step.

Every forward model runs on the GPU through `trx.Plan`; the Gaussian
log-likelihood of the binned spectra is summed on the host over the
channels (B x n_ch values).
"""

import time

import numpy as np


class UniformPrior:
    """Uniform prior of one parameter; bounds in linear space, the
    parameter sampled uniformly in linear or log10 space."""

    def __init__(self, name, lo, hi, mode="linear"):
        assert mode in ("linear", "log") and hi > lo
        self.name, self.lo, self.hi, self.mode = name, float(lo), float(hi), mode
        if mode == "log":
            assert lo > 0
            self.a, self.b = np.log10(lo), np.log10(hi)
        else:
            self.a, self.b = self.lo, self.hi

    def __call__(self, u):
        """Unit-cube coordinate -> the sampled value (log10 of the parameter
        in log mode)."""
        return self.a + (self.b - self.a) * np.asarray(u)


def paper_transit_priors(absorbers):
    """The paper's transmission priors: abundances 1e-12..1e-1 (log),
    T 400..2000 K, radius 1.2..1.5 R_J, cloud-top pressure 1e-8..1 bar
    (log; in Pa here)."""
    pri = [UniformPrior(f"log10_{a}", 1e-12, 1e-1, "log") for a in absorbers]
    pri += [UniformPrior("T_K", 400.0, 2000.0), UniformPrior("Rp_RJ", 1.2, 1.5),
            UniformPrior("log10_Pcloud_Pa", 1e-3, 1e5, "log")]
    return pri


class LikelihoodBudgetExhausted(Exception):
    """nested_sample stopped: it spent its likelihood budget (max_evals)
    before the evidence converged.  Not a RuntimeError, so that library and
    device errors are never mistaken for it."""


def _logsubexp(a, b):
    return a + np.log1p(-np.exp(b - a))


def nested_sample(loglike, ndim, n_live=400, batch=1024, dlogz=0.1, enlarge=1.25, seed=0,
                  max_iter=200000, max_evals=10 ** 7, method="multi"):
    """Nested sampling of the unit cube [0, 1]^ndim (the priors are applied
    by `loglike`, which maps an [K, ndim] array of unit-cube points to K
    log-likelihoods, -inf for a rejected model).

    Each iteration removes the live point of lowest likelihood L_min, books
    it with the prior volume shrinking by e^{-1/n_live} per iteration, and
    replaces it by a point with L > L_min drawn uniformly from a bound of the
    live points intersected with the cube: their bounding ellipsoid (scaled
    to contain them all, volume enlarged by `enlarge`; method "single"), or
    a union of such ellipsoids from recursive 2-means splits kept while they
    halve the volume (method "multi", the MultiNest construction; a point
    covered by q ellipsoids is kept with probability 1/q, and no ellipsoid is
    smaller than its share n_k/n_live of the expected prior volume left).
    Proposals come from a pool
    filled `batch` at a time (one `loglike` call each); a `loglike` with
    submit(u) / collect() methods gets the next batch, drawn from the bound
    of the moment, submitted as soon as a pool is taken, so that it is
    evaluated while the pool is consumed.  Stops when the live points can
    add less than `dlogz` to log Z.

    Returns dict(logz, logz_err, information, samples [M, ndim] unit-cube,
    logl [M], logwt [M], n_iter, n_eval, n_calls, seconds)."""
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    u = rng.random((n_live, ndim))
    logl = np.asarray(loglike(u), dtype=np.float64)
    n_eval, n_calls = n_live, 1
    dead_u, dead_l, dead_v = [], [], []
    logvol = 0.0
    logz, h = -np.inf, 0.0
    pool_u = np.zeros((0, ndim))
    pool_l = np.zeros(0)
    overlap = hasattr(loglike, "submit") and hasattr(loglike, "collect")
    pending = None
    it = 0
    step = -1.0 / n_live
    while it < max_iter:
        # remaining evidence bound: the live points' best L over the volume left
        lmax = np.max(logl)
        if np.isfinite(logz) and np.logaddexp(logz, lmax + logvol) - logz < dlogz:
            break
        w = int(np.argmin(logl))
        lmin = logl[w]
        # the shell between e^{logvol} and e^{logvol - 1/n_live}
        logwt = _logsubexp(logvol, logvol + step) + lmin
        if np.isfinite(logwt):
            lz_new = np.logaddexp(logz, logwt)
            h = (np.exp(logwt - lz_new) * lmin
                 + (np.exp(logz - lz_new) * (h + logz) if np.isfinite(logz) else 0.0) - lz_new)
            logz = lz_new
        dead_u.append(u[w].copy())
        dead_l.append(lmin)
        dead_v.append(logwt)
        logvol += step
        # replacement: the first pool candidate with L > L_min; refill the pool
        # from the current ellipsoid when it runs dry
        while True:
            ok = np.flatnonzero(pool_l > lmin)
            if ok.size:
                k = int(ok[0])
                u[w], logl[w] = pool_u[k], pool_l[k]
                pool_u, pool_l = pool_u[k + 1:], pool_l[k + 1:]
                break
            if n_eval >= max_evals:
                raise LikelihoodBudgetExhausted("nested_sample: likelihood budget exhausted")
            ells = ([_bounding_ellipsoid(u, enlarge)] if method == "single"
                    else _split_ellipsoids(u, enlarge, np.exp(logvol), n_live))
            if pending is not None:
                pool_u, pool_l = pending, np.asarray(loglike.collect(), dtype=np.float64)
                pending = None
            else:
                pool_u = _union_draws(ells, batch, rng)
                pool_l = np.asarray(loglike(pool_u), dtype=np.float64)
            n_eval += len(pool_u)
            n_calls += 1
            if overlap:
                pending = _union_draws(ells, batch, rng)
                loglike.submit(pending)
        it += 1
    if pending is not None:
        loglike.collect()          # the batch in flight at the end is not used
    # the live points share the remaining volume equally
    live_wt = logvol - np.log(n_live) + logl
    for k in np.argsort(logl):
        lz_new = np.logaddexp(logz, live_wt[k])
        if np.isfinite(live_wt[k]):
            h = (np.exp(live_wt[k] - lz_new) * logl[k]
                 + np.exp(logz - lz_new) * (h + logz) - lz_new)
        logz = lz_new
    samples = np.vstack([np.array(dead_u).reshape(-1, ndim), u])
    lw = np.concatenate([np.array(dead_v), live_wt])
    ll = np.concatenate([np.array(dead_l), logl])
    return {"logz": float(logz), "logz_err": float(np.sqrt(max(h, 0.0) / n_live)),
            "information": float(h), "samples": samples, "logl": ll, "logwt": lw,
            "n_iter": it, "n_eval": n_eval, "n_calls": n_calls,
            "seconds": time.perf_counter() - t0}


class _Ellipsoid:
    """{x : (x - mu)^T A^{-1} (x - mu) <= 1} with A = scale^2 cov."""

    def __init__(self, mu, cov, scale2):
        self.mu, self.d = mu, len(mu)
        self.A = cov * scale2
        self.L = np.linalg.cholesky(self.A)
        self.Ainv = np.linalg.inv(self.A)
        self.logvol = float(np.sum(np.log(np.diag(self.L))))   # up to the unit ball's volume

    def grow_to(self, logvol):
        if logvol > self.logvol:
            f = np.exp(2.0 * (logvol - self.logvol) / self.d)
            self.__init__(self.mu, self.A, f)

    def contains(self, x):
        y = x - self.mu
        return np.einsum("ij,jk,ik->i", y, self.Ainv, y) <= 1.0

    def draw(self, n, rng):
        g = rng.standard_normal((n, self.d))
        g /= np.linalg.norm(g, axis=1)[:, None]
        rad = rng.random(n) ** (1.0 / self.d)
        return self.mu + (g * rad[:, None]) @ self.L.T


def _bounding_ellipsoid(x, enlarge):
    """The ellipsoid of the points' covariance shape scaled to contain them
    all, its volume times `enlarge`."""
    d = x.shape[1]
    mu = x.mean(axis=0)
    cov = np.cov(x, rowvar=False) + 1e-12 * np.eye(d)
    y = x - mu
    r2 = np.max(np.einsum("ij,jk,ik->i", y, np.linalg.inv(cov), y))
    return _Ellipsoid(mu, cov, r2 * enlarge ** (2.0 / d))


def _two_means(x, iters=10):
    """Lloyd's 2-means from the two points farthest apart along the first
    principal axis."""
    y = x - x.mean(axis=0)
    ax = np.linalg.svd(y, full_matrices=False)[2][0]
    p = y @ ax
    c = np.stack([x[np.argmin(p)], x[np.argmax(p)]])
    lab = np.zeros(len(x), dtype=int)
    for _ in range(iters):
        lab = np.argmin(((x[:, None, :] - c[None]) ** 2).sum(-1), axis=1)
        if lab.min() == lab.max():
            break
        c = np.stack([x[lab == k].mean(axis=0) for k in (0, 1)])
    return lab


def _split_ellipsoids(x, enlarge, x_vol, n_live, min_pts=None):
    """Recursive 2-means splits of the points, kept while the two children's
    bounding ellipsoids fill less than half their parent's volume; each
    ellipsoid then grown, if needed, to its share of the prior volume left
    (the cube has volume 1; volumes in units of the d-ball's)."""
    d = x.shape[1]
    min_pts = 2 * (d + 1) if min_pts is None else min_pts
    from math import lgamma, log, pi
    log_ball = 0.5 * d * log(pi) - lgamma(0.5 * d + 1.0)

    def rec(pts):
        e = _bounding_ellipsoid(pts, enlarge)
        if len(pts) < 2 * min_pts:
            return [(e, len(pts))]
        lab = _two_means(pts)
        a, b = pts[lab == 0], pts[lab == 1]
        if len(a) < min_pts or len(b) < min_pts:
            return [(e, len(pts))]
        ea, eb = _bounding_ellipsoid(a, enlarge), _bounding_ellipsoid(b, enlarge)
        if np.logaddexp(ea.logvol, eb.logvol) < e.logvol + np.log(0.5):
            return rec(a) + rec(b)
        return [(e, len(pts))]

    out = []
    for e, n in rec(x):
        e.grow_to(np.log(n / n_live * x_vol) - log_ball)
        out.append(e)
    return out


def _union_draws(ells, n, rng):
    """n points uniform in the union of the ellipsoids intersected with the
    unit cube: an ellipsoid picked with probability proportional to its
    volume, a uniform point in it, kept with probability 1/q (q = the number
    of ellipsoids holding it) and only inside the cube; refilled until n
    points are kept, so that a likelihood launch carries a full batch."""
    lv = np.array([e.logvol for e in ells])
    p = np.exp(lv - lv.max())
    p /= p.sum()
    out, have = [], 0
    for _ in range(256):
        k = rng.choice(len(ells), size=2 * n, p=p)
        pts = np.empty((2 * n, ells[0].d))
        for j, e in enumerate(ells):
            m = k == j
            if m.any():
                pts[m] = e.draw(int(m.sum()), rng)
        if len(ells) > 1:
            q = np.sum([e.contains(pts) for e in ells], axis=0)
            pts = pts[rng.random(len(pts)) * q < 1.0]
        pts = pts[np.all((pts > 0.0) & (pts < 1.0), axis=1)]
        out.append(pts)
        have += len(pts)
        if have >= n:
            break
    return np.vstack(out)[:n]


def posterior(result, priors=None):
    """Normalised posterior weights, weighted mean and standard deviation of
    the samples (in the priors' sampled coordinates when given)."""
    w = np.exp(result["logwt"] - result["logz"])
    w = w / w.sum()
    x = result["samples"]
    if priors is not None:
        x = np.column_stack([p(x[:, i]) for i, p in enumerate(priors)])
    mean = w @ x
    std = np.sqrt(np.maximum(w @ (x - mean) ** 2, 0.0))
    return w, mean, std


class TransitRetrieval:
    """Log-likelihood of the paper's transmission retrieval on forward plans:
    isothermal atmospheres of `n_layers` layers between p_bot and p_top (Pa),
    constant abundances of the tables' absorbers, radius in Jupiter radii, a
    fully opaque cloud deck from the cloud-top pressure down, on the whole
    wavenumber grid, binned to `bins`; Gaussian likelihood of `obs` with
    per-channel `sigma`.  Candidates are evaluated up to `B_max` per launch
    of a graph-captured plan whose device inputs are rewritten in place.  Two
    plans, each with its own inputs and pinned staging buffers, alternate
    under submit() / collect(), so that one batch runs on the GPU while the
    caller works on the previous one."""

    R_JUP = 6.9911e7

    def __init__(self, ctx, tables, bins, obs, sigma, absorbers, Rs, GM, n_layers=100,
                 p_bot=1e6, p_top=1e-4, B_max=2048, precision="bf16x2"):
        import torch
        from . import trx
        self.trx, self.torch = trx, torch
        self.priors = paper_transit_priors(absorbers)
        self.n_abs = len(absorbers)
        self.obs = np.asarray(obs, dtype=np.float64)
        self.sigma = np.asarray(sigma, dtype=np.float64)
        self.N, self.B_max = int(n_layers), int(B_max)
        B, N, na = self.B_max, self.N, self.n_abs
        W = tables.n_wn
        self.slots = []
        for _ in range(2):
            db = trx.DeviceBatch(np.full(B, N), np.full(B * N, 1000.0), np.full(B, p_bot),
                                 np.full(B, p_top), np.full((B, na), -6.0),
                                 np.full(B, 1.3 * self.R_JUP), np.full(B, Rs), np.full(B, GM),
                                 np.zeros(B), np.full(B, W), max_layers=N,
                                 cloud_sigma=np.full(B, np.inf), cloud_p_top=np.full(B, 1e3),
                                 cloud_p_bottom=np.full(B, p_bot))
            plan = trx.Plan(ctx, tables, bins, B_max=B, N_max=N, precision=precision, graph=True)
            pin = lambda *shape: torch.empty(shape, dtype=torch.float64, pin_memory=True)
            self.slots.append({"db": db, "plan": plan, "T": pin(B * N), "vmr": pin(B, na),
                               "Rp": pin(B), "pc": pin(B)})
        self.turn = 0
        self.inflight = None
        self.n_eval = 0
        self.n_launch = 0
        self.wait_seconds = 0.0   # host time blocked in collect()

    def physical(self, u):
        """Unit-cube points -> sampled coordinates (log10 abundances, T,
        Rp/R_J, log10 cloud-top pressure in Pa)."""
        return np.column_stack([p(u[:, i]) for i, p in enumerate(self.priors)])

    def __call__(self, u):
        u = np.atleast_2d(u)
        out = np.empty(len(u))
        for s in range(0, len(u), self.B_max):
            self.submit(u[s:s + self.B_max])
            out[s:s + self.B_max] = self.collect()
        return out

    def submit(self, u):
        """Queue the likelihoods of at most B_max unit-cube points (one plan
        launch); the results come from the next collect()."""
        assert self.inflight is None, "collect() the batch in flight first"
        u = np.atleast_2d(u)
        assert len(u) <= self.B_max
        x = self.physical(u)
        K, N, na = len(x), self.N, self.n_abs
        sl = self.slots[self.turn]
        self.turn ^= 1
        db = sl["db"]
        # the staging buffers of this slot were last read by its previous
        # launch, which its collect() has waited for
        sl["T"][:K * N].numpy()[:] = np.repeat(x[:, na], N)
        sl["vmr"][:K].numpy()[:] = x[:, :na]
        sl["Rp"][:K].numpy()[:] = x[:, na + 1] * self.R_JUP
        sl["pc"][:K].numpy()[:] = 10.0 ** x[:, na + 2]
        db.T[:K * N].copy_(sl["T"][:K * N], non_blocking=True)
        db.log10_vmr[:K].copy_(sl["vmr"][:K], non_blocking=True)
        db.Rp[:K].copy_(sl["Rp"][:K], non_blocking=True)
        db.cloud[1][:K].copy_(sl["pc"][:K], non_blocking=True)
        _, binned, status = sl["plan"].launch(_Prefix(db, K))
        self.inflight = (binned, status, K)

    def collect(self):
        """Log-likelihoods of the batch in flight (waits for it)."""
        binned, status, K = self.inflight
        self.inflight = None
        t0 = time.perf_counter()
        binned = binned[:K].cpu().numpy()
        status = status[:K].cpu().numpy()
        self.wait_seconds += time.perf_counter() - t0
        self.n_eval += K
        self.n_launch += 1
        r = (binned - self.obs[None, :]) / self.sigma[None, :]
        ll = -0.5 * np.sum(r * r, axis=1) - np.sum(np.log(np.sqrt(2.0 * np.pi) * self.sigma))
        # rejected models (Model Rejection subsection): lowest log-likelihood
        ll[(status != 0) | ~np.isfinite(ll)] = -np.inf
        return ll

    def close(self):
        if self.inflight is not None:
            self.collect()
        for sl in self.slots:
            sl["plan"].close()


class _Prefix:
    """The first K models of a DeviceBatch (same device arrays)."""

    def __init__(self, db, K):
        self.db, self.B = db, int(K)

    def cstruct(self):
        return self.db.cstruct(self.B)
