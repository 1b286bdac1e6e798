"""The nested sampler and the priors of the retrieval driver, on the CPU,
against closed forms: the evidence and moments of a Gaussian likelihood in
the unit cube, the evidence lost to a rejected region (Model Rejection
subsection: the lowest log-likelihood), and the uniform priors in linear
and log10 space with bounds given in linear space (Optimization section)."""

import numpy as np
import pytest
from scipy.special import erf

from paper_1912_07759_amd.retrieval import (UniformPrior, nested_sample, paper_transit_priors,
                                            posterior)

MU, SIG, D = 0.4, 0.05, 3


def _gauss(u):
    u = np.atleast_2d(u)
    return (-0.5 * np.sum(((u - MU) / SIG) ** 2, axis=1)
            - D * np.log(np.sqrt(2.0 * np.pi) * SIG))


def _cube_mass(lo, hi):
    """Mass of N(MU, SIG^2) in [lo, hi] per dimension."""
    c = lambda x: 0.5 * (1.0 + erf((x - MU) / (SIG * np.sqrt(2.0))))
    return c(hi) - c(lo)


def test_gaussian_evidence_and_moments():
    r = nested_sample(_gauss, D, n_live=300, batch=256, seed=1)
    exact = D * np.log(_cube_mass(0.0, 1.0))          # ~0: the density is normalised
    assert abs(r["logz"] - exact) <= 4.0 * r["logz_err"] + 0.02, (r["logz"], r["logz_err"])
    w, mean, std = posterior(r)
    assert np.all(np.abs(mean - MU) < 0.01)
    assert np.all(np.abs(std - SIG) < 0.01)
    assert abs(np.sum(w) - 1.0) < 1e-12
    # the information H of a Gaussian posterior under a unit-volume prior
    h_exact = -D * (0.5 + np.log(np.sqrt(2.0 * np.pi) * SIG))
    assert abs(r["information"] - h_exact) < 0.3


@pytest.mark.parametrize("method", ["single", "multi"])
def test_gaussian_evidence_both_bounds(method):
    r = nested_sample(_gauss, D, n_live=300, batch=256, seed=4, method=method)
    assert abs(r["logz"] - D * np.log(_cube_mass(0.0, 1.0))) <= 4.0 * r["logz_err"] + 0.02


def test_bimodal_evidence_and_mode_weights():
    """Two equal, well separated Gaussians (each of weight 1/2, normalised):
    Z = 1 and half the posterior mass in each mode; the multi-ellipsoid
    bound keeps both modes."""
    c1, c2, s = np.array([0.25] * D), np.array([0.75] * D), 0.03

    def ll(u):
        u = np.atleast_2d(u)
        a = -0.5 * np.sum(((u - c1) / s) ** 2, axis=1)
        b = -0.5 * np.sum(((u - c2) / s) ** 2, axis=1)
        return np.logaddexp(a, b) + np.log(0.5) - D * np.log(np.sqrt(2.0 * np.pi) * s)
    r = nested_sample(ll, D, n_live=400, batch=512, seed=3, method="multi")
    assert abs(r["logz"]) <= 4.0 * r["logz_err"] + 0.02, (r["logz"], r["logz_err"])
    w, _, _ = posterior(r)
    left = np.sum(w[r["samples"][:, 0] < 0.5])
    assert abs(left - 0.5) < 0.1


def test_rejected_region_removes_its_evidence():
    def ll(u):
        v = _gauss(u)
        v[np.atleast_2d(u)[:, 0] > 0.45] = -np.inf
        return v
    r = nested_sample(ll, D, n_live=300, batch=256, seed=2)
    exact = np.log(_cube_mass(0.0, 0.45)) + (D - 1) * np.log(_cube_mass(0.0, 1.0))
    assert abs(r["logz"] - exact) <= 4.0 * r["logz_err"] + 0.02, (r["logz"], exact)
    w, _, _ = posterior(r)
    assert np.all(w[r["samples"][:, 0] > 0.45] == 0.0)


def test_deterministic_for_a_seed():
    a = nested_sample(_gauss, D, n_live=100, batch=128, seed=7)
    b = nested_sample(_gauss, D, n_live=100, batch=128, seed=7)
    assert a["logz"] == b["logz"] and a["n_eval"] == b["n_eval"]
    assert a["n_calls"] < a["n_eval"] / 10      # candidates come in batches


def test_uniform_priors():
    lin = UniformPrior("T", 400.0, 2000.0)
    assert lin(0.0) == 400.0 and lin(1.0) == 2000.0 and lin(0.25) == 800.0
    lg = UniformPrior("x", 1e-12, 1e-1, "log")
    assert lg(0.0) == pytest.approx(-12.0) and lg(1.0) == pytest.approx(-1.0)
    pri = paper_transit_priors(["H2O", "CH4", "CO", "CO2", "NH3"])
    assert [p.name for p in pri][-3:] == ["T_K", "Rp_RJ", "log10_Pcloud_Pa"]
    assert pri[-1](0.0) == pytest.approx(-3.0) and pri[-1](1.0) == pytest.approx(5.0)
    assert (pri[-2].lo, pri[-2].hi) == (1.2, 1.5)


class _Deferred:
    """A likelihood with the submit / collect interface of the GPU
    retrieval, evaluated on the CPU: submit() only stores the candidates,
    collect() evaluates them, so the sampler's overlap path (a pending
    batch drawn from an earlier bound) runs as it does on the GPU."""

    def __init__(self, f):
        self.f, self.pending, self.n_submit = f, None, 0

    def __call__(self, u):
        return self.f(u)

    def submit(self, u):
        assert self.pending is None
        self.pending = np.array(u, copy=True)
        self.n_submit += 1

    def collect(self):
        u, self.pending = self.pending, None
        return self.f(u)


def test_overlapped_batches_keep_the_gaussian_pins():
    lk = _Deferred(_gauss)
    r = nested_sample(lk, D, n_live=300, batch=256, seed=11)
    assert lk.n_submit > 5 and lk.pending is None
    assert abs(r["logz"] - D * np.log(_cube_mass(0.0, 1.0))) <= 4.0 * r["logz_err"] + 0.02
    w, mean, std = posterior(r)
    assert np.all(np.abs(mean - MU) < 0.01) and np.all(np.abs(std - SIG) < 0.01)


def test_overlapped_batches_keep_the_bimodal_pins():
    c1, c2, s = np.array([0.25] * D), np.array([0.75] * D), 0.03

    def ll(u):
        u = np.atleast_2d(u)
        a = -0.5 * np.sum(((u - c1) / s) ** 2, axis=1)
        b = -0.5 * np.sum(((u - c2) / s) ** 2, axis=1)
        return np.logaddexp(a, b) + np.log(0.5) - D * np.log(np.sqrt(2.0 * np.pi) * s)
    r = nested_sample(_Deferred(ll), D, n_live=400, batch=512, seed=13, method="multi")
    assert abs(r["logz"]) <= 4.0 * r["logz_err"] + 0.02, (r["logz"], r["logz_err"])
    w, _, _ = posterior(r)
    assert abs(np.sum(w[r["samples"][:, 0] < 0.5]) - 0.5) < 0.1


def test_budget_exhaustion_is_its_own_exception():
    """A spent likelihood budget raises LikelihoodBudgetExhausted, which is
    not a RuntimeError (so library and device errors are never taken for
    it)."""
    from paper_1912_07759_amd.retrieval import LikelihoodBudgetExhausted
    assert not issubclass(LikelihoodBudgetExhausted, RuntimeError)
    with pytest.raises(LikelihoodBudgetExhausted):
        nested_sample(_gauss, D, n_live=50, batch=64, seed=1, max_evals=200)
