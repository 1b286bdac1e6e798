"""The synthetic transmission retrieval on the GPU: the retrieval's
log-likelihoods against the oracle's for random prior points (each through
an opaque cloud deck, as in the paper's transit retrieval), and a nested
sampling run that recovers the truth of a synthetic observation (the
oracle's binned spectrum of the truth plus seeded 50 ppm noise)."""

import numpy as np
import pytest

import oracle
from synth.constants import GM_JUP, R_JUP, R_SUN
from synth.atmosphere import log_uniform_channels
from synth.workloads import Channels, make_tables, observation_noise

pytestmark = pytest.mark.gpu

N = 60


def _model(tables, x, N, absorbers):
    """Oracle model dict of a sampled point x (log10 abundances, T, Rp/R_J,
    log10 cloud-top pressure)."""
    na = len(absorbers)
    return dict(T=np.full(N, x[na]), p_bot=1e6, p_top=1e-4, log10_vmr=np.array(x[:na]),
                Rp=x[na + 1] * 6.9911e7, Rs=R_SUN, GM=GM_JUP, wn_lo=0, wn_hi=tables.n_wn,
                he_h2=0.17, k_B=1.380649e-23, amu=1.66053906660e-27, gravity=0,
                cloud_sigma=np.inf, cloud_p_top=10.0 ** x[na + 2], cloud_p_bottom=1e6)


@pytest.fixture(scope="module")
def setup(gpu_ctx):
    from paper_1912_07759_amd import trx
    from paper_1912_07759_amd.retrieval import TransitRetrieval
    tables = make_tables(2, n_wn=1500, n_lines=150)
    lo, hi = log_uniform_channels(tables.wn, 30)
    ch = Channels(lo, hi)
    absorbers = tables.names
    truth = np.array([-3.5, -6.0, -5.0, -7.0, -8.0, 1200.0, 1.35, 3.0])
    ref = oracle.forward_model(_model(tables, truth, N, absorbers), tables, ch)["binned"]
    noise, sigma = observation_noise(2, 1, len(ch.lo))
    obs = ref + noise[0]
    T = trx.Tables.from_synth(gpu_ctx, tables)
    bins = trx.Bins(gpu_ctx, T, ch.lo, ch.hi)
    ret = TransitRetrieval(gpu_ctx, T, bins, obs, sigma, absorbers, R_SUN, GM_JUP, n_layers=N,
                           B_max=2048, precision="bf16x2")
    yield tables, ch, absorbers, truth, obs, sigma, ret
    ret.close()
    bins.close()
    T.close()


def test_loglike_matches_oracle(setup):
    tables, ch, absorbers, truth, obs, sigma, ret = setup
    u = np.random.default_rng(3).random((12, len(ret.priors)))
    u[0] = [(t - p.a) / (p.b - p.a) for t, p in zip(truth, ret.priors)]
    ll = ret(u)
    # both alternating plans (submit / collect) give the same bits
    for _ in range(2):
        ret.submit(u)
        assert np.array_equal(ret.collect(), ll)
    x = ret.physical(u)
    for k in range(len(u)):
        b = oracle.forward_model(_model(tables, x[k], N, absorbers), tables, ch)["binned"]
        r = (b - obs) / sigma
        want = -0.5 * np.sum(r * r) - np.sum(np.log(np.sqrt(2.0 * np.pi) * sigma))
        # bound from the fast mode's 1e-6 relative error of each binned value
        d = 1e-6 * np.abs(b) / sigma
        bound = np.sum(np.abs(r) * d) + 0.5 * np.sum(d * d) + 1e-9 * abs(want)
        print(f"point {k}: lnL {ll[k]:.6e} oracle {want:.6e} (bound {bound:.1e})")
        assert abs(ll[k] - want) <= bound


def test_nested_sampling_recovers_truth(setup):
    from paper_1912_07759_amd.retrieval import nested_sample, posterior
    tables, ch, absorbers, truth, obs, sigma, ret = setup
    r = nested_sample(ret, len(ret.priors), n_live=150, batch=2048, dlogz=0.5, seed=5)
    w, mean, std = posterior(r, ret.priors)
    names = [p.name for p in ret.priors]
    print(f"logz {r['logz']:.2f} +- {r['logz_err']:.2f}, {r['n_iter']} iterations, "
          f"{r['n_eval']} likelihoods in {r['n_calls']} launches, {r['seconds']:.1f} s "
          f"(host waited {ret.wait_seconds:.1f} s)")
    for n, t, m, s in zip(names, truth, mean, std):
        print(f"  {n}: truth {t:.4g}, posterior {m:.4g} +- {s:.2g}")
    # the well-constrained parameters: the main absorber, T, Rp, within 3
    # posterior sigmas and fixed bounds (2.5 dex, 400 K, 0.05 R_J: the prior
    # spans 11 dex, 1600 K, 0.3 R_J)
    for i, cap in ((0, 2.5), (5, 400.0), (6, 0.05)):
        assert abs(mean[i] - truth[i]) <= 3.0 * std[i] + 1e-9, names[i]
        assert abs(mean[i] - truth[i]) <= cap, names[i]
    # the best sample fits the observation to the noise (chi^2 ~ n_ch)
    assert np.max(r["logl"]) > -0.5 * 3.0 * len(obs) - np.sum(np.log(np.sqrt(2 * np.pi) * sigma))
