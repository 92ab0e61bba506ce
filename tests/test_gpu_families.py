"""GPU parity of the further response families and of exact bin contents (section 2.3 names
the modified Gaussian, generalized gamma and scaled Poisson; section 2.5 the response mesh):
the direct per-pair path through the C ABI against the CPU oracle, element by element, at the
Borexino-scale size (4000 cells x 900 bins) and on ragged small models, plus batches that mix
these toys with the fast-path families, fits, and the refusal and degenerate cases.

Bars as for the other families: |dNLL|/|NLL| <= 1e-11; per-bin expected counts within 1e-12
relative for mu >= 1e-3; gradient per component |dg_p| s_p <= 1e-8 max(|g_p| s_p, 1)."""
import numpy as np
import pytest

import gsgen

pytestmark = pytest.mark.gpu

NLL_TOL = 1e-11
MU_TOL = 1e-12
GRAD_TOL = 1e-8
G = gsgen


@pytest.fixture(scope="module")
def gs():
    import paper_1812_05686_amd as gs
    gs.lib()
    return gs


def _grad_err(g, og, scale):
    return np.max(np.abs(g - og) * scale / np.maximum(np.abs(og) * scale, 1.0))


def _ragged(family, shape=0.0, exact=0, seed=4):
    return G.small_gamma_model(n_true=333, n_reco=211, seed=seed, family=family, shape=shape,
                               exact_bins=exact).replace(win_lo=7, win_hi=150)


CASES = {
    "c1_gengamma_p1.6": lambda: G.family_model(G.GENGAMMA_PE, 1.6),
    "c1_spois": lambda: G.family_model(G.SPOIS_PE),
    "c1_emg_f0.35": lambda: G.family_model(G.EMG_PE, 0.35),
    "c1_gamma_exact": lambda: G.family_model(G.GAMMA_PE, exact_bins=1),
    "c1_gauss_exact": lambda: G.family_model(G.GAUSS_PE, exact_bins=1),
    "c1_gengamma_exact": lambda: G.family_model(G.GENGAMMA_PE, 1.6, exact_bins=1),
    "c1_emg_exact": lambda: G.family_model(G.EMG_PE, 0.35, exact_bins=1),
    "c0_exact": lambda: G.config0().replace(exact_bins=1),
    "ragged_gengamma_p0.7": lambda: _ragged(G.GENGAMMA_PE, 0.7),
    "ragged_spois": lambda: _ragged(G.SPOIS_PE, seed=5),
    "ragged_emg_exact_f0.8": lambda: _ragged(G.EMG_PE, 0.8, exact=1, seed=6),
    "ragged_gamma_exact": lambda: _ragged(G.GAMMA_PE, exact=1, seed=7),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, orc):
    m = CASES[request.param]()
    return request.param, m, orc.Oracle(m)


def test_expected_nll_gradient(gs, case):
    """Expected counts, -ln L and gradient at an off-minimum point; -ln L at the truth."""
    name, m, o = case
    model = gs.Model(m)
    th = G.offset_point(m, 1.5, seed=2)
    ref = o.expected(th)[:, m.win_lo:m.win_hi, :]
    mu = model.expected(th).reshape(ref.shape)
    big = ref >= 1e-3
    rel = np.abs(mu - ref)[big] / ref[big]
    worst = tuple(int(q) for q in np.argwhere(big)[np.argmax(rel)])
    assert rel.max() <= MU_TOL, (name, rel.max(), worst, mu[worst], ref[worst])
    np.testing.assert_allclose(mu, ref, rtol=1e-9, atol=1e-12)
    v, g, st = model.nll_grad(th)
    ov, og, ost = o.nll_grad(th)
    assert st == ost == 0, (name, st, ost)
    assert abs(v - ov) / abs(ov) <= NLL_TOL, (name, v, ov)
    assert _grad_err(g, og, m.fd_scale) <= GRAD_TOL, (name, _grad_err(g, og, m.fd_scale))
    v0, st0 = model.nll(m.theta_true)
    ov0 = o.nll(m.theta_true)[0]
    assert st0 == 0 and abs(v0 - ov0) / abs(ov0) <= NLL_TOL, (name, v0, ov0)


@pytest.mark.parametrize("which", ["ragged_gengamma_p0.7", "ragged_spois", "ragged_emg_exact_f0.8",
                                   "ragged_gamma_exact", "c1_spois"])
def test_species_spectra_and_plain_path(gs, orc, which):
    """Per-species folded spectra (the direct path's per-species fold) against the oracle, and
    the plain path's cached fold across a rate-only change."""
    m = CASES[which]()
    o = orc.Oracle(m)
    model = gs.Model(m)
    th = G.offset_point(m, 1.0, seed=5)
    F = model.species_spectra(th)
    ref = o.species_fold(th)[m.win_lo:m.win_hi]
    big = np.abs(th[: m.n_species])[None, :] * ref >= 1e-3
    rel = np.abs(F - ref)[big] / ref[big]
    assert rel.max() <= MU_TOL, (which, rel.max())
    v1, st = model.nll(th)
    ov = o.nll(th)[0]
    assert st == 0 and abs(v1 - ov) / abs(ov) <= NLL_TOL
    th2 = th.copy()
    th2[: m.n_species] *= 1.03
    v2, _ = model.nll(th2)
    assert abs(v2 - o.nll(th2)[0]) / abs(ov) <= NLL_TOL


def test_mixed_batch_with_fast_path_toys(gs, orc):
    """One batch of direct-path toys (each new family, exact bins) and fast-path toys (gamma,
    Gaussian, energy family): every toy equals its own single-model evaluation, and the
    direct-path toys the oracle."""
    import torch
    toys = [_ragged(G.GENGAMMA_PE, 1.3, seed=11), G.small_gamma_model(n_true=200, n_reco=90, seed=12),
            _ragged(G.SPOIS_PE, seed=13), G.config0(), _ragged(G.EMG_PE, 0.5, exact=1, seed=14),
            G.small_gamma_model(n_true=200, n_reco=181, seed=15, family=G.GAUSS_PE),  # 8-pe bins: admitted
            G.config0().replace(exact_bins=1), _ragged(G.GAMMA_PE, exact=1, seed=16)]
    batch = gs.Batch(toys)
    th = np.zeros((len(toys), batch.stride))
    for t, m in enumerate(toys):
        th[t, : m.n_params] = G.offset_point(m, 1.0, seed=t)
    nll, grad, st = batch.nll_grad(torch.tensor(th, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    nll, grad, st = nll.cpu().numpy(), grad.cpu().numpy(), st.cpu().numpy()
    for t, m in enumerate(toys):
        P = m.n_params
        v, g, s = gs.Model(m).nll_grad(th[t, :P])
        assert st[t] == s == 0
        assert abs(nll[t] - v) <= 1e-13 * abs(v), t
        np.testing.assert_allclose(grad[t, :P], g, rtol=1e-10, atol=1e-9)
        if m.family >= G.GENGAMMA_PE or m.exact_bins:
            ov, og, _ = orc.Oracle(m).nll_grad(th[t, :P])
            assert abs(nll[t] - ov) / abs(ov) <= NLL_TOL, t
            assert _grad_err(grad[t, :P], og, m.fd_scale) <= GRAD_TOL, t


@pytest.mark.parametrize("family,shape,exact", [(G.GENGAMMA_PE, 1.6, 0), (G.SPOIS_PE, 0.0, 0), (G.EMG_PE, 0.35, 0),
                                                (G.GAMMA_PE, 0.0, 1), (G.EMG_PE, 0.35, 1)])
def test_fits_match_oracle(gs, orc, family, shape, exact):
    """Host adjoint fit, host finite-difference fit and the device batched fit land within
    1e-3 sigma of the oracle's fit."""
    import torch
    m = G.small_gamma_model(n_true=300, n_reco=120, seed=2, family=family, shape=shape, exact_bins=exact)
    ref = orc.Oracle(m).fit()
    assert ref["ok"]
    model = gs.Model(m)
    for use_fd in (False, True):
        r = model.fit(m.theta0, m.fd_scale, use_fd=use_fd)
        assert r["ok"], (use_fd, r["status"])
        z = np.abs(r["theta"] - ref["theta"]) / ref["sigma"]
        assert z.max() <= 1e-3, (use_fd, z.max())
        assert abs(r["nll"] - ref["nll"]) <= 1e-6
    batch = gs.Batch([m, m])
    th0 = torch.tensor(np.stack([m.theta0, m.theta0]), dtype=torch.float64, device="cuda")
    sc = torch.tensor(np.stack([m.fd_scale, m.fd_scale]), dtype=torch.float64, device="cuda")
    rb = batch.fit(th0, sc)
    torch.cuda.synchronize()
    for t in range(2):
        assert int(rb["status"][t]) & gs.ST_CONVERGED
        z = np.abs(rb["theta"][t].cpu().numpy() - ref["theta"]) / ref["sigma"]
        assert z.max() <= 1e-3


def test_sharp_response_with_exact_bins(gs, orc):
    """Exact bin contents have no bin-width limit: a 5 eV response on 10 keV bins (refused by the
    midpoint fast path) is evaluated, and matches the oracle."""
    base = G.config0()
    edges = 2.5 + 10.0 * np.arange(201.0)
    th = base.theta_true.copy()
    th[3:] = (0.005, 0.0)
    m = base.replace(reco_edges=edges, theta_true=th, pull_centre=th.copy(), exact_bins=1)
    mu_true = orc.Oracle(m).expected(th)
    m = m.replace(counts=np.random.default_rng(11).poisson(mu_true).astype(float))
    o = orc.Oracle(m)
    model = gs.Model(m)
    ref = o.expected(th)[:, m.win_lo:m.win_hi, :]
    mu = model.expected(th).reshape(ref.shape)
    big = ref >= 1e-3
    assert big.sum() > 20 and np.max(np.abs(mu - ref)[big] / ref[big]) <= MU_TOL
    v, g, st = model.nll_grad(th)
    ov, og, ost = o.nll_grad(th)
    assert st == ost == 0 and abs(v - ov) / abs(ov) <= NLL_TOL
    assert _grad_err(g, og, m.fd_scale) <= GRAD_TOL


def test_direct_path_refusals_and_invalid(gs, orc):
    """A generalized-gamma response too narrow for its mean (m > 300 s) is refused with
    UNRESOLVED and NaN; an invalid quenching constant is DOMAIN on both sides."""
    m = G.small_gamma_model(n_true=120, n_reco=60, seed=3, family=G.GENGAMMA_PE, shape=1.4)
    th = m.theta_true.copy()
    S = m.n_species
    th[S + 2:S + 5] = (0.3, 1e-4, 0.0)  # s ~ 0.3 pe at m ~ 1000 pe
    v, g, st = gs.Model(m).nll_grad(th)
    assert st == gs.ST_UNRESOLVED and np.isnan(v) and np.all(np.isnan(g))
    th = m.theta_true.copy()
    th[S + 1] = -0.01
    assert gs.Model(m).nll_grad(th)[2] == orc.Oracle(m).nll(th)[1] == 1
