"""The Monte Carlo template fit (section 3.2, cost model Eq.1) on the GPU against the oracle:
mu_dj = eps_d sum_s R_s T_sj with the species' reco-space templates, no fold.  Element-wise
expectations, -ln L and the rate gradient at the NLL / gradient bars, fits within 1e-3 sigma,
batches of template toys, and template toys mixed with analytic ones in one batch."""
import numpy as np
import pytest

import gsgen

pytestmark = pytest.mark.gpu

NLL_TOL, MU_TOL, GRAD_TOL = 1e-11, 1e-12, 1e-8


@pytest.fixture(scope="module")
def gs():
    import paper_1812_05686_amd as gs
    gs.lib()
    return gs


def _grad_err(g, og, scale):
    return np.max(np.abs(g - og) * scale / np.maximum(np.abs(og) * scale, 1.0))


def _cases():
    t1 = gsgen.template_model()
    yield "tmpl", t1
    yield "tmpl2d_flat", gsgen.template_model(flat2d=True)
    # a window inside the histogram, two datasets with exposures 1 and 0.6
    cnt = np.concatenate([t1.counts, np.random.default_rng(4).poisson(0.6 * t1.counts).astype(float)], axis=0)
    yield "tmpl_window_2ds", t1.replace(exposure=np.array([1.0, 0.6]), counts=cnt, win_lo=37, win_hi=811)


@pytest.mark.parametrize("name,m", list(_cases()), ids=lambda x: x if isinstance(x, str) else "")
def test_template_parity(gs, orc, name, m):
    o = orc.Oracle(m)
    model = gs.Model(m)
    for th in (m.theta_true, m.theta0, gsgen.offset_point(m, 2.0, seed=3)):
        ref = o.expected(th)[:, m.win_lo:m.win_hi, :]
        mu = model.expected(th).reshape(ref.shape)
        big = ref >= 1e-3
        assert np.max(np.abs(mu - ref)[big] / ref[big]) <= MU_TOL
        v, g, st = model.nll_grad(th)
        ov, og, ost = o.nll_grad(th)
        assert st == ost == 0
        assert abs(v - ov) / abs(ov) <= NLL_TOL, (name, v, ov)
        assert _grad_err(g, og, m.fd_scale) <= GRAD_TOL, (name, _grad_err(g, og, m.fd_scale))
        v2, st2 = model.nll(th)
        assert st2 == 0 and abs(v2 - ov) / abs(ov) <= NLL_TOL
    F = model.species_spectra(m.theta_true)
    assert np.array_equal(F, m.spectra[:, m.win_lo:m.win_hi].T)


def test_template_fits_match_oracle(gs, orc):
    """Host fits (adjoint and central finite differences) and the device BFGS of a template
    fit land within 1e-3 sigma of the oracle's fit."""
    import torch
    m = gsgen.template_model()
    ref = orc.Oracle(m).fit()
    assert ref["ok"]
    model = gs.Model(m)
    for use_fd in (False, True):
        r = model.fit(m.theta0, m.fd_scale, use_fd=use_fd, hesse=False)
        assert r["ok"]
        assert np.max(np.abs(r["theta"] - ref["theta"]) / ref["sigma"]) <= 1e-3
        assert abs(r["nll"] - ref["nll"]) <= 1e-6
    batch = gs.Batch([m])
    rb = batch.fit(torch.tensor(m.theta0[None, :], dtype=torch.float64, device="cuda"), m.fd_scale)
    torch.cuda.synchronize()
    assert int(rb["status"][0]) & gs.ST_CONVERGED
    th = rb["theta"][0].cpu().numpy()
    assert np.max(np.abs(th - ref["theta"]) / ref["sigma"]) <= 1e-3


def test_template_toys_and_mixed_batch(gs, orc):
    """A batch of template toys with their own rates and data, mixed with Borexino-scale toys
    and a pulse-shape toy: every toy's batched value equals its single-model value, and sampled
    template toys match the oracle; the batched fit converges for every toy."""
    import torch
    base = gsgen.template_model()
    tt = gsgen.template_toys(6, base)
    toys = tt[:3] + gsgen.config3(3, base=gsgen.config1()) + tt[3:] + [
        gsgen.small_gamma_model(n_true=150, n_reco=90, seed=9, n_psd=13, n_datasets=2)]
    batch = gs.Batch(toys)
    th = np.zeros((len(toys), batch.stride))
    for t, m in enumerate(toys):
        th[t, : m.n_params] = m.theta_true
    nll, grad, st = batch.nll_grad(torch.tensor(th, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    nll, grad, st = nll.cpu().numpy(), grad.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all()
    for t, m in enumerate(toys):
        v, g, s = gs.Model(m).nll_grad(m.theta_true)
        assert abs(nll[t] - v) / abs(v) <= 1e-13
        np.testing.assert_allclose(grad[t, : m.n_params], g, rtol=1e-10, atol=1e-9)
    for t in (0, 7):
        ov, og, _ = orc.Oracle(toys[t]).nll_grad(toys[t].theta_true)
        assert abs(nll[t] - ov) / abs(ov) <= NLL_TOL
        assert _grad_err(grad[t, : toys[t].n_params], og, toys[t].fd_scale) <= GRAD_TOL
    th0 = np.zeros_like(th)
    for t, m in enumerate(toys):
        th0[t, : m.n_params] = m.theta0
    r = batch.fit(torch.tensor(th0, dtype=torch.float64, device="cuda"), batch.scales(toys),
                  free=batch.free_masks(toys))
    torch.cuda.synchronize()
    assert np.all(r["status"].cpu().numpy() & gs.ST_CONVERGED)
