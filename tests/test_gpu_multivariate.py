"""The multivariate slice likelihood of section 2.4 (cost model Eq.3) on the GPU against the
oracle: the energy histogram's Poisson likelihood plus one pulse-shape piece per energy
slice (the slice's histogram given its total).  -ln L and the gradient at the NLL / gradient
bars, the identity with the joint 2-D likelihood for one-bin slices, fits within 1e-3 sigma,
and multivariate toys mixed with joint 2-D and 1-D toys in one batch."""
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


def _small(width, datasets=2):
    m = gsgen.small_gamma_model(n_true=150, n_reco=90, seed=9, n_psd=13, n_datasets=datasets).replace(
        win_lo=11, win_hi=77)
    return gsgen.multivariate_model(m, width)


CASES = {"c2_mv": lambda: gsgen.multivariate_model(gsgen.config2(), 90),
         "small_mv_ragged": lambda: _small(7),
         "small_mv_one_slice": lambda: _small(66, datasets=1)}


@pytest.mark.parametrize("name", list(CASES))
def test_multivariate_parity(gs, orc, name):
    m = CASES[name]()
    o = orc.Oracle(m)
    model = gs.Model(m)
    pts = [m.theta_true, m.theta0, gsgen.offset_point(m, 2.0, seed=2)]
    pts[-1] = pts[-1].copy()
    pts[-1][-3:] = (0.02, 1.1, -0.3)
    for th in pts:
        v, g, st = model.nll_grad(th)
        ov, og, ost = o.nll_grad(th)
        assert st == ost == 0
        assert abs(v - ov) / abs(ov) <= NLL_TOL, (name, v, ov)
        assert _grad_err(g, og, m.fd_scale) <= GRAD_TOL, (name, _grad_err(g, og, m.fd_scale))
        v2, st2 = model.nll(th)
        assert st2 == 0 and abs(v2 - ov) / abs(ov) <= NLL_TOL
    ref = o.expected(pts[2])[:, m.win_lo:m.win_hi, :]
    mu = model.expected(pts[2]).reshape(ref.shape)
    big = ref >= 1e-3
    assert np.max(np.abs(mu - ref)[big] / ref[big]) <= MU_TOL


def test_one_bin_slices_equal_joint_2d(gs):
    """One slice per energy bin: the GPU's multivariate -ln L and gradient equal its joint 2-D
    ones (the Poisson histogram factorises into its total and the multinomial of its bins)."""
    mv = _small(1)
    joint = mv.replace(slice_edges=None)
    th = gsgen.offset_point(mv, 1.0, seed=5)
    th[-3:] = (0.01, 0.97, 0.2)
    v, g, st = gs.Model(mv).nll_grad(th)
    vj, gj, stj = gs.Model(joint).nll_grad(th)
    assert st == stj == 0
    assert abs(v - vj) / abs(vj) <= 1e-12
    assert _grad_err(g, gj, mv.fd_scale) <= 1e-9


def test_multivariate_fits_and_mixed_batch(gs, orc):
    """Host fit (adjoint) and the device BFGS of a multivariate model against the oracle's fit
    (1e-3 sigma); a batch mixing multivariate, joint 2-D and 1-D toys equals the single-model
    values toy by toy."""
    import torch
    m = _small(11)
    ref = orc.Oracle(m).fit()
    assert ref["ok"]
    r = gs.Model(m).fit(m.theta0, m.fd_scale, hesse=False)
    assert r["ok"] and np.max(np.abs(r["theta"] - ref["theta"]) / ref["sigma"]) <= 1e-3
    assert abs(r["nll"] - ref["nll"]) <= 1e-6
    toys = [m, _small(5, datasets=1), m.replace(slice_edges=None),
            gsgen.small_gamma_model(n_true=180, n_reco=70, seed=4).replace(win_lo=5, win_hi=61)]
    batch = gs.Batch(toys)
    th = np.zeros((len(toys), batch.stride))
    for t, q in enumerate(toys):
        th[t, : q.n_params] = q.theta_true
    nll, grad, st = batch.nll_grad(torch.tensor(th, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    nll, grad, st = nll.cpu().numpy(), grad.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all()
    for t, q in enumerate(toys):
        v, g, s = gs.Model(q).nll_grad(q.theta_true)
        assert abs(nll[t] - v) / abs(v) <= 1e-13, t
        np.testing.assert_allclose(grad[t, : q.n_params], g, rtol=1e-10, atol=1e-9)
    rb = batch.fit(torch.tensor(np.stack([np.pad(q.theta0, (0, batch.stride - q.n_params)) for q in toys]),
                                dtype=torch.float64, device="cuda"), batch.scales(toys))
    torch.cuda.synchronize()
    assert int(rb["status"][0]) & gs.ST_CONVERGED
    assert np.max(np.abs(rb["theta"][0, : m.n_params].cpu().numpy() - ref["theta"]) / ref["sigma"]) <= 1e-3
