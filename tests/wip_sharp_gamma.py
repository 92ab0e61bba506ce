"""GPU test pending its first run: the gamma family's clamped pair loops (fold staging flag,
adjoint per-block vote).  Not collected by pytest until it has passed on the GPU."""
import numpy as np
import pytest

import gsgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    import paper_1812_05686_amd as gs
    gs.lib()
    return gs


def test_sharp_gamma_response_exponent_range(gs, orc):
    """The gamma family with sigma = 0.01 pe on 36-pe bins (cell means on the bin midpoints:
    LY 1200 pe/MeV on 30-keV cells, kB ~ 0): pair exponents reach about -7e9 inside a fold
    tile and an adjoint block, so both kernels must take their clamped exponentials (the
    fold by its staging flag, the adjoint by its per-block wave vote).  The tile-relative
    exponent then carries u64 k |ln x - ln x_r| of rounding (k up to 2e10), which sets the
    bar; the gradient is only required to be finite."""
    base = gsgen.small_gamma_model(n_true=100, n_reco=40, seed=8)
    th = base.theta_true.copy()
    th[base.n_species:] = (1200.0, 1e-12, 0.01, 0.0, 0.0)
    m = base.replace(theta_true=th, pull_centre=th.copy(), pull_sigma=np.zeros(len(th)))
    m = m.replace(counts=np.random.default_rng(11).poisson(orc.Oracle(m).expected(th)).astype(float))
    o = orc.Oracle(m)
    x = 0.5 * (m.reco_edges[1:] + m.reco_edges[:-1])
    tol = 3.0 * 2.0 ** -53 * (x.max() / 0.01) ** 2 * np.log(x.max() / x.min())
    model = gs.Model(m)
    ref = o.expected(th)[:, m.win_lo:m.win_hi, :]
    mu = model.expected(th).reshape(ref.shape)
    assert np.all(np.isfinite(mu))
    big = ref >= 1e-3
    assert big.sum() >= 30
    assert np.max(np.abs(mu - ref)[big] / ref[big]) <= tol
    v, g, st = model.nll_grad(th)
    ov, og, ost = o.nll_grad(th)
    assert st == ost == 0
    assert abs(v - ov) / abs(ov) <= tol
    assert np.all(np.isfinite(g))
