"""The profile-likelihood discovery test of section 4.2 (Eq.5) over batched pseudo-experiments
on the GPU (gs_discovery_batched: per toy a fit with the signal free and a fit with it fixed at
zero, t = 2 (-ln L_null - (-ln L_free))), against the oracle's two fits toy by toy, and the
distribution of t under the null hypothesis against chi-square with one degree of freedom."""
import numpy as np
import pytest
from scipy import stats

import gsgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    import paper_1812_05686_amd as gs
    gs.lib()
    return gs


def _run(gs, toys, signal=0):
    import torch
    batch = gs.Batch(toys)
    th0 = np.zeros((len(toys), batch.stride))
    for t, m in enumerate(toys):
        th0[t, : m.n_params] = m.theta0
    r = gs.discovery(batch, torch.tensor(th0, dtype=torch.float64, device="cuda"), batch.scales(toys),
                     [signal] * len(toys), free=batch.free_masks(toys))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


@pytest.mark.parametrize("which", ["energy", "gamma"])
def test_discovery_matches_oracle(gs, orc, which):
    """Null pseudo-experiments of the Gaussian-signal model (energy family) and of a small
    photoelectron-family model with its 862 keV line as the signal: t, and both fits' -ln L,
    toy by toy against the oracle (|dt| <= 2e-6, |d(-ln L)| <= 1e-6)."""
    if which == "energy":
        toys = gsgen.discovery_toys(24)
    else:
        toys = gsgen.discovery_toys(12, base=gsgen.small_gamma_model(n_true=300, n_reco=120, seed=2), study=6)
    r = _run(gs, toys)
    assert np.all(r["status_free"] & gs.ST_CONVERGED) and np.all(r["status_null"] & gs.ST_CONVERGED)
    assert np.all(r["theta_null"][:, 0] == 0.0)
    for t, m in enumerate(toys):
        ref = orc.Oracle(m).discovery(0, free=m.free_mask())
        assert ref["ok"], (t, ref)
        assert abs(r["t"][t] - ref["t"]) <= 2e-6, (t, r["t"][t], ref["t"])
        assert abs(r["nll_free"][t] - ref["nll_free"]) <= 1e-6
        assert abs(r["nll_null"][t] - ref["nll_null"]) <= 1e-6


def test_discovery_null_distribution(gs):
    """4096 null pseudo-experiments: every pair of fits converges, t >= 0, and t follows
    chi-square with one degree of freedom (Wilks; the signal rate is unbounded): a
    Kolmogorov-Smirnov test and the mean (1 +- 4 standard errors)."""
    toys = gsgen.discovery_toys(4096)
    r = _run(gs, toys)
    assert np.all(r["status_free"] & gs.ST_CONVERGED) and np.all(r["status_null"] & gs.ST_CONVERGED)
    t = r["t"]
    assert np.all(np.isfinite(t)) and t.min() >= -1e-6
    assert stats.kstest(np.maximum(t, 0.0), stats.chi2(1).cdf).pvalue > 1e-3
    assert abs(t.mean() - 1.0) <= 4.0 * np.sqrt(2.0 / len(t))
