"""GPU fits against stored oracle fits of the benchmark workloads.

tests/golden/fit_goldens.json holds oracle fits (analytic gradient, BFGS to EDM < 1e-9, Hesse
sigma) written by tests/golden/make_fit_goldens.py from the oracle and the seeded generator
only.  Here the same models are rebuilt from the generator and fitted on the GPU: the host
quasi-Newton driver over device evaluations with the adjoint gradient and with central
finite differences (gs_fit), and the device BFGS over all of them in one batch
(gs_fit_batched).  Bars: every free parameter within 1e-3 sigma of the oracle's fitted value,
fixed ones untouched, and |d(-ln L)| <= 1e-6 at the minimum."""
import json
import os

import numpy as np
import pytest

import gsgen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fit_goldens.json")
THETA_TOL = 1e-3   # in units of the oracle's sigma
NLL_ABS = 1e-6


@pytest.fixture(scope="module")
def gs():
    import paper_1812_05686_amd as gs
    gs.lib()
    return gs


@pytest.fixture(scope="module")
def goldens():
    with open(GOLDEN) as f:
        doc = json.load(f)
    cache = {}

    def build(recipe):
        c = recipe["config"]
        if c in ("c0", "c1", "c2"):
            if c not in cache:
                cache[c] = {"c0": gsgen.config0, "c1": gsgen.config1, "c2": gsgen.config2}[c]()
            return cache[c]
        key = (c, recipe["pool"])
        if key not in cache:
            cache[key] = gsgen.config3(recipe["pool"], base=gsgen.config1()) if c == "c3" else gsgen.config4(recipe["pool"])
        return cache[key][recipe["toy"]]

    out = []
    for name, g in doc["cases"].items():
        assert g["ok"], name
        m = build(g["recipe"])
        assert len(g["theta0"]) == m.n_params and np.array_equal(np.asarray(g["free"], bool), m.free_mask() > 0), name
        out.append((name, m, g))
    return out


def _check(name, m, g, theta, nll, what):
    """Free parameters with a finite oracle sigma within THETA_TOL sigma; a free rate whose
    spectrum has no weight in the toy's window leaves -ln L flat (no finite sigma): both fits
    must leave it where it started; fixed parameters untouched."""
    free = np.asarray(g["free"], bool)
    th_hat, sig, th0 = np.asarray(g["theta_hat"]), np.asarray(g["sigma"]), np.asarray(g["theta0"])
    fin = free & np.isfinite(sig) & (sig > 0)
    z = np.abs(theta[fin] - th_hat[fin]) / sig[fin]
    assert z.max() <= THETA_TOL, (name, what, z.max(), int(np.nonzero(fin)[0][np.argmax(z)]))
    flat = free & ~fin
    assert np.all(np.abs(theta[flat] - th_hat[flat]) <= 1e-6 * np.maximum(1.0, np.abs(th0[flat]))), (name, what)
    assert np.array_equal(theta[~free], th0[~free]), (name, what)
    assert abs(nll - g["nll"]) <= NLL_ABS, (name, what, nll, g["nll"])
    return float(z.max())


def test_host_fits_match_oracle_goldens(gs, goldens):
    """gs_fit with the adjoint gradient and with central finite differences (the plain path)
    on every stored case: the single 1-D and Borexino-scale fits, the pulse-shape model, the
    toy-study pseudo-experiments with their free masks and one toy of each class of the mix."""
    worst = {}
    for name, m, g in goldens:
        model = gs.Model(m)
        for use_fd in (False, True):
            r = model.fit(np.asarray(g["theta0"]), np.asarray(g["scale"]), use_fd=use_fd,
                          free=np.asarray(g["free"], np.uint8), hesse=False)
            assert r["ok"], (name, use_fd, r["status"])
            worst[(name, use_fd)] = _check(name, m, g, r["theta"], r["nll"], "fd" if use_fd else "adjoint")
        model.close()
    print("worst |dtheta|/sigma", max(worst.values()))


def test_batched_fit_matches_oracle_goldens(gs, goldens):
    """gs_fit_batched over every stored case in one uneven batch (1-D energy-family,
    Borexino-scale and pulse-shape models together), each toy with its own start, free mask
    and parameter scales."""
    import torch
    models = [m for _, m, _ in goldens]
    batch = gs.Batch(models)
    n, P = len(models), batch.stride
    th0, free, sc = np.zeros((n, P)), np.zeros((n, P), np.uint8), np.ones((n, P))
    for t, (_, m, g) in enumerate(goldens):
        k = m.n_params
        th0[t, :k], free[t, :k], sc[t, :k] = g["theta0"], g["free"], g["scale"]
    r = batch.fit(torch.tensor(th0, dtype=torch.float64, device="cuda"),
                  torch.tensor(sc, dtype=torch.float64, device="cuda"),
                  free=torch.tensor(free, device="cuda"))
    torch.cuda.synchronize()
    th, nll, st = r["theta"].cpu().numpy(), r["nll"].cpu().numpy(), r["status"].cpu().numpy()
    worst = 0.0
    for t, (name, m, g) in enumerate(goldens):
        assert st[t] & gs.ST_CONVERGED, (name, int(st[t]))
        worst = max(worst, _check(name, m, g, th[t, : m.n_params], nll[t], "batched"))
    print("worst |dtheta|/sigma", worst)
