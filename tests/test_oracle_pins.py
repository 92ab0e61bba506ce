"""Pins of the CPU oracle against things other than itself.

Each test ties one part of the oracle to a closed form, a library routine,
quadrature, brute force, or an invariant of the method (GooStats,
arXiv:1812.05686).  The paper prints no worked numerical example (its figures
are absent and Table 1 holds only timings), so no printed value is pinned.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate, special, stats

import gsgen

GAUSS_E, GAUSS_PE, GAMMA_PE = gsgen.GAUSS_E, gsgen.GAUSS_PE, gsgen.GAMMA_PE
NOM = gsgen.C1_RESP


def _line_model(family, e0, resp, edges, rate=1000.0):
    """One monoenergetic species (AnaPeak-type, section 4.3) and nothing else."""
    th = np.concatenate([[rate], resp])
    return gsgen.Model(name="line", family=family, n_true=1, e_lo=0.0, e_step=1.0,
                       spectra=np.zeros((1, 1)), line_energy=np.array([e0]), reco_edges=edges,
                       exposure=np.ones(1), counts=np.zeros((1, len(edges) - 1, 1)), win_lo=0,
                       win_hi=len(edges) - 1, pull_centre=th.copy(), pull_sigma=np.zeros(len(th)),
                       theta_true=th, theta0=th.copy(), fd_scale=np.ones(len(th)))


# ------------------------------------------------------------- quenching ---
@pytest.mark.parametrize("kb", [0.005, 0.011, 0.02])
@pytest.mark.parametrize("e", [0.0004, 0.01, 0.25, 1.0, 3.0])
def test_quench_vs_quadrature(orc, e, kb):
    """Birks' integral (reading R7) against adaptive quadrature in u = sqrt(E')."""
    mpmath.mp.dps = 40
    c = mpmath.mpf(kb) * 2
    val = mpmath.quad(lambda u: 2 * u * u / (u + c), [0, mpmath.sqrt(mpmath.mpf(e))])
    assert orc.quench(e, kb) == pytest.approx(float(val / mpmath.mpf(e)), rel=2e-15)


@pytest.mark.parametrize("e", [0.0004, 0.1, 1.0, 3.0])
def test_quench_kb_derivative(orc, e):
    kb, h = 0.011, 1e-6
    d1 = (orc.quench(e, kb + h) - orc.quench(e, kb - h)) / (2 * h)
    d2 = (orc.quench(e, kb + h / 2) - orc.quench(e, kb - h / 2)) / h
    fd = (4 * d2 - d1) / 3
    assert orc.dquench_dkb(e, kb) == pytest.approx(fd, rel=1e-7)


def test_quench_limits(orc):
    # kB -> 0: no quenching; tiny E: Q ~ 2y/3 with y = sqrt(E)/(kB A)
    assert orc.quench(1.0, 1e-9) == pytest.approx(1.0, abs=1e-7)
    e, kb = 1e-12, 0.011
    y = math.sqrt(e) / (kb * 2.0)
    assert orc.quench(e, kb) == pytest.approx(2 * y / 3 - y * y / 2, rel=1e-6)


def test_digamma_vs_scipy(orc):
    xs = np.concatenate([np.geomspace(1e-3, 1e4, 97), [0.5, 1.0, 2.0, 9.999, 10.0, 10.001]])
    for x in xs:
        assert orc.digamma(x) == pytest.approx(special.digamma(x), rel=2e-14, abs=1e-15)


# ------------------------------------------------------------ moments ------
def test_moments_special_cases(orc):
    E = 0.862
    # energy family: b = 0 gives constant width a; a = 0 gives variance b E
    assert orc.moments(GAUSS_E, [10.0, 0.0], 862.0) == pytest.approx((862.0, 10.0))
    assert orc.moments(GAUSS_E, [0.0, 5.0], 862.0)[1] == pytest.approx(math.sqrt(5 * 862.0))
    # pe family: mean is LY * Q * E, linear in LY; without quenching it is LY*E
    m1, _ = orc.moments(GAMMA_PE, [500.0, 0.011, 2.0, 1.15, 0.015], E)
    m2, _ = orc.moments(GAMMA_PE, [250.0, 0.011, 2.0, 1.15, 0.015], E)
    assert m1 == pytest.approx(2 * m2, rel=1e-15)
    assert m1 == pytest.approx(500.0 * orc.quench(E, 0.011) * E, rel=1e-15)
    assert orc.moments(GAMMA_PE, [500.0, 1e-12, 2.0, 0.0, 0.0], E)[0] == pytest.approx(500.0 * E, rel=1e-9)
    # width: only a -> s = a; only b -> s^2 = b m (photostatistics); only c -> s = c m
    _, s = orc.moments(GAMMA_PE, [500.0, 0.011, 2.0, 0.0, 0.0], E)
    assert s == pytest.approx(2.0)
    _, s = orc.moments(GAMMA_PE, [500.0, 0.011, 0.0, 1.15, 0.0], E)
    assert s * s == pytest.approx(1.15 * m1)
    _, s = orc.moments(GAMMA_PE, [500.0, 0.011, 0.0, 0.0, 0.015], E)
    assert s == pytest.approx(0.015 * m1)
    assert orc.moments(GAMMA_PE, [500.0, -0.011, 2.0, 1.15, 0.015], E) is None


# ------------------------------------------------------------ densities ----
@pytest.mark.parametrize("m,s", [(480.0, 24.7), (30.0, 6.3), (1460.0, 46.0), (5.0, 2.9), (0.4, 2.0)])
def test_gamma_density_vs_scipy(orc, m, s):
    k, th = (m / s) ** 2, s * s / m
    for x in np.linspace(max(m - 6 * s, 0.05), m + 6 * s, 41):
        ref = stats.gamma.pdf(x, k, scale=th)
        assert orc.density(GAMMA_PE, x, m, s) == pytest.approx(ref, rel=5e-12, abs=1e-300)


@pytest.mark.parametrize("m,s", [(862.0, 66.4), (0.0, 1.0), (480.0, 24.7)])
def test_gauss_density_vs_scipy(orc, m, s):
    for x in np.linspace(m - 8 * s, m + 8 * s, 33):
        assert orc.density(GAUSS_PE, x, m, s) == pytest.approx(stats.norm.pdf(x, m, s), rel=1e-14)


@pytest.mark.parametrize("fam,m,s", [(GAUSS_E, 862.0, 66.4), (GAMMA_PE, 480.0, 24.7), (GAMMA_PE, 1460.0, 46.0),
                                     (GAMMA_PE, 30.0, 6.3), (GAMMA_PE, 3.0, 2.5), (GAMMA_PE, 0.2, 2.0)])
def test_density_normalisation_and_moments(orc, fam, m, s):
    """P1: integral 1, mean m, second moment m^2 + s^2 over the real line / (0, inf)."""
    f = lambda x: orc.density(fam, x, m, s)
    if fam == GAMMA_PE:
        k = (m / s) ** 2
        if k < 1:
            # singular at 0: substitute t = x^k, dx = t^(1/k - 1)/k dt
            g = lambda t, p: (t ** (1 / k)) ** p * f(t ** (1 / k)) * t ** (1 / k - 1) / k
            hi = (m + 60 * s + 60 * s * s / m) ** k
            mom = [integrate.quad(g, 0, hi, args=(p,), epsabs=0, epsrel=1e-13, limit=400)[0] for p in range(3)]
        else:
            pts = [m - 10 * s, m, m + 10 * s]
            lo, hi = max(m - 40 * s, 0.0), m + 60 * s + 60 * s * s / m
            mom = [integrate.quad(lambda x, p=p: x ** p * f(x), lo, hi, epsabs=0, epsrel=1e-13, limit=400,
                                  points=[q for q in pts if lo < q < hi])[0] for p in range(3)]
    else:
        mom = [integrate.quad(lambda x, p=p: x ** p * f(x), m - 40 * s, m + 40 * s, epsabs=0, epsrel=1e-13,
                              limit=400, points=[m])[0] for p in range(3)]
    assert mom[0] == pytest.approx(1.0, rel=1e-12)
    assert mom[1] == pytest.approx(m, rel=1e-12, abs=1e-12)
    assert mom[2] == pytest.approx(m * m + s * s, rel=1e-11)


@pytest.mark.parametrize("fam,m,s", [(GAUSS_PE, 480.0, 24.7), (GAMMA_PE, 480.0, 24.7), (GAMMA_PE, 4.0, 2.5)])
def test_density_log_derivatives(orc, fam, m, s):
    for x in [m - 2 * s, m - 0.3 * s, m + s, m + 3 * s]:
        if x <= 0:
            continue
        dm, ds = orc.density_dms(fam, x, m, s)
        hm, hs = 1e-5 * s, 1e-5 * s
        fdm = (math.log(orc.density(fam, x, m + hm, s)) - math.log(orc.density(fam, x, m - hm, s))) / (2 * hm)
        fds = (math.log(orc.density(fam, x, m, s + hs)) - math.log(orc.density(fam, x, m, s - hs))) / (2 * hs)
        assert dm == pytest.approx(fdm, rel=1e-6, abs=1e-9)
        assert ds == pytest.approx(fds, rel=1e-6, abs=1e-9)


# ------------------------------------------------------------- fold ---------
@pytest.mark.parametrize("sigma,e0", [(10.0, 1003.0), (7.0, 1003.0), (12.5, 998.7)])
def test_midpoint_lattice_normalisation(orc, sigma, e0):
    """P2: sum_j dx N(xbar_j; m, s^2) over an unbounded uniform lattice equals
    1 + 2 sum_q exp(-2 pi^2 q^2 s^2/dx^2) cos(2 pi q (xbar_0 - m)/dx) (Poisson summation)."""
    dx = 10.0
    edges = 500.0 + dx * np.arange(101)
    M = _line_model(GAUSS_E, e0, np.array([sigma, 0.0]), edges, rate=1.0)
    tot = orc.Oracle(M).expected(M.theta_true).sum()
    x0 = 0.5 * (edges[0] + edges[1])
    q = np.arange(1, 6)
    ref = 1 + 2 * np.sum(np.exp(-2 * np.pi ** 2 * q ** 2 * sigma ** 2 / dx ** 2) * np.cos(2 * np.pi * q * (x0 - e0) / dx))
    assert tot == pytest.approx(ref, rel=2e-15)
    if abs(ref - 1.0) > 1e-11:  # the lattice effect itself is resolved, not just the total
        assert tot - 1.0 == pytest.approx(ref - 1.0, rel=1e-4)


@pytest.mark.parametrize("fam", [GAUSS_PE, GAMMA_PE])
def test_delta_spectrum_reproduces_response(orc, fam):
    """P3: a line species gives mu_j = R eps dx_j r(xbar_j | E0)."""
    edges = np.linspace(0.0, 1440.0, 901)
    e0, R = 0.862, 12345.0
    M = _line_model(fam, e0, NOM, edges, rate=R).replace(exposure=np.array([0.6]))
    mu = orc.Oracle(M).expected(M.theta_true)[0, :, 0]
    m, s = orc.moments(fam, NOM, e0)
    x = 0.5 * (edges[1:] + edges[:-1])
    if fam == GAMMA_PE:
        ref = stats.gamma.pdf(x, (m / s) ** 2, scale=s * s / m)
    else:
        ref = stats.norm.pdf(x, m, s)
    ref = 0.6 * R * np.diff(edges) * ref
    big = ref > 1e-3
    np.testing.assert_allclose(mu[big], ref[big], rtol=5e-12)
    np.testing.assert_allclose(mu, ref, rtol=1e-9, atol=1e-12)


def test_gaussian_of_gaussian(orc):
    """P4: Gaussian true spectrum (E0, s) sampled as density x h on a fine grid, folded with a
    constant-width Gaussian response a, is R dx N(x; E0, s^2 + a^2)."""
    E0, s, a, h = 1000.0, 20.0, 15.0, 2.0
    lo = E0 - 14 * s
    n = int(28 * s / h)
    cent = lo + h * (np.arange(n) + 0.5)
    w = h * stats.norm.pdf(cent, E0, s)
    edges = np.linspace(700.0, 1300.0, 121)
    th = np.array([1e5, a, 0.0])
    M = gsgen.Model(name="gg", family=GAUSS_E, n_true=n, e_lo=lo, e_step=h, spectra=w[None, :],
                    line_energy=np.array([np.nan]), reco_edges=edges, exposure=np.ones(1),
                    counts=np.zeros((1, 120, 1)), win_lo=0, win_hi=120, pull_centre=th, pull_sigma=np.zeros(3),
                    theta_true=th, theta0=th, fd_scale=np.ones(3))
    mu = orc.Oracle(M).expected(th)[0, :, 0]
    x = 0.5 * (edges[1:] + edges[:-1])
    ref = 1e5 * np.diff(edges) * stats.norm.pdf(x, E0, math.hypot(s, a))
    core = np.abs(x - E0) < 6 * math.hypot(s, a)
    np.testing.assert_allclose(mu[core], ref[core], rtol=1e-13)


def test_rate_linearity(orc, c0):
    """P8: mu is linear in every rate with slope eps F_s (F from the species fold)."""
    o = orc.Oracle(c0)
    th = c0.theta_true
    F = o.species_fold(th)
    mu0 = o.expected(th)[0, :, 0]
    for s in range(3):
        for t in (-0.3, 0.45):
            th2 = th.copy()
            th2[s] += t * th[s]
            np.testing.assert_allclose(o.expected(th2)[0, :, 0] - mu0, t * th[s] * F[:, s], rtol=1e-9, atol=1e-9)


def test_rate_gradient_closed_form(orc, c0):
    """P8: d(-ln L)/dR_s = sum_j (1 - n_j/mu_j) eps F_js."""
    o = orc.Oracle(c0)
    th = gsgen.offset_point(c0, 2.0, seed=1)
    F = o.species_fold(th)
    mu = o.expected(th)[0, :, 0]
    n = c0.counts[0, :, 0]
    g_ref = ((1 - n / mu)[:, None] * F).sum(axis=0)
    _, g, st = o.nll_grad(th)
    assert st == 0
    np.testing.assert_allclose(g[:3], g_ref, rtol=1e-10, atol=1e-10)


# ---------------------------------------------------- secondary observable --
def _small2d(orc, n_psd=20, n_datasets=3):
    M = gsgen.small_gamma_model(n_true=120, n_reco=40, seed=3, n_psd=n_psd, n_datasets=n_datasets)
    return M, orc.Oracle(M)


def test_psd_probs_vs_mixture_density(orc):
    """With fine bins well inside the range, P_sk/dy tends to the mixture density."""
    M = gsgen.small_gamma_model(n_true=60, n_reco=10, seed=5, n_psd=4000)
    M = M.replace(psd_edges=np.linspace(-1.0, 2.0, 4001))
    P = orc.Oracle(M).psd_probs(M.theta_true)
    y = 0.5 * (M.psd_edges[1:] + M.psd_edges[:-1])
    dy = np.diff(M.psd_edges)
    for s, (w1, m1, s1, m2, s2) in enumerate(M.psd_mix):
        ref = w1 * stats.norm.pdf(y, m1, s1) + (1 - w1) * stats.norm.pdf(y, m2, s2)
        np.testing.assert_allclose(P[s] / dy, ref, rtol=1e-9, atol=1e-12)


def test_psd_nuisance_invariants(orc):
    M, o = _small2d(orc, n_datasets=1)
    S = M.n_species
    base = M.theta_true.copy()
    # delta shifts both means; kappa scales both widths
    for idx, (delta, kappa) in enumerate([(0.05, 1.0), (0.0, 1.3), (-0.03, 0.8)]):
        th = base.copy()
        th[-3], th[-2] = delta, kappa
        mix = M.psd_mix.copy()
        mix[:, 1] += delta
        mix[:, 3] += delta
        mix[:, 2] *= kappa
        mix[:, 4] *= kappa
        ref = orc.Oracle(M.replace(psd_mix=mix)).psd_probs(base)
        np.testing.assert_allclose(o.psd_probs(th), ref, rtol=1e-13)
    # eta multiplies the odds of component 1 by exp(eta)
    th = base.copy()
    th[-1] = 0.7
    w1 = M.psd_mix[:, 0]
    odds = w1 / (1 - w1) * math.exp(0.7)
    ref = orc.Oracle(M.replace(psd_mix=np.column_stack([odds / (1 + odds), M.psd_mix[:, 1:]]))).psd_probs(base)
    np.testing.assert_allclose(o.psd_probs(th), ref, rtol=1e-13)
    assert np.allclose(o.psd_probs(base).sum(axis=1), 1.0, rtol=1e-15)
    assert S == M.psd_mix.shape[0]


def test_2d_marginal_separability_exposure(orc):
    """P9: sum_k mu_djk equals the 1-D expectation for any nuisances; the likelihood of three
    datasets is the sum of the single-dataset likelihoods; mu scales with exposure."""
    M, o = _small2d(orc)
    th = gsgen.offset_point(M, 1.0, seed=2)
    th[-3:] = [0.04, 1.2, -0.5]
    mu2 = o.expected(th)
    M1 = M.replace(psd_edges=None, psd_mix=None, counts=np.zeros((3, M.n_reco, 1)),
                   pull_centre=M.pull_centre[:-3], pull_sigma=M.pull_sigma[:-3])
    mu1 = orc.Oracle(M1).expected(th[:-3])
    np.testing.assert_allclose(mu2.sum(axis=2), mu1[:, :, 0], rtol=1e-13)
    np.testing.assert_allclose(mu2[1], 0.6 * mu2[0], rtol=1e-14)
    np.testing.assert_allclose(mu2[2], 0.3 * mu2[0], rtol=1e-14)
    total, _ = o.nll(th)
    parts = 0.0
    for d in range(3):
        Md = M.replace(exposure=M.exposure[d:d + 1], counts=M.counts[d:d + 1])
        parts += orc.Oracle(Md).nll(th)[0]
    assert total == pytest.approx(parts, rel=1e-13)


# ---------------------------------------------------------- likelihood ------
def _terms(mu, n):
    return np.where(n > 0, mu - n * np.log(mu), mu)


@pytest.mark.parametrize("which", ["c0", "small", "small2d"])
def test_nll_equals_exactly_rounded_sum(orc, c0, which):
    """P11: -ln L equals math.fsum of the per-bin terms (plus pulls)."""
    if which == "c0":
        M = c0
    elif which == "small":
        M = gsgen.small_gamma_model(n_true=150, n_reco=60, seed=1)
    else:
        M = _small2d(orc)[0]
    M = M.replace(win_lo=3, win_hi=M.n_reco - 2)
    ps = np.zeros(M.n_params)
    ps[M.n_species] = 0.7 * M.fd_scale[M.n_species]
    M = M.replace(pull_sigma=ps)
    o = orc.Oracle(M)
    th = gsgen.offset_point(M, 1.0, seed=3)
    mu = o.expected(th)[:, 3:M.n_reco - 2]
    n = M.counts[:, 3:M.n_reco - 2]
    pull = 0.5 * ((th[M.n_species] - M.pull_centre[M.n_species]) / ps[M.n_species]) ** 2
    ref = math.fsum(list(_terms(mu, n).ravel()) + [pull])
    v, st = o.nll(th)
    assert st == 0
    assert v == pytest.approx(ref, rel=1e-14)


def test_domain_and_status(orc, c0):
    o = orc.Oracle(c0)
    th = c0.theta_true.copy()
    th[0] = -1e6  # drives mu negative in the line region
    v, st = o.nll(th)
    assert v == math.inf and st == 1
    v, g, st = o.nll_grad(th)
    assert np.all(np.isnan(g))
    th = c0.theta_true.copy()
    th[1] = np.nan
    v, st = o.nll(th)
    assert math.isnan(v) and st == 2
    # mu = 0 with n = 0 contributes nothing; with n > 0 it is a domain error
    M = _line_model(GAUSS_E, 1000.0, np.array([10.0, 0.0]), np.linspace(0, 2000, 21), rate=0.0)
    om = orc.Oracle(M)
    v, st = om.nll(M.theta_true)
    assert v == 0.0 and st == 0
    cnt = M.counts.copy()
    cnt[0, 0, 0] = 1.0   # bin far from the line: mu underflows to exactly 0
    v, st = orc.Oracle(M.replace(counts=cnt)).nll(np.array([1.0, 10.0, 0.0]))
    assert v == math.inf and st == 1
    # invalid response: negative quenching constant
    M = gsgen.small_gamma_model(n_true=50, n_reco=20)
    th = M.theta_true.copy()
    th[M.n_species + 1] = -0.01
    assert orc.Oracle(M).nll(th)[1] == 1


def tiny_mu_model(rate):
    """One line at 500 keV, Gaussian response of 10 keV, bins of 10 keV on [0, 1000), one
    count in each of the bins at 565 and 575 keV (6.5 and 7.5 sigma from the line): at
    rate 1e-300 their expectations are ~2.7e-310 and ~2.5e-313, below FP64's normal range."""
    M = _line_model(GAUSS_E, 500.0, np.array([10.0, 0.0]), np.linspace(0.0, 1000.0, 101), rate=rate)
    cnt = np.zeros_like(M.counts)
    cnt[0, 56, 0] = cnt[0, 57, 0] = 1.0
    return M.replace(counts=cnt)


@pytest.mark.parametrize("rate", [1e-300, 1e-290])
def test_tiny_mu_gives_the_finite_poisson_term(orc, rate):
    """Eq.4 (reading R2): every mu > 0 contributes mu - n ln mu, however small mu is.  At
    rate 1e-300 two bins with one count hold mu ~ 1e-310: -ln L is finite and equals the
    sum written out in 60-digit arithmetic from the oracle's own FP64 expectations (which
    are themselves checked against scipy's normal density); the FP64 gradient seed 1 - n/mu
    overflows there, so the status is GRAD_RANGE and the gradient NaN.  At rate 1e-290 the
    seeds fit FP64 and the rate gradient is the closed form sum_j F_j - sum_j n_j / R (rate
    linearity)."""
    M = tiny_mu_model(rate)
    o = orc.Oracle(M)
    th = M.theta_true
    mu = o.expected(th)[0, :, 0]
    x = np.arange(100) * 10.0 + 5.0
    ref_mu = rate * 10.0 * stats.norm.pdf(x, 500.0, 10.0)
    big = ref_mu > 1e-320
    assert np.max(np.abs(mu[big] - ref_mu[big]) / ref_mu[big]) <= 1e-12
    mpmath.mp.dps = 60
    n = M.counts[0, :, 0]
    ref = mpmath.fsum(mpmath.mpf(float(u)) - (mpmath.mpf(float(k)) * mpmath.log(mpmath.mpf(float(u))) if k else 0)
                      for u, k in zip(mu, n))
    v, g, st = o.nll_grad(th)
    assert np.isfinite(v) and abs(v - float(ref)) <= 1e-15 * abs(float(ref))
    assert o.nll(th) == (v, st)
    if rate == 1e-300:
        assert mu[56] < 1e-308 and mu[57] < 1e-308
        assert st == orc.ST_GRAD_RANGE and np.all(np.isnan(g))
        assert 1420 < v < 1440
    else:
        assert st == 0
        F = mu / rate
        assert g[0] == pytest.approx(F.sum() - n.sum() / rate, rel=1e-12)


# ------------------------------------------------------------ gradient -------
def _richardson(f, th, p, h):
    def d(hh):
        a, b = th.copy(), th.copy()
        a[p] += hh
        b[p] -= hh
        return (f(a) - f(b)) / (2 * hh)
    return (4 * d(h / 2) - d(h)) / 3


@pytest.mark.parametrize("which", ["c0", "gamma", "gauss_pe", "gamma2d"])
def test_gradient_vs_richardson(orc, c0, which):
    """P10: analytic gradient against Richardson-extrapolated central differences at
    off-minimum points: |dg_p| s_p <= 1e-6 max(|g_p| s_p, 1)."""
    if which == "c0":
        M = c0
    elif which == "gamma":
        M = gsgen.small_gamma_model(n_true=200, n_reco=80, seed=2)
    elif which == "gauss_pe":
        M = gsgen.small_gamma_model(n_true=200, n_reco=80, seed=2, family=GAUSS_PE)
    else:
        M = _small2d(orc, n_psd=12, n_datasets=2)[0]
    ps = np.zeros(M.n_params)
    ps[M.n_species + 1] = 2 * M.fd_scale[M.n_species + 1]
    ps[0] = 3 * M.fd_scale[0]
    M = M.replace(pull_sigma=ps, win_lo=2, win_hi=M.n_reco - 1)
    o = orc.Oracle(M)
    for seed in (4, 5):
        th = gsgen.offset_point(M, 2.0, seed=seed)
        v, g, st = o.nll_grad(th)
        assert st == 0
        f = lambda t: o.nll(t)[0]
        for p in range(M.n_params):
            s = M.fd_scale[p]
            fd = _richardson(f, th, p, 0.01 * s)
            assert abs(g[p] - fd) * s <= 1e-6 * max(abs(g[p]) * s, 1.0), (which, p, g[p], fd)


# ------------------------------------------------------------------ fits ----
@pytest.mark.parametrize("which", ["c0", "gamma", "gamma2d"])
def test_asimov_minimum_at_truth(orc, c0, which):
    """P6: with n = mu(theta_true), the gradient vanishes at theta_true, -ln L there is
    sum(mu - mu ln mu), and the fit from theta0 returns theta_true."""
    if which == "c0":
        M = c0
    elif which == "gamma":
        M = gsgen.small_gamma_model(n_true=200, n_reco=80, seed=2)
    else:
        M = _small2d(orc, n_psd=12, n_datasets=2)[0]
    o = orc.Oracle(M)
    mu = o.expected(M.theta_true)
    A = gsgen.asimov(M, mu)
    oa = orc.Oracle(A)
    v, g, st = oa.nll_grad(M.theta_true)
    assert st == 0
    assert np.all(np.abs(g) * M.fd_scale <= 1e-9 * np.abs(mu).sum())
    assert v == pytest.approx(math.fsum((mu - mu * np.log(mu)).ravel()), rel=1e-14)
    th0 = M.theta_true * np.where(np.arange(M.n_params) < M.n_species, 1.08, 0.97)
    if M.n_psd:
        th0[-3:] = [0.01, 1.02, 0.05]
    r = oa.fit(th0)
    assert r["ok"], r
    z = (r["theta"] - M.theta_true) / r["sigma"]
    assert np.all(np.abs(z) < 1e-4), z


def test_fisher_sigma_rates(orc, c0):
    """At an Asimov point with only rates free, sigma^2 = diag(I^-1) with the Poisson
    Fisher information I_pq = sum_j dmu_j/dR_p dmu_j/dR_q / mu_j."""
    o = orc.Oracle(c0)
    mu = o.expected(c0.theta_true)
    A = gsgen.asimov(c0, mu)
    free = np.array([1, 1, 1, 0, 0], dtype=np.uint8)
    r = orc.Oracle(A).fit(c0.theta_true * np.array([1.05, 0.95, 1.1, 1, 1]), free=free)
    assert r["ok"]
    F = o.species_fold(c0.theta_true)
    I = (F[:, :, None] * F[:, None, :] / mu[0, :, 0][:, None, None]).sum(axis=0)
    np.testing.assert_allclose(r["sigma"][:3], np.sqrt(np.diag(np.linalg.inv(I))), rtol=1e-6)


def test_pull_adds_inverse_variance(orc, c0):
    """Reading R1 (factor 1/2): a Gaussian pull of width sp adds exactly 1/sp^2 to the
    Hessian, so at an Asimov point with rates free the covariance is inv(I + e e^T/sp^2)."""
    o = orc.Oracle(c0)
    mu = o.expected(c0.theta_true)
    sp = 150.0
    ps = np.zeros(5)
    ps[0] = sp
    A = gsgen.asimov(c0, mu).replace(pull_sigma=ps, pull_centre=c0.theta_true.copy())
    free = np.array([1, 1, 1, 0, 0], dtype=np.uint8)
    r = orc.Oracle(A).fit(c0.theta_true * np.array([1.05, 0.95, 1.1, 1, 1]), free=free)
    assert r["ok"]
    F = o.species_fold(c0.theta_true)
    I = (F[:, :, None] * F[:, None, :] / mu[0, :, 0][:, None, None]).sum(axis=0)
    I[0, 0] += 1 / sp ** 2
    np.testing.assert_allclose(r["sigma"][:3], np.sqrt(np.diag(np.linalg.inv(I))), rtol=1e-6)


def _grid_nll(F, n, rates):
    mu = rates @ F.T  # [N, J]
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(n[None, :] > 0, mu - n[None, :] * np.log(mu), mu)
        t = np.where(mu > 0, t, np.inf)
    return t.sum(axis=1)


@pytest.mark.slow
def test_bruteforce_grid_c0(orc, c0):
    """P7: brute-force grid minimisation of config 0 (response nodes from the oracle fold,
    rates on a dense grid per node, two refinement levels) lands on the oracle fit."""
    o = orc.Oracle(c0)
    fit = o.fit()
    assert fit["ok"]
    sig = fit["sigma"]
    n = c0.counts[0, :, 0]
    centre = c0.theta_true.copy()
    half = 3.0
    for level in range(3):
        na, nrate = (21, 11) if level == 0 else (11, 11)
        ax = [np.linspace(centre[p] - half * sig[p], centre[p] + half * sig[p], na if p >= 3 else nrate)
              for p in range(5)]
        R = np.stack(np.meshgrid(ax[0], ax[1], ax[2], indexing="ij"), axis=-1).reshape(-1, 3)
        best = (np.inf, None)
        for a in ax[3]:
            for b in ax[4]:
                F = o.species_fold(np.array([0, 0, 0, a, b], dtype=float))
                v = _grid_nll(F, n, R)
                i = int(np.argmin(v))
                if v[i] < best[0]:
                    best = (v[i], np.concatenate([R[i], [a, b]]))
        centre = best[1]
        spacing = 2 * half / (np.array([nrate] * 3 + [na] * 2) - 1)
        half = half * 2.0 / (na - 1) * 2
    z = np.abs(centre - fit["theta"]) / sig
    assert np.all(z <= np.maximum(spacing, 0.03)), (z, spacing)
    assert best[0] >= fit["nll"] - 1e-6


@pytest.mark.parametrize("which", ["c0", "gamma"])
def test_fd_fit_agrees_with_analytic_fit(orc, c0, which):
    M = c0 if which == "c0" else gsgen.small_gamma_model(n_true=200, n_reco=80, seed=2)
    o = orc.Oracle(M)
    ra = o.fit()
    rf = o.fit(use_fd=True)
    assert ra["ok"] and rf["ok"]
    assert np.all(np.abs(ra["theta"] - rf["theta"]) <= 1e-3 * ra["sigma"])


# ------------------------------------------------------ discovery test -------
def test_discovery_counting_closed_form(orc, c0):
    """Eq.5 on a one-bin counting experiment: with only the signal rate free (backgrounds and
    response fixed), the free fit reaches mu = n exactly and the null fit has mu = b, the
    backgrounds' expectation, so t = 2 (n ln(n/b) - (n - b)), the textbook closed form of the
    Poisson likelihood ratio (reading: t = 2 (NLL_null - NLL_free) >= 0)."""
    th = c0.theta_true.copy()
    free = np.zeros(c0.n_params, np.uint8)
    free[0] = 1
    bkg = th.copy()
    bkg[0] = 0.0
    mu_b = orc.Oracle(c0).expected(bkg)[0, :, 0]
    # bins where the signal's folded content is large enough to determine its rate (n < b: a negative rate)
    for j, n in ((86, 5200.0), (90, 3000.0), (80, 2500.0), (95, 100.0)):
        cnt = np.zeros_like(c0.counts)
        cnt[0, j, 0] = n
        m = c0.replace(counts=cnt, win_lo=j, win_hi=j + 1)
        r = orc.Oracle(m).discovery(0, theta0=th, free=free)
        assert r["ok"], r
        b = mu_b[j]
        ref = 2.0 * (n * math.log(n / b) - (n - b))
        assert abs(r["t"] - ref) <= 1e-8 * max(1.0, ref), (j, r["t"], ref)
        assert r["theta_null"][0] == 0.0 and np.array_equal(r["theta_null"][1:], th[1:])


def test_discovery_null_distribution_is_chi2(orc):
    """Under the null hypothesis (data without signal) and with the signal rate unbounded, t
    follows the chi-square law with one degree of freedom asymptotically (Wilks): 240 null toys
    of the Gaussian-signal model, rates profiled, against chi2(1) by a Kolmogorov-Smirnov test
    and by its mean (1 +- 4 standard errors); every t >= 0."""
    from concurrent.futures import ThreadPoolExecutor
    toys = gsgen.discovery_toys(240)

    def one(m):
        return orc.Oracle(m).discovery(0, free=m.free_mask())

    with ThreadPoolExecutor(max_workers=8) as ex:
        res = list(ex.map(one, toys))
    assert all(r["ok"] for r in res)
    t = np.array([r["t"] for r in res])
    assert t.min() >= -1e-8
    assert stats.kstest(np.maximum(t, 0.0), stats.chi2(1).cdf).pvalue > 1e-3
    assert abs(t.mean() - 1.0) <= 4.0 * math.sqrt(2.0 / len(t))


# ------------------------------------------------------ Monte Carlo templates ----
def test_template_single_species_closed_form(orc):
    """A template fit with one species: mu_j = R T_j is linear in R, so the maximum-likelihood
    rate is sum_j n_j / sum_j T_j over the window (exposure 1), and -ln L there is
    sum (mu - n ln mu) at that rate."""
    base = gsgen.template_model()
    T_all = base.spectra[6:7].copy()  # the 1.32 MeV beta
    cnt = np.random.default_rng(3).poisson(base.theta_true[6] * T_all[0]).astype(float)[None, :, None]
    m = base.replace(spectra=T_all, line_energy=base.line_energy[6:7], counts=cnt,
                     theta_true=base.theta_true[6:7], theta0=base.theta_true[6:7] * 1.3,
                     pull_centre=base.theta_true[6:7], pull_sigma=np.zeros(1), fd_scale=base.fd_scale[6:7],
                     win_lo=100, win_hi=700)
    r = orc.Oracle(m).fit()
    assert r["ok"]
    T = m.spectra[0, 100:700]
    n = m.counts[0, 100:700, 0]
    R = n.sum() / T.sum()
    sigma = R / math.sqrt(n.sum())  # the Poisson error of the rate
    assert abs(r["theta"][0] - R) <= 1e-3 * sigma
    mu = R * T
    ref = math.fsum(mu - np.where(n > 0, n * np.log(mu), 0.0))
    assert abs(r["nll"] - ref) <= 1e-8


def test_template_equals_analytic_at_fixed_response(orc, c1):
    """Templates equal to the analytic model's own folded spectra at a fixed response give the
    same -ln L and the same rate gradient at any rates (the Monte Carlo fit and the analytic
    fit share the likelihood and differ only in where the spectra come from)."""
    o = orc.Oracle(c1)
    F = o.species_fold(c1.theta_true)  # [n_reco, S], unit rate, bin width included
    S = c1.n_species
    m = c1.replace(family=gsgen.TEMPLATE, n_true=c1.n_reco, e_lo=0.0, e_step=1.0, spectra=np.ascontiguousarray(F.T),
                   line_energy=np.full(S, np.nan), pull_centre=c1.pull_centre[:S], pull_sigma=c1.pull_sigma[:S],
                   theta_true=c1.theta_true[:S], theta0=c1.theta0[:S], fd_scale=c1.fd_scale[:S])
    ot = orc.Oracle(m)
    for seed in (1, 2):
        rates = c1.theta_true[:S] * gsgen._rng(500, 1, seed).uniform(0.8, 1.2, S)
        th = np.concatenate([rates, c1.theta_true[S:]])
        v, g, st = o.nll_grad(th)
        vt, gt, stt = ot.nll_grad(rates)
        assert st == stt == 0
        # the template path rounds F to FP64 once; the analytic path keeps it in long double
        assert vt == pytest.approx(v, rel=1e-14)
        np.testing.assert_allclose(gt, g[:S], rtol=1e-9, atol=1e-9)


# ------------------------------------------ multivariate slice likelihood ----
def _mv_small(slice_width, n_datasets=2, species=None):
    m = gsgen.small_gamma_model(n_true=150, n_reco=60, seed=9, n_psd=13, n_datasets=n_datasets).replace(
        win_lo=3, win_hi=57)
    if species is not None:
        S = m.n_species
        keep = np.r_[species, S:m.n_params]
        m = m.replace(spectra=m.spectra[species:species + 1], line_energy=m.line_energy[species:species + 1],
                      psd_mix=m.psd_mix[species:species + 1], theta_true=m.theta_true[keep],
                      theta0=m.theta0[keep], pull_centre=m.pull_centre[keep], pull_sigma=m.pull_sigma[keep],
                      fd_scale=m.fd_scale[keep])
    return gsgen.multivariate_model(m, slice_width)


def test_mv_single_bin_slices_equal_joint_2d(orc):
    """R17: with one slice per energy bin, the energy likelihood plus the slices' pieces is the
    joint 2-D Poisson likelihood, term by term (a Poisson histogram factorises into the Poisson
    total times the multinomial of its bins): -ln L and the gradient agree."""
    mv = _mv_small(1)
    joint = mv.replace(slice_edges=None)
    for th in (mv.theta_true, gsgen.offset_point(mv, 2.0, seed=4)):
        th = th.copy()
        th[-3:] = (0.03, 1.08, -0.2)
        v, g, st = orc.Oracle(mv).nll_grad(th)
        vj, gj, stj = orc.Oracle(joint).nll_grad(th)
        assert st == stj == 0
        assert v == pytest.approx(vj, rel=1e-13)
        np.testing.assert_allclose(g, gj, rtol=1e-10, atol=1e-8)


def test_mv_slice_piece_one_species_closed_form(orc):
    """With one species the slice's expected pulse-shape shape is the species' own
    probabilities, so each slice contributes -sum_k n_ik ln P_k: -ln L = the energy histogram's
    Poisson terms (the joint expectation summed over pulse-shape bins) + that sum, with P from
    the pulse-shape probabilities (pinned against the mixture's CDFs)."""
    mv = _mv_small(9, species=2)
    o = orc.Oracle(mv)
    th = mv.theta_true.copy()
    th[-3:] = (-0.02, 0.95, 0.3)
    mu = orc.Oracle(mv.replace(slice_edges=None)).expected(th)  # [D][J][K]
    P = o.psd_probs(th)[0]
    ref = []
    for d in range(mv.n_datasets):
        for j in range(mv.win_lo, mv.win_hi):
            n, m_ = mv.counts[d, j].sum(), mu[d, j].sum()
            ref.append(m_ - (n * math.log(m_) if n > 0 else 0.0))
        for i in range(len(mv.slice_edges) - 1):
            nk = mv.counts[d, mv.slice_edges[i]:mv.slice_edges[i + 1]].sum(axis=0)
            ref.extend(-nk[nk > 0] * np.log(P[nk > 0]))
    v, st = o.nll(th)
    assert st == 0 and v == pytest.approx(math.fsum(ref), rel=1e-13)


def test_mv_gradient_vs_richardson(orc):
    mv = _mv_small(7)
    o = orc.Oracle(mv)
    th = gsgen.offset_point(mv, 1.5, seed=6)
    th[-3:] = (0.01, 1.05, 0.1)
    v, g, st = o.nll_grad(th)
    assert st == 0
    f = lambda t: o.nll(t)[0]
    for p in range(mv.n_params):
        fd = _richardson(f, th, p, 1e-4 * mv.fd_scale[p])
        assert abs(g[p] - fd) * mv.fd_scale[p] <= 1e-6 * max(abs(fd) * mv.fd_scale[p], 1.0), (p, g[p], fd)
