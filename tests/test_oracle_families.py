"""Pins of the oracle's further response families and exact bin contents against what
mathematics and independent libraries fix (section 2.3 names the families, section 2.5 the
response mesh; the paper gives no formulas, so each family follows the reading stated in the
oracle's header):

* the regularised incomplete gamma and its shape derivative against mpmath;
* the generalized gamma against scipy's Stacy distribution (and the gamma family at p = 1),
  its mean against the moment it is built to match;
* the scaled Poisson against the Poisson probabilities at lattice points, and its missing
  mass against Ramanujan's integral;
* the modified Gaussian against scipy's exponentially modified normal, with its mean and
  variance;
* exact bin contents against adaptive quadrature of the independent library densities, in
  the bulk and in both far tails, and their convergence to the midpoint rule;
* every derivative against Richardson-extrapolated central differences of the oracle's own
  values, and the model gradient against differences of -ln L.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special, stats

import gsgen
import oracle as orc

FAMS = [(orc.GENGAMMA_PE, 0.6), (orc.GENGAMMA_PE, 1.8), (orc.SPOIS_PE, 0.0), (orc.EMG_PE, 0.35)]


def _rich(f, x, h):
    """Richardson-extrapolated central difference."""
    d1 = (f(x + h) - f(x - h)) / (2 * h)
    d2 = (f(x + h / 2) - f(x - h / 2)) / h
    return (4 * d2 - d1) / 3


def _gg_theta(m, s, p):
    k = (m / (p * s)) ** 2
    with mp.workdps(40):
        th = mp.mpf(m) * mp.exp(mp.loggamma(k) - mp.loggamma(k + mp.mpf(1) / p))
    return k, float(th)


# ------------------------------------------------------------ incomplete gamma --
@pytest.mark.parametrize("k", [0.4, 1.0, 3.5, 20.0, 150.0, 1200.0, 9000.0])
def test_incomplete_gamma_against_mpmath(k):
    mp.mp.dps = 50
    us = [k * 0.02, k * 5 + 10] + [k + c * math.sqrt(k) for c in (-6, -2, -0.5, 0.0, 0.7, 2, 6)]
    for u in us:
        if u <= 0:
            continue
        P, Q, dP = orc.igam(k, u)
        Pm = mp.gammainc(k, 0, u, regularized=True)
        Qm = mp.gammainc(k, u, mp.inf, regularized=True)
        dPm = mp.diff(lambda kk: mp.gammainc(kk, 0, u, regularized=True), k)
        if Pm > 1e-290:
            assert abs(P - Pm) <= 1e-13 * Pm, (k, u, P, Pm)
        if Qm > 1e-290:
            assert abs(Q - Qm) <= 1e-13 * Qm, (k, u, Q, Qm)
        if abs(dPm) > 1e-290:
            assert abs(dP - dPm) <= 1e-9 * abs(dPm), (k, u, dP, dPm)


# ------------------------------------------------------------ densities -------
@pytest.mark.parametrize("p", [0.6, 1.0, 1.8])
@pytest.mark.parametrize("m,s", [(60.0, 12.0), (400.0, 25.0)])
def test_generalized_gamma_is_stacy_with_matched_mean(p, m, s):
    k, th = _gg_theta(m, s, p)
    dist = stats.gengamma(k, p, scale=th)
    assert abs(dist.mean() - m) <= 1e-10 * m
    for z in (-3.0, -1.0, 0.0, 0.5, 2.0, 4.0):
        x = m + z * s
        if x <= 0:
            continue
        ref = dist.pdf(x)
        assert abs(orc.density3(orc.GENGAMMA_PE, p, x, m, s) - ref) <= 2e-11 * ref, (p, m, s, z)
    if p == 1.0:  # the gamma family is the unit power
        for z in (-2.0, 0.3, 3.0):
            x = m + z * s
            a, b = orc.density3(orc.GENGAMMA_PE, 1.0, x, m, s), orc.density(orc.GAMMA_PE, x, m, s)
            assert abs(a - b) <= 1e-14 * b
    # the variance is s^2 up to O(1/k)
    assert abs(dist.std() / s - 1.0) <= 2.0 / k


@pytest.mark.parametrize("m,s", [(30.0, 6.0), (400.0, 25.0)])
def test_scaled_poisson_at_lattice_points(m, s):
    g, lam = s * s / m, (m / s) ** 2
    for n in sorted({0, 1, int(lam) - 3, int(lam), int(lam) + 5, int(2 * lam)}):
        if n < 0:
            continue
        ref = stats.poisson.pmf(n, lam)
        got = orc.density3(orc.SPOIS_PE, 0.0, n * g, m, s) * g
        assert abs(got - ref) <= 1e-12 * ref, (m, s, n, got, ref)
    assert orc.density3(orc.SPOIS_PE, 0.0, -1e-9, m, s) == 0.0


def test_scaled_poisson_missing_mass_is_ramanujans():
    """The continued density is not renormalised: its integral over x >= 0 is
    1 - e^-lambda int_0^inf e^(-lambda t) / (t (pi^2 + ln^2 t)) dt."""
    m, s = 5.0, math.sqrt(10.0)  # lambda = 2.5
    lam = (m / s) ** 2
    mp.mp.dps = 30
    mass = mp.quad(lambda x: orc.density3(orc.SPOIS_PE, 0.0, float(x), m, s), [0, 5, 15, 40, 120])
    # J with t = e^u; below u = -60 the factor exp(-lambda e^u) is 1 to 1e-25 and the rest integrates in closed form
    U = mp.mpf(60)
    J = mp.quad(lambda u: mp.exp(-lam * mp.exp(u)) / (mp.pi ** 2 + u ** 2), [-U, -20, -5, 0, 2, 5])
    J += (mp.pi / 2 - mp.atan(U / mp.pi)) / mp.pi
    assert abs(mass - (1 - mp.exp(-lam) * J)) <= 1e-10
    assert 1 - mass > 1e-3  # visibly short of 1 at this lambda


@pytest.mark.parametrize("f", [0.1, 0.35, 0.8])
def test_modified_gaussian_is_exponentially_modified_normal(f):
    m, s = 300.0, 20.0
    sg, tau = s * math.sqrt(1 - f * f), f * s
    dist = stats.exponnorm(tau / sg, loc=m - tau, scale=sg)
    assert abs(dist.mean() - m) <= 1e-9 * m and abs(dist.std() - s) <= 1e-9 * s
    for z in (-6.0, -2.0, 0.0, 1.0, 3.0, 8.0, 15.0):
        x = m + z * s
        ref = dist.pdf(x)
        assert abs(orc.density3(orc.EMG_PE, f, x, m, s) - ref) <= 1e-11 * ref, (f, z)


@pytest.mark.parametrize("fam,shape", FAMS)
def test_density_derivatives_against_differences(fam, shape):
    m, s = 250.0, 18.0
    for z in (-2.5, -0.7, 0.4, 2.2):
        x = m + z * s
        dm, ds = orc.density_dms3(fam, shape, x, m, s)
        fm = _rich(lambda mm: math.log(orc.density3(fam, shape, x, mm, s)), m, 1e-3 * s)
        fs = _rich(lambda ss: math.log(orc.density3(fam, shape, x, m, ss)), s, 1e-3 * s)
        assert abs(dm - fm) <= 1e-7 * (abs(fm) + 1 / s), (fam, z, dm, fm)
        assert abs(ds - fs) <= 1e-7 * (abs(fs) + 1 / s), (fam, z, ds, fs)


# ------------------------------------------------------------ exact bins ------
def _lib_pdf(fam, shape, m, s):
    if fam in (orc.GAUSS_PE, orc.GAUSS_E):
        return stats.norm(m, s).pdf
    if fam == orc.GAMMA_PE:
        return stats.gamma((m / s) ** 2, scale=s * s / m).pdf
    if fam == orc.GENGAMMA_PE:
        k, th = _gg_theta(m, s, shape)
        return stats.gengamma(k, shape, scale=th).pdf
    f = shape
    sg = s * math.sqrt(1 - f * f)
    return stats.exponnorm(f * s / sg, loc=m - f * s, scale=sg).pdf


EXACT = [(orc.GAUSS_PE, 0.0), (orc.GAMMA_PE, 0.0), (orc.GENGAMMA_PE, 0.6), (orc.GENGAMMA_PE, 1.8), (orc.EMG_PE, 0.35)]


@pytest.mark.parametrize("fam,shape", EXACT)
def test_exact_bins_against_quadrature(fam, shape):
    """Bin integrals in the bulk, straddling the mode and in both far tails (where a
    difference of distribution functions taken on the wrong side would cancel to 0)."""
    m, s = 400.0, 22.0
    pdf = _lib_pdf(fam, shape, m, s)
    mp.mp.dps = 30
    for zl, w in ((-0.4, 1.0), (0.6, 0.3), (-2.0, 1.5), (-7.0, 0.8), (5.0, 1.0), (9.0, 0.7)):
        lo, hi = m + zl * s, m + (zl + w) * s
        K, _, _ = orc.bin_content(fam, shape, 1, lo, hi, m, s)
        ref = float(mp.quad(lambda x: pdf(float(x)), [lo, (lo + hi) / 2, hi]))
        assert ref > 0 and abs(K - ref) <= 1e-11 * ref, (fam, zl, K, ref)


@pytest.mark.parametrize("fam,shape", EXACT)
def test_exact_bin_derivatives_and_midpoint_limit(fam, shape):
    m, s = 180.0, 15.0
    lo, hi = m - 0.3 * s, m + 0.5 * s
    K, dm, ds = orc.bin_content(fam, shape, 1, lo, hi, m, s)
    fm = _rich(lambda mm: orc.bin_content(fam, shape, 1, lo, hi, mm, s)[0], m, 1e-3 * s)
    fs = _rich(lambda ss: orc.bin_content(fam, shape, 1, lo, hi, m, ss)[0], s, 1e-3 * s)
    assert abs(dm - fm) <= 1e-7 * abs(K) / s and abs(ds - fs) <= 1e-7 * abs(K) / s
    # exact -> midpoint rule with an O(w^2) error as the bin narrows
    x0 = m + 0.7 * s
    errs = []
    for w in (0.4 * s, 0.2 * s, 0.1 * s):
        Ke = orc.bin_content(fam, shape, 1, x0 - w / 2, x0 + w / 2, m, s)[0]
        Km = orc.bin_content(fam, shape, 0, x0 - w / 2, x0 + w / 2, m, s)[0]
        errs.append(abs(Ke / Km - 1))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_scaled_poisson_has_no_exact_bins():
    assert orc.bin_content(orc.SPOIS_PE, 0.0, 1, 10.0, 11.0, 30.0, 6.0) is None
    assert orc.bin_content(orc.SPOIS_PE, 0.0, 0, 10.0, 11.0, 30.0, 6.0) is not None


# ------------------------------------------------------------ model level -----
@pytest.mark.parametrize("fam,shape,exact", [(orc.GENGAMMA_PE, 1.6, 0), (orc.SPOIS_PE, 0.0, 0), (orc.EMG_PE, 0.35, 0),
                                             (orc.GAMMA_PE, 0.0, 1), (orc.GAUSS_PE, 0.0, 1), (orc.EMG_PE, 0.35, 1),
                                             (orc.GENGAMMA_PE, 0.7, 1)])
def test_model_gradient_against_differences(fam, shape, exact):
    m = gsgen.small_gamma_model(n_true=120, n_reco=48, seed=3, family=fam, shape=shape, exact_bins=exact)
    O = orc.Oracle(m)
    th = gsgen.offset_point(m, 2.0, seed=1)
    v, g, st = O.nll_grad(th)
    assert st == 0 and np.isfinite(v)
    for p in range(m.n_params):
        h = 1e-4 * m.fd_scale[p]
        fd = _rich(lambda x: O.nll(np.where(np.arange(m.n_params) == p, x, th))[0], th[p], h)
        noise = 50 * np.finfo(float).eps * abs(v) / h  # rounding of -ln L in the differences
        assert abs(g[p] - fd) <= 1e-6 * max(abs(fd), 1.0 / m.fd_scale[p]) + noise, (fam, exact, p, g[p], fd)
