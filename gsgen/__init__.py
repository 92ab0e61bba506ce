"""Seeded synthetic workloads for the binned Poisson spectral fit.

This module is shared by the CPU oracle tests and the GPU path.  It holds
none of the likelihood arithmetic: it builds the *inputs* of a fit
(true-energy spectra, reco binning, data histograms, windows, starting
points) and simulates data with its own "nature" detector model.

Nature versus the fitted model
------------------------------
The fitted model (section 2.3 and Eq.2 of the paper) evaluates the detector
response at the reco-bin midpoint on the visible-energy x true-energy mesh.
The data here are drawn from exact reco-bin integrals (CDF differences from
scipy.special) of the same synthetic detector, with the quenched light
yield obtained by Gauss-Legendre quadrature of Birks' law rather than a
closed form.  So the data are statistically consistent with the model but
come from different arithmetic; nothing here is compared against either
implementation.

Seeds: numpy SeedSequence([1812, 5686, config, stream, toy]) into PCG64,
stream 0 = data counts, 1 = toy parameters / starting points, 2 = PSD shapes.

Units: the Gaussian-in-energy family (GAUSS_E) uses keV on both axes; the
photoelectron families use MeV on the true axis and photoelectrons (pe) on
the reco axis.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np
from scipy import special

GAUSS_E, GAUSS_PE, GAMMA_PE, TEMPLATE = 0, 1, 2, 3
GENGAMMA_PE, SPOIS_PE, EMG_PE = 4, 5, 6  # generalized gamma, scaled Poisson, modified Gaussian
M_E = 0.51099895  # electron mass, MeV
BIRKS_A = 2.0     # synthetic stopping-power constant, MeV^1.5/cm

_GL_X, _GL_W = np.polynomial.legendre.leggauss(16)


@dataclass
class Model:
    """One fit problem: inputs of the likelihood plus the truth used to make it."""
    name: str
    family: int
    n_true: int
    e_lo: float
    e_step: float
    spectra: np.ndarray          # [S, n_true] float64, row sums 1 (zeros for line species)
    line_energy: np.ndarray      # [S] float64, NaN for grid species
    reco_edges: np.ndarray       # [n_reco + 1]
    exposure: np.ndarray         # [D]
    counts: np.ndarray           # [D, n_reco, max(n_psd, 1)]
    win_lo: int
    win_hi: int
    pull_centre: np.ndarray      # [P]
    pull_sigma: np.ndarray       # [P], <= 0 means no pull
    theta_true: np.ndarray       # [P]
    theta0: np.ndarray           # [P] starting point of fits
    fd_scale: np.ndarray         # [P] parameter scales (FD steps, initial metric)
    birks_A: float = BIRKS_A
    psd_edges: np.ndarray | None = None   # [n_psd + 1]
    psd_mix: np.ndarray | None = None     # [S, 5] = (w1, mean1, sigma1, mean2, sigma2)
    species: list = field(default_factory=list)
    free: np.ndarray | None = None        # [P] bool, parameters a fit may move (None: all)
    slice_edges: np.ndarray | None = None  # [n_slices + 1] energy-bin edges of the multivariate slices
    exact_bins: int = 0          # 1: reco-bin contents are the response's bin integrals
    shape: float = 0.0           # generalized gamma power p / modified Gaussian tail fraction f

    @property
    def n_species(self) -> int:
        return self.spectra.shape[0]

    @property
    def n_reco(self) -> int:
        return len(self.reco_edges) - 1

    @property
    def n_psd(self) -> int:
        return 0 if self.psd_edges is None else len(self.psd_edges) - 1

    @property
    def n_datasets(self) -> int:
        return len(self.exposure)

    @property
    def n_params(self) -> int:
        n_resp = 0 if self.family == TEMPLATE else 2 if self.family == GAUSS_E else 5
        return self.n_species + n_resp + (3 if self.n_psd else 0)

    def replace(self, **kw) -> "Model":
        return dataclasses.replace(self, **kw)

    def free_mask(self) -> np.ndarray:
        """[P] uint8: 1 for parameters a fit may move."""
        return np.ones(self.n_params, np.uint8) if self.free is None else self.free.astype(np.uint8)


def _rng(config: int, stream: int, toy: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1812, 5686, config, stream, toy])))


# ---------------------------------------------------------------- spectra ---
def cell_edges(n_true: int, e_lo: float, e_step: float) -> np.ndarray:
    return e_lo + e_step * np.arange(n_true + 1, dtype=np.float64)


def _normalise(w: np.ndarray) -> np.ndarray:
    w = np.maximum(w, 0.0)
    return w / w.sum()


def spectrum_flat(edges):
    return _normalise(np.diff(edges))


def spectrum_exp(edges, slope):
    return _normalise(slope * (np.exp(-edges[:-1] / slope) - np.exp(-edges[1:] / slope)))


def spectrum_gauss(edges, mean, width):
    return _normalise(special.ndtr((edges[1:] - mean) / width) - special.ndtr((edges[:-1] - mean) / width))


def spectrum_beta(edges, q_value):
    """Allowed beta shape p*E*(Q-T)^2 (T kinetic, E = T + m_e, no Fermi function),
    integrated over each cell with 16-point Gauss-Legendre."""
    a = np.minimum(edges[:-1], q_value)
    b = np.minimum(edges[1:], q_value)
    half = 0.5 * (b - a)
    mid = 0.5 * (b + a)
    t = mid[:, None] + half[:, None] * _GL_X[None, :]
    e_tot = t + M_E
    p = np.sqrt(np.maximum(t * (t + 2 * M_E), 0.0))
    f = p * e_tot * (q_value - t) ** 2
    return _normalise((f * _GL_W[None, :]).sum(axis=1) * half)


# ------------------------------------------------------------------ nature ---
def _nature_light(e_mev: np.ndarray, ly: float, kb: float, birks_a: float) -> np.ndarray:
    """Quenched light LY * int_0^E dE'/(1 + kB*A/sqrt(E')) by Gauss-Legendre in u = sqrt(E')
    (integrand 2u^2/(u + kB*A)), accumulated over [0, sqrt(E)]."""
    c = kb * birks_a
    u_hi = np.sqrt(np.asarray(e_mev, dtype=np.float64))
    # split [0, u_hi] into 8 panels for accuracy at large u
    out = np.zeros_like(u_hi)
    for p in range(8):
        lo = u_hi * p / 8.0
        hi = u_hi * (p + 1) / 8.0
        half = 0.5 * (hi - lo)
        mid = 0.5 * (hi + lo)
        u = mid[..., None] + half[..., None] * _GL_X
        out += (2.0 * u * u / (u + c) * _GL_W).sum(axis=-1) * half
    return ly * out


def _nature_moments(model_family: int, e: np.ndarray, resp: np.ndarray, birks_a: float):
    if model_family == GAUSS_E:
        a, b = resp
        return e.copy(), np.sqrt(a * a + b * e)
    ly, kb, a, b, c = resp
    m = _nature_light(e, ly, kb, birks_a)
    return m, np.sqrt(a * a + b * m + c * c * m * m)


def _nature_bin_probs(family: int, edges: np.ndarray, m: np.ndarray, s: np.ndarray, shape: float = 0.0) -> np.ndarray:
    """[n_reco, n_cells] probability that a deposit with response moments (m, s) lands in each bin.
    The scaled-Poisson family's data are drawn from the gamma law of the same moments."""
    if family in (GAMMA_PE, SPOIS_PE):
        k = (m / s) ** 2
        th = s * s / m
        cdf = special.gammainc(k[None, :], np.maximum(edges, 0.0)[:, None] / th[None, :])
    elif family == GENGAMMA_PE:
        p = shape
        k = (m / (p * s)) ** 2
        th = m * np.exp(special.gammaln(k) - special.gammaln(k + 1.0 / p))
        cdf = special.gammainc(k[None, :], (np.maximum(edges, 0.0)[:, None] / th[None, :]) ** p)
    elif family == EMG_PE:
        from scipy import stats
        f = shape
        sg = s * np.sqrt(1.0 - f * f)
        cdf = stats.exponnorm.cdf(edges[:, None], (f * s / sg)[None, :], loc=(m - f * s)[None, :], scale=sg[None, :])
    else:
        cdf = special.ndtr((edges[:, None] - m[None, :]) / s[None, :])
    return np.diff(cdf, axis=0)


def nature_species_hist(model: Model, resp: np.ndarray) -> np.ndarray:
    """Expected reco histogram [n_reco, S] per unit rate for each species."""
    centres = model.e_lo + model.e_step * (np.arange(model.n_true) + 0.5)
    m, s = _nature_moments(model.family, centres, resp, model.birks_A)
    # chunk the cells to bound memory
    out = np.zeros((model.n_reco, model.n_species))
    grid = np.isnan(model.line_energy)
    for c0 in range(0, model.n_true, 1000):
        sl = slice(c0, min(c0 + 1000, model.n_true))
        pr = _nature_bin_probs(model.family, model.reco_edges, m[sl], s[sl], model.shape)
        out[:, grid] += pr @ model.spectra[grid][:, sl].T
    for sp in np.nonzero(~grid)[0]:
        ml, sl_ = _nature_moments(model.family, np.array([model.line_energy[sp]]), resp, model.birks_A)
        out[:, sp] = _nature_bin_probs(model.family, model.reco_edges, ml, sl_, model.shape)[:, 0]
    return out


def nature_psd_probs(psd_edges: np.ndarray, psd_mix: np.ndarray, nuis=(0.0, 1.0, 0.0)) -> np.ndarray:
    """[S, n_psd] exact bin integrals of the two-Gaussian pulse-shape mixture, renormalised on the range."""
    delta, kappa, eta = nuis
    w1 = psd_mix[:, 0]
    w1 = 1.0 / (1.0 + np.exp(-(np.log(w1 / (1 - w1)) + eta)))
    out = np.zeros((psd_mix.shape[0], len(psd_edges) - 1))
    for comp, w in ((1, w1), (3, 1.0 - w1)):
        mu = psd_mix[:, comp] + delta
        sg = psd_mix[:, comp + 1] * kappa
        cdf = special.ndtr((psd_edges[None, :] - mu[:, None]) / sg[:, None])
        out += w[:, None] * np.diff(cdf, axis=1)
    return out / out.sum(axis=1, keepdims=True)


def nature_expected(model: Model, theta: np.ndarray, species_hist: np.ndarray | None = None) -> np.ndarray:
    """Nature's expected counts [D, n_reco, max(n_psd,1)] at parameters theta."""
    S = model.n_species
    nr = 2 if model.family == GAUSS_E else 5
    if species_hist is None:
        species_hist = nature_species_hist(model, theta[S:S + nr])
    rates = theta[:S]
    if model.n_psd:
        P = nature_psd_probs(model.psd_edges, model.psd_mix, theta[S + nr:S + nr + 3])
        mu1 = np.einsum("js,s,sk->jk", species_hist, rates, P)
    else:
        mu1 = (species_hist @ rates)[:, None]
    return model.exposure[:, None, None] * mu1[None, :, :]


def draw_counts(mu: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    return rng.poisson(mu).astype(np.float64)


# ----------------------------------------------------------------- configs ---
def _scales_pe(S, rates):
    return np.concatenate([np.sqrt(rates), [5.0, 1e-3, 0.4, 0.05, 3e-3]])


def config0() -> Model:
    """Gaussian line + flat + exponential on a 500 x 5 keV true grid, Gaussian response
    sigma^2 = a^2 + b*E, 200 reco bins of 10 keV (the paper's Gaussian-signal-plus-flat
    example, section 4.1, with an exponential added)."""
    edges_t = cell_edges(500, 0.0, 5.0)
    spectra = np.stack([spectrum_gauss(edges_t, 862.0, 1.0), spectrum_flat(edges_t),
                        spectrum_exp(edges_t, 300.0)])
    rates = np.array([5e4, 2e4, 1e4])
    theta = np.concatenate([rates, [10.0, 5.0]])
    m = Model(name="c0", family=GAUSS_E, n_true=500, e_lo=0.0, e_step=5.0, spectra=spectra,
              line_energy=np.full(3, np.nan), reco_edges=10.0 * np.arange(201.0),
              exposure=np.ones(1), counts=np.zeros((1, 200, 1)), win_lo=0, win_hi=200,
              pull_centre=theta.copy(), pull_sigma=np.zeros(5), theta_true=theta,
              theta0=theta * np.array([1.1, 0.9, 1.1, 1.2, 0.8]),
              fd_scale=np.concatenate([np.sqrt(rates), [1.0, 0.5]]),
              species=["gauss862", "flat", "exp300"])
    m.counts = draw_counts(nature_expected(m, theta), _rng(0, 0))
    return m


C1_LINES = [(0.250, 2e4), (0.862, 1e4), (1.460, 5e3), (2.615, 2e3)]
C1_BETAS = [(0.200, 1e5), (0.760, 8e4), (1.320, 5e4), (1.880, 3e4), (2.440, 2e4), (3.000, 1e4)]
C1_EXPS = [(0.150, 4e4), (0.600, 1e4)]
C1_RESP = np.array([500.0, 0.011, 2.0, 1.15, 0.015])


def _c1_shape(n_true=4000, e_step=0.00075, family=GAMMA_PE, lines=C1_LINES, betas=C1_BETAS, exps=C1_EXPS,
              n_reco=900, bin_w=1.6):
    edges_t = cell_edges(n_true, 0.0, e_step)
    rows, le, rates, names = [], [], [], []
    for e0, r in lines:
        rows.append(np.zeros(n_true)); le.append(e0); rates.append(r); names.append(f"line{e0:g}")
    for q, r in betas:
        rows.append(spectrum_beta(edges_t, q)); le.append(np.nan); rates.append(r); names.append(f"beta{q:g}")
    for sl, r in exps:
        rows.append(spectrum_exp(edges_t, sl)); le.append(np.nan); rates.append(r); names.append(f"exp{sl:g}")
    return np.stack(rows), np.array(le), np.array(rates), names, bin_w * np.arange(n_reco + 1.0)


def config1(family: int = GAMMA_PE) -> Model:
    """Borexino-scale: 12 species (4 lines, 6 betas, 2 exponentials) on 4000 x 0.75 keV,
    light yield + Birks quenching + resolution (a, b, c) in photoelectrons, 900 bins of 1.6 pe."""
    spectra, le, rates, names, edges = _c1_shape(family=family)
    S = len(rates)
    theta = np.concatenate([rates, C1_RESP])
    ps = np.zeros(S + 5)
    pc = theta.copy()
    ps[S + 1] = 0.0011   # kB
    ps[S + 2] = 0.4      # a
    ps[S - 1] = 500.0    # rate of the 600 keV exponential background
    m = Model(name="c1" if family == GAMMA_PE else "c1g", family=family, n_true=4000, e_lo=0.0,
              e_step=0.00075, spectra=spectra, line_energy=le, reco_edges=edges,
              exposure=np.ones(1), counts=np.zeros((1, 900, 1)), win_lo=0, win_hi=900,
              pull_centre=pc, pull_sigma=ps, theta_true=theta,
              theta0=theta * _rng(1, 1).uniform(0.9, 1.1, S + 5),
              fd_scale=_scales_pe(S, rates), species=names)
    m.counts = draw_counts(nature_expected(m, theta), _rng(1, 0))
    return m


def config2() -> Model:
    """Config 1 in 2-D (900 energy x 50 pulse-shape bins), 3 datasets with exposures 1:0.6:0.3."""
    base = config1()
    S = base.n_species
    g = _rng(2, 2)
    mix = np.stack([g.uniform(0.3, 0.7, S), g.uniform(0.2, 0.8, S), g.uniform(0.05, 0.15, S),
                    g.uniform(0.2, 0.8, S), g.uniform(0.05, 0.15, S)], axis=1)
    theta = np.concatenate([base.theta_true, [0.0, 1.0, 0.0]])
    pc = np.concatenate([base.pull_centre, [0.0, 1.0, 0.0]])
    ps = np.concatenate([base.pull_sigma, np.zeros(3)])
    m = base.replace(name="c2", psd_edges=np.linspace(0.0, 1.0, 51), psd_mix=mix,
                     exposure=np.array([1.0, 0.6, 0.3]), counts=np.zeros((3, 900, 50)),
                     pull_centre=pc, pull_sigma=ps, theta_true=theta,
                     theta0=np.concatenate([base.theta0, [0.0, 1.0, 0.0]]),
                     fd_scale=np.concatenate([base.fd_scale, [0.01, 0.01, 0.01]]))
    m.counts = draw_counts(nature_expected(m, theta), _rng(2, 0))
    return m


def window_free_params(jac_win: np.ndarray, mu_win: np.ndarray, nominal: np.ndarray, pull_sigma: np.ndarray,
                       max_rel: float = 0.5) -> np.ndarray:
    """Which parameters a fit on this window can determine.

    Rates are unbounded and the resolution only has to stay positive, so a parameter the
    window barely constrains (a rate the window hardly sees; b against c^2 over a narrow
    energy range) drifts until some bin's expectation or some cell's width reaches zero:
    the minimum then lies on the edge of the domain, where a quasi-Newton fit cannot
    converge.  From the Poisson Fisher information at the nominal point (plus the pull
    terms), the parameter whose marginal sigma / |nominal| is largest is fixed while that
    ratio exceeds max_rel.  jac_win: [L, P] d mu / d theta of the window bins; mu_win: [L]."""
    P = len(nominal)
    free = np.ones(P, bool)
    w = 1.0 / np.maximum(mu_win, 1e-300)
    pull = np.where(pull_sigma > 0, 1.0 / np.where(pull_sigma > 0, pull_sigma, 1.0) ** 2, 0.0)
    while free.any():
        idx = np.nonzero(free)[0]
        A = jac_win[:, idx]
        fisher = (A * w[:, None]).T @ A + np.diag(pull[idx])
        try:
            cov = np.linalg.inv(fisher)
            rel = np.sqrt(np.maximum(np.diag(cov), 0.0)) / np.abs(nominal[idx])
            rel[~np.isfinite(rel)] = np.inf
        except np.linalg.LinAlgError:
            rel = 1.0 / np.maximum(np.diag(fisher), 1e-300)
        k = int(np.argmax(rel))
        if rel[k] <= max_rel:
            break
        free[idx[k]] = False
    return free


_JAC_CACHE: dict = {}


def nominal_jacobian(model: Model) -> tuple[np.ndarray, np.ndarray]:
    """Nature's expected 1-D counts mu [n_reco] at the nominal point and d mu / d theta
    [n_reco, S + n_resp] (rates exactly; response parameters by central differences of
    the nature histogram, relative step 1e-4).  Cached per (shape arrays, nominal point)."""
    import hashlib
    h = hashlib.sha256()
    for a in (model.spectra, model.line_energy, model.reco_edges, model.theta_true):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    key = (h.hexdigest(), model.family, model.birks_A, model.n_true, model.e_lo, model.e_step)
    if key in _JAC_CACHE:
        return _JAC_CACHE[key]
    _JAC_CACHE[key] = out = _nominal_jacobian(model)
    return out


def _nominal_jacobian(model: Model) -> tuple[np.ndarray, np.ndarray]:
    S = model.n_species
    th = model.theta_true
    nr = 2 if model.family == GAUSS_E else 5
    hist = nature_species_hist(model, th[S:S + nr])
    mu = hist @ th[:S]
    jac = np.zeros((model.n_reco, S + nr))
    jac[:, :S] = hist
    for q in range(nr):
        h = 1e-4 * abs(th[S + q])
        rp, rm = th[S:S + nr].copy(), th[S:S + nr].copy()
        rp[q] += h
        rm[q] -= h
        jac[:, S + q] = (nature_species_hist(model, rp) @ th[:S] - nature_species_hist(model, rm) @ th[:S]) / (2 * h)
    return mu, jac


def config3(n_toys: int = 4096, base: Model | None = None, full_window: bool = False) -> list[Model]:
    """Toys of config 1: rates drawn +-20% uniform around nominal, response at nominal,
    own contiguous window of L ~ U{200..900} bins starting at lo ~ U{0..900-L} (or the full
    900-bin window); fits start at the config-1 nominal point.  Parameters the window cannot
    determine are fixed at the start value (`free`, see `window_free_params`).  The spectra
    and binning arrays are shared objects."""
    base = config1() if base is None else base
    S = base.n_species
    hist = nature_species_hist(base, base.theta_true[S:])
    mu_nom, jac = nominal_jacobian(base)
    toys = []
    for t in range(n_toys):
        g = _rng(3, 1, t)
        th = base.theta_true.copy()
        th[:S] *= g.uniform(0.8, 1.2, S)
        L = int(g.integers(200, 901))
        lo = int(g.integers(0, 900 - L + 1))
        if full_window:
            lo, L = 0, base.n_reco
        counts = draw_counts(nature_expected(base, th, hist), _rng(3, 0, t))
        free = window_free_params(jac[lo:lo + L], mu_nom[lo:lo + L], base.theta_true, base.pull_sigma)
        toys.append(base.replace(name=f"c3/{t}", counts=counts, win_lo=lo, win_hi=lo + L,
                                 theta_true=th, theta0=base.theta_true.copy(), free=free))
    return toys


# ------------------------------------------------------- mixed batch (c4) ---
C4_A_POOL = [("gauss862", 5e4), ("gauss1460", 2e4), ("flat", 2e4), ("exp300", 1e4), ("exp800", 1e4),
             ("bump1800", 5e3)]
C4_B_LINES = C1_LINES
C4_B_BETAS = [(0.200, 1e5), (0.560, 6e4), (0.760, 8e4), (1.100, 4e4), (1.320, 5e4), (1.880, 3e4), (2.440, 2e4),
              (3.000, 1e4)]
C4_B_EXPS = [(0.150, 4e4), (0.300, 2e4), (0.600, 1e4), (1.000, 5e3)]
C4_B_GRIDS = [(1000, 0.003), (2000, 0.0015), (4000, 0.00075)]


def _c4_a_pool():
    edges_t = cell_edges(500, 0.0, 5.0)
    rows = [spectrum_gauss(edges_t, 862.0, 1.0), spectrum_gauss(edges_t, 1460.0, 2.0), spectrum_flat(edges_t),
            spectrum_exp(edges_t, 300.0), spectrum_exp(edges_t, 800.0), spectrum_gauss(edges_t, 1800.0, 50.0)]
    return np.stack(rows), np.array([r for _, r in C4_A_POOL]), [n for n, _ in C4_A_POOL]


def _pool_jacobian(template: Model, resp: np.ndarray, approx_family: int) -> np.ndarray:
    """d hist_s / d resp_q [n_reco, S, n_resp] by central differences (relative step 1e-4) of the
    nature histogram, computed with approx_family's bin probabilities."""
    t = template.replace(family=approx_family)
    out = np.zeros((template.n_reco, template.n_species, len(resp)))
    for q in range(len(resp)):
        h = 1e-4 * abs(resp[q])
        rp, rm = resp.copy(), resp.copy()
        rp[q] += h
        rm[q] -= h
        out[:, :, q] = (nature_species_hist(t, rp) - nature_species_hist(t, rm)) / (2 * h)
    return out


def _free_from_pool(hist: np.ndarray, jac: np.ndarray, idx, rates_nom, resp_nom, lo, hi, pull_sigma, extra=0):
    """window_free_params for a shape that takes species columns idx of a pool."""
    hw = hist[lo:hi][:, idx]
    jw = np.concatenate([hw, np.einsum("jsq,s->jq", jac[lo:hi][:, idx], rates_nom)], axis=1)
    free = window_free_params(jw, hw @ rates_nom, np.concatenate([rates_nom, resp_nom]), pull_sigma[:jw.shape[1]])
    return np.concatenate([free, np.ones(extra, bool)])


def config4(n_toys: int = 16384, n_shapes_a: int = 8, n_shapes_b: int = 9, fractions=(0.5, 0.4, 0.1)) -> list[Model]:
    """Large uneven batch mixing three kinds of fit problem (seeded class per toy):
      A  small energy-family models: 3-5 species drawn from a 6-shape pool (Gaussian lines, a
         bump, flat, two exponentials) on 500 x 5 keV cells, Gaussian response (a, b), own
         window of 100-200 of 200 bins of 10 keV;
      B  photoelectron-family models like config 1: 6-16 species drawn from a 16-shape pool
         (4 lines, 8 betas, 4 exponentials) on 1000, 2000 or 4000 cells over 0-3 MeV, gamma
         response, own window of 200-900 of 900 bins of 1.6 pe, pulls on kB and a;
      C  the pulse-shape model of config 2 with 1-3 datasets (exposures 1, 0.6, 0.3), full
         window: 45,000-135,000 bins.
    Toys of a class share a pool of shapes (species subset, grid), so toys of one shape share
    their spectra and binning arrays.  Rates are drawn +-20% uniform around nominal; fits start
    at nominal; parameters a window cannot determine are fixed (window_free_params, with the
    Fisher matrix's response derivatives from the Gaussian approximation of the response)."""
    g = _rng(4, 1)
    # --- class A pool
    a_spec, a_rates, a_names = _c4_a_pool()
    a_resp = np.array([10.0, 5.0])
    a_tmpl = Model(name="c4a", family=GAUSS_E, n_true=500, e_lo=0.0, e_step=5.0, spectra=a_spec,
                   line_energy=np.full(6, np.nan), reco_edges=10.0 * np.arange(201.0), exposure=np.ones(1),
                   counts=np.zeros((1, 200, 1)), win_lo=0, win_hi=200, pull_centre=np.zeros(8),
                   pull_sigma=np.zeros(8), theta_true=np.concatenate([a_rates, a_resp]),
                   theta0=np.concatenate([a_rates, a_resp]), fd_scale=np.ones(8), species=a_names)
    a_hist = nature_species_hist(a_tmpl, a_resp)
    a_jac = _pool_jacobian(a_tmpl, a_resp, GAUSS_E)
    a_shapes = []
    for q in range(n_shapes_a):
        idx = np.sort(g.choice(6, size=int(g.integers(3, 6)), replace=False))
        a_shapes.append((idx, np.ascontiguousarray(a_spec[idx]), np.full(len(idx), np.nan), a_tmpl.reco_edges))
    # --- class B pools, one per grid
    b_pool = []
    for n_true, step in C4_B_GRIDS:
        spectra, le, rates, names, edges = _c1_shape(n_true=n_true, e_step=step, lines=C4_B_LINES, betas=C4_B_BETAS,
                                                     exps=C4_B_EXPS)
        S = len(rates)
        tmpl = Model(name="c4b", family=GAMMA_PE, n_true=n_true, e_lo=0.0, e_step=step, spectra=spectra,
                     line_energy=le, reco_edges=edges, exposure=np.ones(1), counts=np.zeros((1, 900, 1)), win_lo=0,
                     win_hi=900, pull_centre=np.zeros(S + 5), pull_sigma=np.zeros(S + 5),
                     theta_true=np.concatenate([rates, C1_RESP]), theta0=np.concatenate([rates, C1_RESP]),
                     fd_scale=_scales_pe(S, rates), species=names)
        b_pool.append((tmpl, nature_species_hist(tmpl, C1_RESP), _pool_jacobian(tmpl, C1_RESP, GAUSS_PE)))
    b_shapes = []
    for q in range(n_shapes_b):
        gi = q % len(C4_B_GRIDS)
        tmpl = b_pool[gi][0]
        idx = np.sort(g.choice(16, size=int(g.integers(6, 17)), replace=False))
        b_shapes.append((gi, idx, np.ascontiguousarray(tmpl.spectra[idx]), np.ascontiguousarray(tmpl.line_energy[idx])))
    # --- class C: the pulse-shape model
    c2 = config2()
    S2 = c2.n_species
    c_hist = nature_species_hist(c2, c2.theta_true[S2:S2 + 5])

    cls = g.choice(3, size=n_toys, p=np.asarray(fractions) / np.sum(fractions))
    toys = []
    for t in range(n_toys):
        gt = _rng(4, 1, 1 + t)
        if cls[t] == 0:
            idx, spec, le, edges = a_shapes[int(gt.integers(n_shapes_a))]
            S = len(idx)
            rates_nom = a_rates[idx]
            theta = np.concatenate([rates_nom * gt.uniform(0.8, 1.2, S), a_resp])
            L = int(gt.integers(100, 201))
            lo = int(gt.integers(0, 200 - L + 1))
            m = Model(name=f"c4/A/{t}", family=GAUSS_E, n_true=500, e_lo=0.0, e_step=5.0, spectra=spec,
                      line_energy=le, reco_edges=edges, exposure=np.ones(1), counts=np.zeros((1, 200, 1)),
                      win_lo=lo, win_hi=lo + L, pull_centre=np.concatenate([rates_nom, a_resp]),
                      pull_sigma=np.zeros(S + 2), theta_true=theta, theta0=np.concatenate([rates_nom, a_resp]),
                      fd_scale=np.concatenate([np.sqrt(rates_nom), [1.0, 0.5]]),
                      species=[a_names[i] for i in idx])
            m.free = _free_from_pool(a_hist, a_jac, idx, rates_nom, a_resp, lo, lo + L, m.pull_sigma)
            m.counts = draw_counts(nature_expected(m, theta, a_hist[:, idx]), _rng(4, 0, t))
        elif cls[t] == 1:
            gi, idx, spec, le = b_shapes[int(gt.integers(n_shapes_b))]
            tmpl, hist, jac = b_pool[gi]
            S = len(idx)
            rates_nom = tmpl.theta_true[:16][idx]
            theta = np.concatenate([rates_nom * gt.uniform(0.8, 1.2, S), C1_RESP])
            L = int(gt.integers(200, 901))
            lo = int(gt.integers(0, 900 - L + 1))
            ps = np.zeros(S + 5)
            ps[S + 1] = 0.0011
            ps[S + 2] = 0.4
            m = Model(name=f"c4/B/{t}", family=GAMMA_PE, n_true=tmpl.n_true, e_lo=0.0, e_step=tmpl.e_step,
                      spectra=spec, line_energy=le, reco_edges=tmpl.reco_edges, exposure=np.ones(1),
                      counts=np.zeros((1, 900, 1)), win_lo=lo, win_hi=lo + L,
                      pull_centre=np.concatenate([rates_nom, C1_RESP]), pull_sigma=ps, theta_true=theta,
                      theta0=np.concatenate([rates_nom, C1_RESP]), fd_scale=_scales_pe(S, rates_nom),
                      species=[tmpl.species[i] for i in idx])
            m.free = _free_from_pool(hist, jac, idx, rates_nom, C1_RESP, lo, lo + L, ps)
            m.counts = draw_counts(nature_expected(m, theta, hist[:, idx]), _rng(4, 0, t))
        else:
            D = int(gt.integers(1, 4))
            theta = c2.theta_true.copy()
            theta[:S2] *= gt.uniform(0.8, 1.2, S2)
            m = c2.replace(name=f"c4/C/{t}", exposure=np.array([1.0, 0.6, 0.3][:D]),
                           counts=np.zeros((D, 900, 50)), theta_true=theta, theta0=c2.theta_true.copy())
            m.counts = draw_counts(nature_expected(m, theta, c_hist), _rng(4, 0, t))
        toys.append(m)
    return toys


def multivariate_model(base: Model | None = None, slice_width: int = 90) -> Model:
    """The multivariate slice likelihood of section 2.4 on the pulse-shape model (config 2 by
    default): the same data, the energy likelihood over the window plus one pulse-shape piece
    per slice of `slice_width` energy bins (the last slice takes the remainder)."""
    base = config2() if base is None else base
    edges = list(range(base.win_lo, base.win_hi, slice_width)) + [base.win_hi]
    return base.replace(name=base.name + "/mv", slice_edges=np.array(edges, dtype=np.int32))


def template_model(flat2d: bool = False, seed: int = 0) -> Model:
    """A Monte Carlo template fit (section 3.2): each species' reco spectrum at unit rate is
    given as a template (here nature's exact bin integrals at the nominal response of the
    Borexino-scale model, i.e. a noiseless Monte Carlo histogram), so the fit has no response
    parameters and no fold.  flat2d: the templates of the pulse-shape model's 900 energy x 50
    pulse-shape bins, flattened to 45,000 bins (one dataset).  Parameters: the 12 rates, with
    the pull of config 1 on the 600 keV exponential's rate."""
    base = config2() if flat2d else config1()
    S = base.n_species
    hist = nature_species_hist(base, base.theta_true[S:S + 5])  # [n_reco, S]
    if flat2d:
        P = nature_psd_probs(base.psd_edges, base.psd_mix)      # [S, K]
        tmpl = np.einsum("js,sk->sjk", hist, P).reshape(S, -1)
    else:
        tmpl = np.ascontiguousarray(hist.T)
    n = tmpl.shape[1]
    rates = base.theta_true[:S]
    ps = np.zeros(S)
    ps[S - 1] = 500.0
    m = Model(name="tmpl2d" if flat2d else "tmpl", family=TEMPLATE, n_true=n, e_lo=0.0, e_step=1.0,
              spectra=np.ascontiguousarray(tmpl), line_energy=np.full(S, np.nan),
              reco_edges=np.arange(n + 1.0), exposure=np.ones(1), counts=np.zeros((1, n, 1)), win_lo=0, win_hi=n,
              pull_centre=rates.copy(), pull_sigma=ps, theta_true=rates.copy(),
              theta0=rates * _rng(7, 1, seed).uniform(0.9, 1.1, S), fd_scale=np.sqrt(rates),
              species=list(base.species))
    m.counts = draw_counts((tmpl.T @ rates)[None, :, None], _rng(7, 0, seed))
    return m


def template_toys(n_toys: int, base: Model | None = None) -> list[Model]:
    """Pseudo-experiments of a template fit: rates drawn +-20% uniform around nominal, own
    Poisson data over the full histogram, fits from the nominal rates; the templates are
    shared arrays."""
    base = template_model() if base is None else base
    mu_s = base.spectra.T  # [n, S]
    toys = []
    for t in range(n_toys):
        g = _rng(8, 1, t)
        th = base.theta_true * g.uniform(0.8, 1.2, base.n_species)
        counts = draw_counts((mu_s @ th)[None, :, None], _rng(8, 0, t))
        toys.append(base.replace(name=f"tmpl/{t}", counts=counts, theta_true=th, theta0=base.theta_true.copy()))
    return toys


def discovery_toys(n_toys: int, base: Model | None = None, signal: int = 0, study: int = 5) -> list[Model]:
    """Pseudo-experiments of the null hypothesis for the discovery test (section 4.2): the base
    model (config 0 by default: a Gaussian line on a flat and an exponential background, the
    paper's signal-plus-background example) with the signal species' rate at zero and data
    drawn per toy; the rates are free, the response parameters fixed at their nominal values;
    fits start at the nominal rates with the signal at zero.  Seeds: study index `study`."""
    base = config0() if base is None else base
    S = base.n_species
    nr = 2 if base.family == GAUSS_E else 5
    th = base.theta_true.copy()
    th[signal] = 0.0
    hist = nature_species_hist(base, th[S:S + nr])
    free = np.zeros(base.n_params, bool)
    free[:S] = True
    toys = []
    for t in range(n_toys):
        counts = draw_counts(nature_expected(base, th, hist), _rng(study, 0, t))
        toys.append(base.replace(name=f"null/{t}", counts=counts, theta_true=th.copy(), theta0=th.copy(),
                                 free=free.copy()))
    return toys


def asimov(model: Model, mu: np.ndarray) -> Model:
    """Same model with data replaced by the given expectation (no fluctuation)."""
    return model.replace(counts=np.asarray(mu, dtype=np.float64).reshape(model.counts.shape).copy())


def small_gamma_model(n_true=300, n_reco=64, seed=7, n_psd=0, n_datasets=1, family=GAMMA_PE, shape=0.0,
                      exact_bins=0, wide=False) -> Model:
    """A small photoelectron-family model (lines, betas, exponentials) that the oracle
    evaluates in milliseconds; used for oracle pins and ragged GPU parity cases.  wide: the
    16 species of the mixed batch's pool (4 lines, 8 betas, 4 exponentials) instead of 5."""
    e_step = 3.0 / n_true
    if wide:
        pools = dict(lines=C4_B_LINES, betas=C4_B_BETAS, exps=C4_B_EXPS)
    else:
        pools = dict(lines=[(0.862, 1e4), (1.46, 5e3)], betas=[(0.76, 5e4), (1.88, 3e4)], exps=[(0.6, 1e4)])
    spectra, le, rates, names, _ = _c1_shape(n_true=n_true, e_step=e_step, family=family, **pools)
    edges = np.linspace(0.0, 1440.0, n_reco + 1)
    S = len(rates)
    theta = np.concatenate([rates, C1_RESP])
    g = _rng(100 + seed, 2)
    m = Model(name=f"small{seed}", family=family, n_true=n_true, e_lo=0.0, e_step=e_step,
              spectra=spectra, line_energy=le, reco_edges=edges, exposure=np.ones(n_datasets),
              counts=np.zeros((n_datasets, n_reco, max(n_psd, 1))), win_lo=0, win_hi=n_reco,
              pull_centre=theta.copy(), pull_sigma=np.zeros(S + 5), theta_true=theta,
              theta0=theta.copy(), fd_scale=_scales_pe(S, rates), species=names, shape=shape,
              exact_bins=exact_bins)
    if n_psd:
        mix = np.stack([g.uniform(0.3, 0.7, S), g.uniform(0.2, 0.8, S), g.uniform(0.05, 0.15, S),
                        g.uniform(0.2, 0.8, S), g.uniform(0.05, 0.15, S)], axis=1)
        m = m.replace(psd_edges=np.linspace(0.0, 1.0, n_psd + 1), psd_mix=mix,
                      exposure=np.array([1.0, 0.6, 0.3][:n_datasets]),
                      theta_true=np.concatenate([theta, [0.0, 1.0, 0.0]]),
                      theta0=np.concatenate([theta, [0.0, 1.0, 0.0]]),
                      pull_centre=np.concatenate([theta, [0.0, 1.0, 0.0]]),
                      pull_sigma=np.zeros(S + 8),
                      fd_scale=np.concatenate([_scales_pe(S, rates), [0.01, 0.01, 0.01]]))
    else:
        m = m.replace(exposure=np.array([1.0, 0.6, 0.3][:n_datasets]))
    m.counts = draw_counts(nature_expected(m, m.theta_true), _rng(100 + seed, 0))
    return m


def offset_point(model: Model, sigma_mult: float = 2.0, seed: int = 0) -> np.ndarray:
    """An off-minimum parameter point theta_true + sigma_mult * scale * u, u ~ U(-1, 1)."""
    u = _rng(200 + seed, 1).uniform(-1.0, 1.0, model.n_params)
    return model.theta_true + sigma_mult * model.fd_scale * u


def family_model(family: int, shape: float = 0.0, exact_bins: int = 0, base: Model | None = None) -> Model:
    """The Borexino-scale model (config 1 shape, 12 species on 4000 cells, 900 bins of 1.6 pe) with
    another response family and/or exact bin contents, its data drawn from nature for that family."""
    base = base or config1()
    m = base.replace(name=f"{base.name}_f{family}" + ("x" if exact_bins else ""), family=family, shape=shape,
                     exact_bins=exact_bins)
    m.counts = draw_counts(nature_expected(m, m.theta_true), _rng(1, 0, 10 + family))
    return m
