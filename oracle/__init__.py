"""ctypes wrapper of the CPU oracle (oracle.c) -- TEST INFRASTRUCTURE ONLY.

The oracle is the plain FP64/long-double CPU definition of the binned Poisson
likelihood with analytic response fold (GooStats, arXiv:1812.05686: section
2.3 response, section 2.4 multivariate likelihood, Eq.2 fold cost model,
Eq.4 likelihood).  Only tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package.  It shares no code with the GPU
library; `build()` compiles it with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GS_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

ST_DOMAIN, ST_NONFINITE, ST_LS_FAIL, ST_MAXITER, ST_BFGS_RESET, ST_GRAD_RANGE = 1, 2, 4, 8, 16, 64
GAUSS_E, GAUSS_PE, GAMMA_PE, TEMPLATE, GENGAMMA_PE, SPOIS_PE, EMG_PE = 0, 1, 2, 3, 4, 5, 6


def build(force: bool = True, src: str | None = None, out: str | None = None) -> str:
    """Compile oracle.c into liboracle.so (plain -O2, no fast-math)."""
    src = src or os.path.join(HERE, "oracle.c")
    if out is not None:
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-I", HERE, "-o", out, src, "-lquadmath", "-lm"])
        return out
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-Wall", "-o", tmp, src, "-lquadmath", "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Model(C.Structure):
    _fields_ = [("n_true", C.c_int32), ("e_lo", C.c_double), ("e_step", C.c_double),
                ("n_species", C.c_int32), ("spectra", C.POINTER(C.c_double)),
                ("line_energy", C.POINTER(C.c_double)), ("n_reco", C.c_int32),
                ("reco_edges", C.POINTER(C.c_double)), ("n_psd", C.c_int32),
                ("psd_edges", C.POINTER(C.c_double)), ("psd_mix", C.POINTER(C.c_double)),
                ("n_datasets", C.c_int32), ("exposure", C.POINTER(C.c_double)),
                ("counts", C.POINTER(C.c_double)), ("win_lo", C.c_int32), ("win_hi", C.c_int32),
                ("family", C.c_int32), ("birks_A", C.c_double),
                ("pull_centre", C.POINTER(C.c_double)), ("pull_sigma", C.POINTER(C.c_double)),
                ("n_slices", C.c_int32), ("slice_edges", C.POINTER(C.c_int32)),
                ("exact_bins", C.c_int32), ("shape", C.c_double)]


class _FitOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("edm_tol", C.c_double), ("use_fd", C.c_int32),
                ("scale", C.POINTER(C.c_double)), ("free_mask", C.POINTER(C.c_uint8)),
                ("hesse", C.c_int32)]


class _FitRes(C.Structure):
    _fields_ = [("nll", C.c_double), ("edm", C.c_double), ("iters", C.c_int32),
                ("n_eval", C.c_int32), ("status", C.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_num_params.restype = C.c_int32
        L.orc_quench.restype = C.c_double
        L.orc_quench.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_dquench_dkB.restype = C.c_double
        L.orc_dquench_dkB.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_digamma.restype = C.c_double
        L.orc_digamma.argtypes = [C.c_double]
        L.orc_moments.restype = C.c_int32
        L.orc_moments.argtypes = [C.c_int32, dp, C.c_double, C.c_double, dp, dp]
        L.orc_density.restype = C.c_double
        L.orc_density.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double]
        L.orc_density_dms.restype = None
        L.orc_density_dms.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_density3.restype = C.c_double
        L.orc_density3.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_density_dms3.restype = None
        L.orc_density_dms3.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_bin_content.restype = C.c_int32
        L.orc_bin_content.argtypes = [C.c_int32, C.c_double, C.c_int32, C.c_double, C.c_double, C.c_double,
                                      C.c_double, dp, dp, dp]
        L.orc_igam.restype = C.c_int32
        L.orc_igam.argtypes = [C.c_double, C.c_double, dp, dp, dp]
        for fn in ("orc_species_fold", "orc_psd_probs", "orc_expected"):
            getattr(L, fn).restype = C.c_int32
            getattr(L, fn).argtypes = [C.POINTER(_Model), dp, dp]
        L.orc_nll.restype = C.c_double
        L.orc_nll.argtypes = [C.POINTER(_Model), dp, C.POINTER(C.c_uint32)]
        L.orc_nll_grad.restype = C.c_double
        L.orc_nll_grad.argtypes = [C.POINTER(_Model), dp, dp, C.POINTER(C.c_uint32)]
        L.orc_fit.restype = C.c_int32
        L.orc_fit.argtypes = [C.POINTER(_Model), dp, C.POINTER(_FitOpts), dp, dp, C.POINTER(_FitRes)]
        L.orc_discovery.restype = C.c_int32
        L.orc_discovery.argtypes = [C.POINTER(_Model), dp, C.POINTER(_FitOpts), C.c_int32, dp, dp, dp,
                                    C.POINTER(_FitRes), C.POINTER(_FitRes)]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _c(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Oracle bound to one gsgen.Model (keeps the marshalled arrays alive)."""

    def __init__(self, m):
        self.model = m
        self._keep = [_c(m.spectra), _c(m.line_energy), _c(m.reco_edges), _c(m.psd_edges),
                      _c(m.psd_mix), _c(m.exposure), _c(m.counts), _c(m.pull_centre), _c(m.pull_sigma)]
        sp, le, re_, pe, pm, ex, cn, pc, ps = self._keep
        se = getattr(m, "slice_edges", None)
        se = None if se is None else np.ascontiguousarray(se, dtype=np.int32)
        self._keep.append(se)
        self.s = _Model(m.n_true, m.e_lo, m.e_step, m.n_species, _p(sp), _p(le), m.n_reco, _p(re_),
                        m.n_psd, _p(pe), _p(pm), m.n_datasets, _p(ex), _p(cn), m.win_lo, m.win_hi,
                        m.family, m.birks_A, _p(pc), _p(ps), 0 if se is None else len(se) - 1,
                        None if se is None else se.ctypes.data_as(C.POINTER(C.c_int32)),
                        int(getattr(m, "exact_bins", 0)), float(getattr(m, "shape", 0.0)))
        self.P = lib().orc_num_params(C.byref(self.s))
        assert self.P == m.n_params

    def species_fold(self, theta):
        F = np.zeros((self.model.n_reco, self.model.n_species))
        ok = lib().orc_species_fold(C.byref(self.s), _p(_c(theta)), _p(F))
        return F if ok else None

    def psd_probs(self, theta):
        P = np.zeros((self.model.n_species, self.model.n_psd))
        ok = lib().orc_psd_probs(C.byref(self.s), _p(_c(theta)), _p(P))
        return P if ok else None

    def expected(self, theta):
        mu = np.zeros(self.model.counts.shape)
        lib().orc_expected(C.byref(self.s), _p(_c(theta)), _p(mu))
        return mu

    def nll(self, theta):
        st = C.c_uint32(0)
        v = lib().orc_nll(C.byref(self.s), _p(_c(theta)), C.byref(st))
        return v, st.value

    def nll_grad(self, theta):
        st = C.c_uint32(0)
        g = np.zeros(self.P)
        v = lib().orc_nll_grad(C.byref(self.s), _p(_c(theta)), _p(g), C.byref(st))
        return v, g, st.value

    def fit(self, theta0=None, use_fd=False, max_iter=500, edm_tol=1e-9, free=None, hesse=True, scale=None):
        m = self.model
        th0 = _c(m.theta0 if theta0 is None else theta0)
        sc = _c(m.fd_scale if scale is None else scale)
        fm = None if free is None else np.ascontiguousarray(free, dtype=np.uint8)
        o = _FitOpts(max_iter, edm_tol, int(use_fd), _p(sc),
                     None if fm is None else fm.ctypes.data_as(C.POINTER(C.c_uint8)), int(hesse))
        th = np.zeros(self.P)
        sg = np.zeros(self.P)
        r = _FitRes()
        ok = lib().orc_fit(C.byref(self.s), _p(th0), C.byref(o), _p(th), _p(sg), C.byref(r))
        return dict(ok=bool(ok), theta=th, sigma=sg, nll=r.nll, edm=r.edm, iters=r.iters,
                    n_eval=r.n_eval, status=r.status)


    def discovery(self, signal, theta0=None, free=None, scale=None, max_iter=500, edm_tol=1e-9):
        """Profile-likelihood discovery statistic t = 2 (-ln L_null - -ln L_free) (section 4.2, Eq.5)
        with parameter `signal` fixed at 0 in the null fit."""
        m = self.model
        th0 = _c(m.theta0 if theta0 is None else theta0)
        sc = _c(m.fd_scale if scale is None else scale)
        fm = None if free is None else np.ascontiguousarray(free, dtype=np.uint8)
        o = _FitOpts(max_iter, edm_tol, 0, _p(sc), None if fm is None else fm.ctypes.data_as(C.POINTER(C.c_uint8)), 0)
        t = C.c_double()
        tf, tn = np.zeros(self.P), np.zeros(self.P)
        rf, rn = _FitRes(), _FitRes()
        ok = lib().orc_discovery(C.byref(self.s), _p(th0), C.byref(o), int(signal), C.byref(t), _p(tf), _p(tn),
                                 C.byref(rf), C.byref(rn))
        return dict(ok=bool(ok), t=t.value, theta_free=tf, theta_null=tn, nll_free=rf.nll, nll_null=rn.nll,
                    status_free=rf.status, status_null=rn.status)


def quench(e, kb, a=2.0):
    return lib().orc_quench(e, kb, a)


def dquench_dkb(e, kb, a=2.0):
    return lib().orc_dquench_dkB(e, kb, a)


def digamma(x):
    return lib().orc_digamma(x)


def moments(family, resp, e, birks_a=2.0):
    r = _c(np.asarray(resp))
    m, s = C.c_double(), C.c_double()
    ok = lib().orc_moments(family, _p(r), birks_a, e, C.byref(m), C.byref(s))
    return (m.value, s.value) if ok else None


def density(family, x, m, s):
    return lib().orc_density(family, x, m, s)


def density_dms(family, x, m, s):
    a, b = C.c_double(), C.c_double()
    lib().orc_density_dms(family, x, m, s, C.byref(a), C.byref(b))
    return a.value, b.value


def density3(family, shape, x, m, s):
    """Response density of any family (shape: the generalized gamma's power or the modified
    Gaussian's tail fraction)."""
    return lib().orc_density3(family, shape, x, m, s)


def density_dms3(family, shape, x, m, s):
    a, b = C.c_double(), C.c_double()
    lib().orc_density_dms3(family, shape, x, m, s, C.byref(a), C.byref(b))
    return a.value, b.value


def bin_content(family, shape, exact, xlo, xhi, m, s):
    """(K, dK/dm, dK/ds) of reco bin [xlo, xhi) for a deposit with response moments (m, s), or None."""
    k, a, b = C.c_double(), C.c_double(), C.c_double()
    ok = lib().orc_bin_content(family, shape, int(exact), xlo, xhi, m, s, C.byref(k), C.byref(a), C.byref(b))
    return (k.value, a.value, b.value) if ok else None


def igam(k, u):
    """Regularised incomplete gamma (P, Q, dP/dk)."""
    p, q, d = C.c_double(), C.c_double(), C.c_double()
    lib().orc_igam(k, u, C.byref(p), C.byref(q), C.byref(d))
    return p.value, q.value, d.value
