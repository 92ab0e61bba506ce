"""Python binding of libgs, the MI355X (gfx950) fold likelihood library.

Argument marshalling only: every step of an evaluation runs in the HIP
kernels behind the C ABI declared in include/gs.h.  The binding raises if the
compiled library is missing; there is no CPU fallback.

Low-level names mirror the C ABI (gs_model_create, gs_nll, gs_nll_grad,
gs_expected, gs_fit, gs_batch_create, gs_nll_grad_batched, gs_fit_batched);
`Model`, `Batch` and `GSNLL` wrap them for numpy / torch callers.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgs.so")

GS_OK, GS_ERR_ARG, GS_ERR_DEVICE, GS_ERR_OOM, GS_ERR_UNSUPPORTED = range(5)
ST_DOMAIN, ST_NONFINITE, ST_LS_FAIL, ST_MAXITER, ST_BFGS_RESET, ST_CONVERGED = 1, 2, 4, 8, 16, 32
ST_GRAD_RANGE, ST_UNRESOLVED = 64, 128
GAUSS_E, GAUSS_PE, GAMMA_PE, TEMPLATE = 0, 1, 2, 3
GENGAMMA_PE, SPOIS_PE, EMG_PE = 4, 5, 6  # generalized gamma, scaled Poisson, modified Gaussian

_dp = C.POINTER(C.c_double)


class gs_model_desc(C.Structure):
    _fields_ = [("n_true", C.c_int32), ("e_lo", C.c_double), ("e_step", C.c_double),
                ("n_species", C.c_int32), ("spectra", _dp), ("line_energy", _dp),
                ("n_reco", C.c_int32), ("reco_edges", _dp), ("n_psd", C.c_int32),
                ("psd_edges", _dp), ("psd_mix", _dp), ("n_datasets", C.c_int32),
                ("exposure", _dp), ("counts", _dp), ("win_lo", C.c_int32), ("win_hi", C.c_int32),
                ("family", C.c_int32), ("birks_A", C.c_double), ("pull_centre", _dp),
                ("pull_sigma", _dp), ("n_slices", C.c_int32), ("slice_edges", C.POINTER(C.c_int32)),
                ("exact_bins", C.c_int32), ("shape", C.c_double)]


def _slices(m):
    se = getattr(m, "slice_edges", None)
    return None if se is None else np.ascontiguousarray(se, dtype=np.int32)


def _sptr(se):
    return None if se is None else se.ctypes.data_as(C.POINTER(C.c_int32))


class gs_fit_opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("edm_tol", C.c_double), ("use_fd", C.c_int32),
                ("scale", _dp), ("free_mask", C.POINTER(C.c_uint8)), ("hesse", C.c_int32)]


class gs_fit_result(C.Structure):
    _fields_ = [("nll", C.c_double), ("edm", C.c_double), ("iters", C.c_int32),
                ("n_eval", C.c_int32), ("status", C.c_uint32)]


EXPORTS = ["gs_last_error", "gs_desc_validate", "gs_model_create", "gs_model_destroy", "gs_model_num_params",
           "gs_nll", "gs_nll_grad", "gs_expected", "gs_fit", "gs_batch_create", "gs_batch_destroy",
           "gs_batch_num_toys", "gs_batch_param_stride", "gs_nll_grad_batched", "gs_fit_batched",
           "gs_batch_set_profiling", "gs_batch_kernel_times", "gs_batch_set_log_cut", "gs_model_set_log_cut",
           "gs_batch_mesh_pairs", "gs_species_spectra", "gs_psd_probs", "gs_batch_fit_trace",
           "gs_batch_set_layout", "gs_batch_autotune", "gs_batch_layout", "gs_nll_grad_batched_noalloc",
           "gs_discovery_batched"]
KERNELS = ["cells", "fold", "nll", "adj", "grad", "folds", "reduce_f", "nll_f", "qn", "finish", "adj_s", "tmpl"]

_lib = None


class GSError(RuntimeError):
    pass


def lib():
    """Load libgs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GSError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # One HIP runtime per process: torch bundles its own libamdhip64 (same soname), so
        # load it first and libgs binds to it; device pointers and streams are then shared.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.gs_last_error.restype = C.c_char_p
        L.gs_desc_validate.restype = C.c_int32
        L.gs_desc_validate.argtypes = [C.POINTER(gs_model_desc)]
        L.gs_model_create.restype = C.c_int
        L.gs_model_create.argtypes = [C.POINTER(gs_model_desc), C.c_int32, C.POINTER(vp)]
        L.gs_model_destroy.argtypes = [vp]
        L.gs_model_num_params.restype = C.c_int32
        L.gs_model_num_params.argtypes = [vp]
        L.gs_nll.restype = C.c_int
        L.gs_nll.argtypes = [vp, _dp, _dp, C.POINTER(C.c_uint32)]
        L.gs_nll_grad.restype = C.c_int
        L.gs_nll_grad.argtypes = [vp, _dp, _dp, _dp, C.POINTER(C.c_uint32)]
        L.gs_expected.restype = C.c_int
        L.gs_expected.argtypes = [vp, _dp, _dp]
        L.gs_fit.restype = C.c_int
        L.gs_fit.argtypes = [vp, _dp, C.POINTER(gs_fit_opts), _dp, _dp, C.POINTER(gs_fit_result)]
        L.gs_batch_create.restype = C.c_int
        L.gs_batch_create.argtypes = [C.POINTER(gs_model_desc), C.c_int32, C.c_int32, C.POINTER(vp)]
        L.gs_batch_destroy.argtypes = [vp]
        L.gs_batch_num_toys.restype = C.c_int32
        L.gs_batch_num_toys.argtypes = [vp]
        L.gs_batch_param_stride.restype = C.c_int32
        L.gs_batch_param_stride.argtypes = [vp]
        L.gs_nll_grad_batched.restype = C.c_int
        L.gs_nll_grad_batched.argtypes = [vp, vp, vp, vp, vp, vp]
        L.gs_nll_grad_batched_noalloc.restype = C.c_int
        L.gs_nll_grad_batched_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
        L.gs_discovery_batched.restype = C.c_int
        L.gs_discovery_batched.argtypes = [vp, vp, vp, vp, vp, C.POINTER(gs_fit_opts), vp, vp, vp, vp, vp, vp, vp, vp]
        L.gs_fit_batched.restype = C.c_int
        L.gs_fit_batched.argtypes = [vp, vp, vp, vp, C.POINTER(gs_fit_opts), vp, vp, vp, vp, vp, vp]
        L.gs_batch_set_profiling.restype = C.c_int
        L.gs_batch_set_profiling.argtypes = [vp, C.c_int32]
        L.gs_batch_kernel_times.restype = C.c_int
        L.gs_batch_kernel_times.argtypes = [vp, _dp, C.POINTER(C.c_int64), C.c_int32]
        L.gs_batch_set_log_cut.restype = C.c_int
        L.gs_batch_set_log_cut.argtypes = [vp, C.c_double]
        L.gs_model_set_log_cut.restype = C.c_int
        L.gs_model_set_log_cut.argtypes = [vp, C.c_double]
        L.gs_species_spectra.restype = C.c_int
        L.gs_species_spectra.argtypes = [vp, _dp, _dp]
        L.gs_psd_probs.restype = C.c_int
        L.gs_psd_probs.argtypes = [vp, _dp, _dp]
        L.gs_batch_mesh_pairs.restype = C.c_int
        L.gs_batch_mesh_pairs.argtypes = [vp, C.POINTER(C.c_int64)]
        L.gs_batch_fit_trace.restype = C.c_int
        L.gs_batch_fit_trace.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_int32,
                                         C.POINTER(C.c_int32)]
        L.gs_batch_set_layout.restype = C.c_int
        L.gs_batch_set_layout.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.gs_batch_autotune.restype = C.c_int
        L.gs_batch_autotune.argtypes = [vp, vp, vp, vp, vp, C.c_int32, vp, _dp]
        L.gs_batch_layout.restype = C.c_int
        L.gs_batch_layout.argtypes = [vp, C.POINTER(C.c_int32)]
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != GS_OK:
        raise GSError(f"{what} failed with status {status}: {lib().gs_last_error().decode()}")


def _arr(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def make_desc(m):
    """Marshal a model description (any object with the gsgen.Model fields) into the C struct.
    Returns (desc, keepalive) -- keep `keepalive` referenced while the struct is used."""
    keep = [_arr(m.spectra), _arr(m.line_energy), _arr(m.reco_edges), _arr(m.psd_edges), _arr(m.psd_mix),
            _arr(m.exposure), _arr(m.counts), _arr(m.pull_centre), _arr(m.pull_sigma), _slices(m)]
    sp, le, re_, pe, pm, ex, cn, pc, ps, se = keep
    d = gs_model_desc(int(m.n_true), float(m.e_lo), float(m.e_step), int(sp.shape[0]), _ptr(sp), _ptr(le),
                      int(len(re_) - 1), _ptr(re_), 0 if pe is None else int(len(pe) - 1), _ptr(pe), _ptr(pm),
                      int(len(ex)), _ptr(ex), _ptr(cn), int(m.win_lo), int(m.win_hi), int(m.family),
                      float(m.birks_A), _ptr(pc), _ptr(ps), 0 if se is None else len(se) - 1, _sptr(se),
                      int(getattr(m, "exact_bins", 0)), float(getattr(m, "shape", 0.0)))
    return d, keep


def gs_desc_validate(m) -> int:
    d, keep = make_desc(m)
    return lib().gs_desc_validate(C.byref(d))


def gs_last_error() -> str:
    return lib().gs_last_error().decode()


class Model:
    """One fit problem on one GPU (gs_model_create)."""

    def __init__(self, m, device: int = 0):
        self.desc_src = m
        d, keep = make_desc(m)
        h = C.c_void_p()
        _check(lib().gs_model_create(C.byref(d), device, C.byref(h)), "gs_model_create")
        self.h = h
        self.P = lib().gs_model_num_params(h)
        self.n_mu = int(len(m.exposure)) * (m.win_hi - m.win_lo) * max(0 if m.psd_edges is None else len(m.psd_edges) - 1, 1)

    def close(self):
        if self.h:
            lib().gs_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_log_cut(self, log_cut: float):
        _check(lib().gs_model_set_log_cut(self.h, float(log_cut)), "gs_model_set_log_cut")

    def nll(self, theta):
        th = _arr(theta)
        v, st = C.c_double(), C.c_uint32()
        _check(lib().gs_nll(self.h, _ptr(th), C.byref(v), C.byref(st)), "gs_nll")
        return v.value, st.value

    def nll_grad(self, theta):
        th = _arr(theta)
        v, st = C.c_double(), C.c_uint32()
        g = np.zeros(self.P)
        _check(lib().gs_nll_grad(self.h, _ptr(th), C.byref(v), _ptr(g), C.byref(st)), "gs_nll_grad")
        return v.value, g, st.value

    def expected(self, theta):
        th = _arr(theta)
        mu = np.zeros(self.n_mu)
        _check(lib().gs_expected(self.h, _ptr(th), _ptr(mu)), "gs_expected")
        return mu

    def species_spectra(self, theta):
        m = self.desc_src
        F = np.zeros((m.win_hi - m.win_lo, m.spectra.shape[0]))
        _check(lib().gs_species_spectra(self.h, _ptr(_arr(theta)), _ptr(F)), "gs_species_spectra")
        return F

    def psd_probs(self, theta):
        m = self.desc_src
        P = np.zeros((m.spectra.shape[0], len(m.psd_edges) - 1))
        _check(lib().gs_psd_probs(self.h, _ptr(_arr(theta)), _ptr(P)), "gs_psd_probs")
        return P

    def fit(self, theta0, scale, use_fd=False, max_iter=500, edm_tol=1e-9, free=None, hesse=True):
        th0, sc = _arr(theta0), _arr(scale)
        fm = None if free is None else np.ascontiguousarray(free, dtype=np.uint8)
        o = gs_fit_opts(max_iter, edm_tol, int(use_fd), _ptr(sc),
                        None if fm is None else fm.ctypes.data_as(C.POINTER(C.c_uint8)), int(hesse))
        th, sg, r = np.zeros(self.P), np.zeros(self.P), gs_fit_result()
        _check(lib().gs_fit(self.h, _ptr(th0), C.byref(o), _ptr(th), _ptr(sg), C.byref(r)), "gs_fit")
        return dict(theta=th, sigma=sg, nll=r.nll, edm=r.edm, iters=r.iters, n_eval=r.n_eval, status=r.status,
                    ok=bool(r.status & ST_CONVERGED))


class Batch:
    """Many fit problems evaluated / fitted together (gs_batch_create).  Batched calls take
    torch CUDA (HIP) tensors and run on torch's current stream."""

    def __init__(self, models, device: int = 0):
        descs = (gs_model_desc * len(models))()
        self._keep = []
        # toys built from the same arrays share device structure: marshal each distinct array once
        cache = {}

        def shared(a):
            if a is None:
                return None
            key = id(a)
            if key not in cache:
                cache[key] = _arr(a)
            return cache[key]

        for t, m in enumerate(models):
            arrs = [shared(m.spectra), shared(m.line_energy), shared(m.reco_edges), shared(m.psd_edges),
                    shared(m.psd_mix), _arr(m.exposure), _arr(m.counts), _arr(m.pull_centre), _arr(m.pull_sigma),
                    _slices(m)]
            self._keep.append(arrs)
            sp, le, re_, pe, pm, ex, cn, pc, ps, se = arrs
            descs[t] = gs_model_desc(int(m.n_true), float(m.e_lo), float(m.e_step), int(sp.shape[0]), _ptr(sp),
                                     _ptr(le), int(len(re_) - 1), _ptr(re_), 0 if pe is None else int(len(pe) - 1),
                                     _ptr(pe), _ptr(pm), int(len(ex)), _ptr(ex), _ptr(cn), int(m.win_lo),
                                     int(m.win_hi), int(m.family), float(m.birks_A), _ptr(pc), _ptr(ps),
                                     0 if se is None else len(se) - 1, _sptr(se),
                                     int(getattr(m, "exact_bins", 0)), float(getattr(m, "shape", 0.0)))
        h = C.c_void_p()
        _check(lib().gs_batch_create(descs, len(models), device, C.byref(h)), "gs_batch_create")
        self._keep = None  # the library copied everything
        self.h = h
        self.n = lib().gs_batch_num_toys(h)
        self.stride = lib().gs_batch_param_stride(h)
        self.device = device

    def close(self):
        if self.h:
            lib().gs_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stream():
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def nll_grad(self, theta, nll=None, grad=None, status=None):
        """theta: torch float64 [n, stride] on the batch device.  Returns (nll, grad, status) tensors."""
        import torch
        assert theta.dtype == torch.float64 and theta.is_cuda and theta.is_contiguous()
        assert tuple(theta.shape) == (self.n, self.stride)
        dev = theta.device
        nll = torch.empty(self.n, dtype=torch.float64, device=dev) if nll is None else nll
        grad = torch.empty(self.n, self.stride, dtype=torch.float64, device=dev) if grad is None else grad
        status = torch.empty(self.n, dtype=torch.int32, device=dev) if status is None else status
        _check(lib().gs_nll_grad_batched(self.h, C.c_void_p(theta.data_ptr()), C.c_void_p(nll.data_ptr()),
                                         C.c_void_p(grad.data_ptr()), C.c_void_p(status.data_ptr()),
                                         self._stream()), "gs_nll_grad_batched")
        return nll, grad, status

    def nll_grad_noalloc(self, theta, nll, grad, status):
        """gs_nll_grad_batched_noalloc into caller-provided tensors (the library's fixed
        workspace holds the partials; nothing is allocated)."""
        import torch
        assert theta.dtype == torch.float64 and theta.is_cuda and theta.is_contiguous()
        assert tuple(theta.shape) == (self.n, self.stride)
        _check(lib().gs_nll_grad_batched_noalloc(self.h, C.c_void_p(theta.data_ptr()), C.c_void_p(nll.data_ptr()),
                                                 C.c_void_p(grad.data_ptr()), C.c_void_p(status.data_ptr()),
                                                 self._stream()), "gs_nll_grad_batched_noalloc")
        return nll, grad, status

    def set_log_cut(self, log_cut: float):
        _check(lib().gs_batch_set_log_cut(self.h, float(log_cut)), "gs_batch_set_log_cut")

    def layout(self):
        """The work layout in force: {target_wg, grad_cells, iter2, adj_waves, candidates}."""
        out = (C.c_int32 * 5)()
        _check(lib().gs_batch_layout(self.h, out), "gs_batch_layout")
        return dict(target_wg=int(out[0]), grad_cells=int(out[1]), iter2=int(out[2]), adj_waves=int(out[3]),
                    candidates=int(out[4]))

    def set_layout(self, target_wg: int, grad_cells: int, iter2: int, adj_waves: int):
        _check(lib().gs_batch_set_layout(self.h, int(target_wg), int(grad_cells), int(iter2), int(adj_waves)),
               "gs_batch_set_layout")

    def autotune(self, theta, reps: int = 3):
        """Times the batched evaluation at theta under every candidate layout and keeps the
        fastest; returns {target_wg, grad_cells, iter2, adj_waves, ms_per_eval}."""
        import torch
        assert theta.dtype == torch.float64 and theta.is_cuda and theta.is_contiguous()
        assert tuple(theta.shape) == (self.n, self.stride)
        dev = theta.device
        nll = torch.empty(self.n, dtype=torch.float64, device=dev)
        grad = torch.empty(self.n, self.stride, dtype=torch.float64, device=dev)
        status = torch.empty(self.n, dtype=torch.int32, device=dev)
        ch = np.zeros(5)
        _check(lib().gs_batch_autotune(self.h, C.c_void_p(theta.data_ptr()), C.c_void_p(nll.data_ptr()),
                                       C.c_void_p(grad.data_ptr()), C.c_void_p(status.data_ptr()), int(reps),
                                       self._stream(), _ptr(ch)), "gs_batch_autotune")
        return dict(target_wg=int(ch[0]), grad_cells=int(ch[1]), iter2=int(ch[2]), adj_waves=int(ch[3]),
                    ms_per_eval=float(ch[4]))

    def mesh_pairs(self):
        """(fold pairs, adjoint pairs, full-mesh pairs, banded-mesh pairs) of the most recent
        evaluation."""
        return self.mesh_counts()[:4]

    def mesh_counts(self):
        """The six counts of gs_batch_mesh_pairs: fold pairs, adjoint pairs, full mesh, banded
        mesh, banded pairs of secondary-observable toys, and those weighted by their cells'
        species count."""
        out = (C.c_int64 * 6)()
        _check(lib().gs_batch_mesh_pairs(self.h, out), "gs_batch_mesh_pairs")
        return tuple(int(out[i]) for i in range(6))

    def fit_trace(self):
        """(active toys, host ms) after each graph launch of the most recent fit."""
        n = C.c_int32(0)
        _check(lib().gs_batch_fit_trace(self.h, None, None, 0, C.byref(n)), "gs_batch_fit_trace")
        a, t = (C.c_int32 * max(n.value, 1))(), (C.c_double * max(n.value, 1))()
        _check(lib().gs_batch_fit_trace(self.h, a, t, n.value, C.byref(n)), "gs_batch_fit_trace")
        return np.array(a[: n.value]), np.array(t[: n.value])

    def set_profiling(self, on: bool):
        _check(lib().gs_batch_set_profiling(self.h, int(on)), "gs_batch_set_profiling")

    def kernel_times(self, reset=True):
        """{kernel: (total_ms, launches)} accumulated while profiling was on."""
        ms = np.zeros(len(KERNELS))
        n = np.zeros(len(KERNELS), dtype=np.int64)
        _check(lib().gs_batch_kernel_times(self.h, _ptr(ms), n.ctypes.data_as(C.POINTER(C.c_int64)), int(reset)),
               "gs_batch_kernel_times")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS)}

    def free_masks(self, models, device="cuda"):
        """uint8 [n, stride] device tensor of the models' free-parameter masks (padding fixed)."""
        import torch
        f = np.zeros((self.n, self.stride), np.uint8)
        for t, m in enumerate(models):
            fm = m.free_mask()
            f[t, : len(fm)] = fm
        return torch.tensor(f, device=device)

    def scales(self, models, device="cuda"):
        """float64 [n, stride] device tensor of the models' parameter scales (padding 1)."""
        import torch
        sc = np.ones((self.n, self.stride))
        for t, m in enumerate(models):
            sc[t, : m.n_params] = m.fd_scale
        return torch.tensor(sc, dtype=torch.float64, device=device)

    def fit(self, theta0, scale, free=None, max_iter=500, edm_tol=1e-9):
        """Device BFGS of every toy from theta0 [n, stride].  scale: one host row [stride] for
        every toy, or a [n, stride] device tensor (one row per toy).  free: optional uint8
        [n, stride] device tensor (1 = parameter may move)."""
        import torch
        dev = theta0.device
        if free is not None:
            free = free.to(device=dev, dtype=torch.uint8).contiguous()
        d_scale = None
        if isinstance(scale, torch.Tensor) and scale.dim() == 2:
            d_scale = scale.to(device=dev, dtype=torch.float64).contiguous()
            scale = np.ones(self.stride)
        th = torch.empty_like(theta0)
        nll = torch.empty(self.n, dtype=torch.float64, device=dev)
        sig = torch.empty_like(theta0)
        iters = torch.empty(self.n, dtype=torch.int32, device=dev)
        st = torch.empty(self.n, dtype=torch.int32, device=dev)
        sc = _arr(scale)
        o = gs_fit_opts(max_iter, edm_tol, 0, _ptr(sc), None, 0)
        fp = C.c_void_p(free.data_ptr()) if free is not None else None
        dsp = C.c_void_p(d_scale.data_ptr()) if d_scale is not None else None
        _check(lib().gs_fit_batched(self.h, C.c_void_p(theta0.data_ptr()), fp, dsp, C.byref(o), C.c_void_p(th.data_ptr()),
                                    C.c_void_p(nll.data_ptr()), C.c_void_p(sig.data_ptr()),
                                    C.c_void_p(iters.data_ptr()), C.c_void_p(st.data_ptr()), self._stream()),
               "gs_fit_batched")
        return dict(theta=th, nll=nll, sigma=sig, iters=iters, status=st)


def discovery(batch, theta0, scale, signal, free=None, max_iter=500, edm_tol=1e-9):
    """Profile-likelihood discovery test of every toy of a Batch (gs_discovery_batched):
    theta0 [n, stride] start, scale [n, stride] device tensor or one host row, signal [n]
    parameter index per toy, free optional uint8 [n, stride].  Returns a dict of tensors:
    t, theta_free, nll_free, status_free, theta_null, nll_null, status_null."""
    import torch
    dev = theta0.device
    n, P = batch.n, batch.stride
    d_scale = None
    if isinstance(scale, torch.Tensor) and scale.dim() == 2:
        d_scale = scale.to(device=dev, dtype=torch.float64).contiguous()
        scale = np.ones(P)
    if free is not None:
        free = free.to(device=dev, dtype=torch.uint8).contiguous()
    sig = torch.as_tensor(np.asarray(signal, dtype=np.int32)).to(dev)
    out = dict(t=torch.empty(n, dtype=torch.float64, device=dev),
               theta_free=torch.empty(n, P, dtype=torch.float64, device=dev),
               nll_free=torch.empty(n, dtype=torch.float64, device=dev),
               status_free=torch.empty(n, dtype=torch.int32, device=dev),
               theta_null=torch.empty(n, P, dtype=torch.float64, device=dev),
               nll_null=torch.empty(n, dtype=torch.float64, device=dev),
               status_null=torch.empty(n, dtype=torch.int32, device=dev))
    sc = _arr(scale)
    o = gs_fit_opts(max_iter, edm_tol, 0, _ptr(sc), None, 0)
    vp = lambda x: None if x is None else C.c_void_p(x.data_ptr())
    _check(lib().gs_discovery_batched(batch.h, vp(theta0), vp(free), vp(d_scale), vp(sig), C.byref(o), vp(out["t"]),
                                      vp(out["theta_free"]), vp(out["nll_free"]), vp(out["status_free"]),
                                      vp(out["theta_null"]), vp(out["nll_null"]), vp(out["status_null"]),
                                      batch._stream()), "gs_discovery_batched")
    return out


def _autograd_fn():
    import torch

    class GSNLL(torch.autograd.Function):
        """-ln L of every toy of a Batch as a differentiable function of theta [n, stride]:
        forward runs the batched fold + likelihood + adjoint kernels once and keeps the
        gradient; backward scales it by the incoming gradient."""

        @staticmethod
        def forward(ctx, theta, batch):
            nll, grad, status = batch.nll_grad(theta.detach().contiguous())
            ctx.save_for_backward(grad)
            ctx.mark_non_differentiable(status)
            return nll, status

        @staticmethod
        def backward(ctx, g_nll, g_status):
            (grad,) = ctx.saved_tensors
            return g_nll[:, None] * grad, None

    return GSNLL


_GSNLL = None


def gsnll(theta, batch):
    """Differentiable batched -ln L: returns (nll [n], status [n])."""
    global _GSNLL
    if _GSNLL is None:
        _GSNLL = _autograd_fn()
    return _GSNLL.apply(theta, batch)
