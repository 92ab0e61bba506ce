"""Host-only checks of the C ABI (no GPU needed): every declared entry point is exported
and the descriptor validator rejects malformed input."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import gsgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gs():
    import paper_1812_05686_amd as gs
    if not os.path.exists(gs.LIB_PATH):
        from paper_1812_05686_amd import build
        build.build()
    return gs


def test_every_declared_symbol_is_exported(gs):
    hdr = open(os.path.join(ROOT, "include", "gs.h")).read()
    names = set(re.findall(r"\b(gs_[a-z_]+)\s*\(", hdr))
    assert {"gs_model_create", "gs_nll", "gs_nll_grad", "gs_nll_grad_batched"} <= names
    lib = C.CDLL(gs.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(gs.EXPORTS) == names


def test_validator_accepts_configs(gs, c0):
    assert gs.gs_desc_validate(c0) == 5
    assert gs.gs_desc_validate(gsgen.small_gamma_model(n_true=50, n_reco=20)) == 10
    assert gs.gs_desc_validate(gsgen.small_gamma_model(n_true=50, n_reco=20, n_psd=5, n_datasets=2)) == 13


@pytest.mark.parametrize("mutate,msg", [
    (lambda m: m.replace(win_lo=5, win_hi=5), "window"),
    (lambda m: m.replace(win_hi=m.n_reco + 1), "window"),
    (lambda m: m.replace(reco_edges=m.reco_edges[::-1].copy()), "increasing"),
    (lambda m: m.replace(exposure=np.array([-1.0])), "exposure"),
    (lambda m: m.replace(e_step=0.0), "grid"),
    (lambda m: m.replace(counts=-m.counts), "count"),
    (lambda m: m.replace(family=7), "family"),
    (lambda m: m.replace(spectra=np.zeros((17, m.n_true)), line_energy=np.full(17, np.nan)), "n_species"),
])
def test_validator_rejects(gs, c0, mutate, msg):
    assert gs.gs_desc_validate(mutate(c0)) == -1
    assert msg in gs.gs_last_error()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1812_05686_amd as gs
    monkeypatch.setattr(gs, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gs, "_lib", None)
    with pytest.raises(gs.GSError):
        gs.lib()


def test_validator_templates(gs):
    """Monte Carlo template models: the rates are the only parameters; templates need
    n_true == n_reco, no line species and no secondary observable."""
    t = gsgen.template_model()
    assert gs.gs_desc_validate(t) == t.n_species == 12
    bad = [(t.replace(n_true=t.n_true - 1, spectra=t.spectra[:, :-1].copy()), "n_true == n_reco"),
           (t.replace(line_energy=np.concatenate([[1.0], t.line_energy[1:]])), "line species"),
           (t.replace(psd_edges=np.linspace(0, 1, 4), psd_mix=np.tile([0.5, 0.3, 0.1, 0.6, 0.1], (12, 1)),
                      counts=np.zeros((1, t.n_reco, 3))), "one-dimensional")]
    for m, msg in bad:
        assert gs.gs_desc_validate(m) == -1 and msg in gs.gs_last_error(), msg


def test_validator_rejects_nonfinite_first_edges(gs, c0):
    e = c0.reco_edges.copy()
    e[0] = -np.inf
    assert gs.gs_desc_validate(c0.replace(reco_edges=e)) == -1
    m = gsgen.small_gamma_model(n_true=50, n_reco=20, n_psd=5)
    pe = m.psd_edges.copy()
    pe[-1] = np.inf
    assert gs.gs_desc_validate(m.replace(psd_edges=pe)) == -1
