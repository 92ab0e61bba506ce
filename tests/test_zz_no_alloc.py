"""gs_nll_grad_batched_noalloc, the evaluation for callers that cannot allocate: the same
kernels and layout as gs_nll_grad_batched with the partials in the library's fixed workspace,
so its outputs must equal gs_nll_grad_batched's bit for bit.  Two calls in a row on different
batches, the second smaller (the workspace keeps the first call's contents), and a batch whose
partials do not fit, which must be refused."""
import numpy as np
import pytest

import gsgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    import paper_1812_05686_amd as gs
    gs.lib()
    return gs


def _theta(toys, stride, seed):
    th = np.zeros((len(toys), stride))
    for t, m in enumerate(toys):
        th[t, : m.n_params] = m.theta_true + 0.5 * m.fd_scale * gsgen._rng(400 + seed, 1, t).uniform(-1, 1, m.n_params)
    return th


def _compare(gs, toys, seed):
    import torch
    batch = gs.Batch(toys)
    th = torch.tensor(_theta(toys, batch.stride, seed), dtype=torch.float64, device="cuda")
    n0, g0, s0 = batch.nll_grad(th)
    n1 = torch.full_like(n0, np.nan)
    g1 = torch.full_like(g0, np.nan)
    s1 = torch.full_like(s0, -1)
    batch.nll_grad_noalloc(th, n1, g1, s1)
    torch.cuda.synchronize()
    assert (s0 == 0).all() and torch.equal(s0, s1)
    assert torch.equal(n0, n1) and torch.equal(g0, g1)
    return n0.cpu().numpy()


def test_noalloc_matches_batched_two_calls(gs):
    base = gsgen.config1()
    first = gsgen.config3(5, base=base) + [gsgen.small_gamma_model(n_true=150, n_reco=90, seed=9, n_psd=13,
                                                                   n_datasets=2).replace(win_lo=11, win_hi=77)]
    second = gsgen.config3(8, base=base)[5:]  # a smaller batch, 1-D only
    a = _compare(gs, first, 1)
    b = _compare(gs, second, 2)
    assert len(a) == 6 and len(b) == 3 and np.all(np.isfinite(a)) and np.all(np.isfinite(b))


def test_noalloc_refuses_oversized_batch(gs):
    import torch
    base = gsgen.config1()
    batch = gs.Batch([base] * 800)  # one shape; 800 x 4004 cells of adjoint partials exceed the workspace
    th = torch.tensor(np.tile(base.theta_true, (800, 1)), dtype=torch.float64, device="cuda")
    n = torch.empty(800, dtype=torch.float64, device="cuda")
    g = torch.empty(800, batch.stride, dtype=torch.float64, device="cuda")
    s = torch.empty(800, dtype=torch.int32, device="cuda")
    with pytest.raises(gs.GSError, match="status 4"):
        batch.nll_grad_noalloc(th, n, g, s)
