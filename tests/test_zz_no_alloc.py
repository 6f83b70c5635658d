"""The allocation-free misfit entry point (msfv_misfit_grad_noalloc) gives
what msfv_misfit_grad gives, on two calls in a row through the C ABI, the
second on a smaller problem (fewer cells, sources and receivers); it
rejects a residual larger than its fixed scratch and a problem whose
electrode tables have not been built yet."""
import numpy as np
import pytest

import _parity as PT
import workloads as W

pytestmark = pytest.mark.gpu


def _problem(n, r, ns, nr, seed):
    import paper_1707_07598_amd as msfv
    inst = W.small_instance(n, r, seed=seed, ns=ns, nr=nr)
    p = msfv.Problem(n, r, "reduced")
    p.set_sources(inst.sources)
    p.set_receivers(inst.receivers)
    return p, inst


def _check_pair(p, inst):
    import torch
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    d_obs = torch.tensor(np.random.default_rng(9).standard_normal((p.ns, p.nr)), device="cuda")
    phi_ref, g_ref = p.misfit_grad(m, d_obs)
    phi_ref, g_ref = phi_ref.clone(), g_ref.clone()
    phi = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    g = torch.full_like(g_ref, np.nan)
    p.misfit_grad_noalloc(m, d_obs, phi, g)
    assert abs(phi.item() - phi_ref.item()) <= 1e-10 * abs(phi_ref.item())
    PT.vector(g.cpu().numpy(), g_ref.cpu().numpy(), 1e-8, "g")
    # same kernels in the same order: bit for bit
    assert torch.equal(phi, phi_ref) and torch.equal(g, g_ref)


def test_noalloc_matches_misfit_grad_twice():
    big, ib = _problem((24, 22, 20), (8, 8, 8), 6, 40, 81)
    small, is_ = _problem((13, 11, 9), (4, 4, 4), 2, 5, 82)
    _check_pair(big, ib)
    _check_pair(small, is_)   # second call: smaller residual, smaller grid
    _check_pair(big, ib)      # and back: nothing carries over from the last call
    big.close()
    small.close()


def test_noalloc_errors():
    import torch
    import paper_1707_07598_amd as msfv
    from paper_1707_07598_amd import _lib
    # electrode tables not built yet: no allocation, so the call refuses
    p, inst = _problem((13, 11, 9), (4, 4, 4), 2, 5, 83)
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    d_obs = torch.zeros((2, 5), dtype=torch.float64, device="cuda")
    phi = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(m.numel(), dtype=torch.float64, device="cuda")
    with pytest.raises(msfv.MsfvError) as e:
        p.misfit_grad_noalloc(m, d_obs, phi, g)
    assert e.value.status == _lib.MSFV_ESTATE
    p.forward(m)
    p.misfit_grad_noalloc(m, d_obs, phi, g)
    p.close()
    # Nr * Ns above the scratch maximum of 65536
    n = (40, 40, 8)
    q = msfv.Problem(n, (4, 4, 4), "reduced")
    q.set_sources(W.surface_dipoles(n, 41))
    q.set_receivers(W.surface_pole_receivers(n, 1600))
    m2 = torch.zeros(int(np.prod(n)), dtype=torch.float64, device="cuda")
    d2 = torch.zeros((41, 1600), dtype=torch.float64, device="cuda")
    g2 = torch.empty_like(m2)
    with pytest.raises(msfv.MsfvError) as e:
        q.misfit_grad_noalloc(m2, d2, phi, g2)
    assert e.value.status == _lib.MSFV_EINVAL
    q.close()
