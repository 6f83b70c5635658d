"""Projected Gauss-Newton-PCG on a synthetic conductive-block model (the
setting of the paper's block-model experiment, Sec. 5, at test size): data
from the multiscale forward model of the true model with 1 % noise; both the
adaptive and the fixed basis decrease the objective at every step, keep the
bounds, and move the model toward the truth."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("basis", ["adaptive", "fixed"])
def test_gauss_newton_two_block(basis):
    import torch
    import paper_1707_07598_amd as msfv
    from paper_1707_07598_amd.inversion import gauss_newton
    n, r = (24, 24, 12), (4, 4, 4)
    N = int(np.prod(n))
    ids = np.arange(N)
    x, y, z = ids % 24, (ids // 24) % 24, ids // (24 * 24)
    blk = (x >= 8) & (x < 16) & (y >= 8) & (y < 16) & (z >= 2) & (z < 7)
    m_true = np.where(blk, np.log(0.1), np.log(0.01))
    prob = msfv.Problem(n, r, "reduced")
    prob.set_sources(W.surface_dipoles(n, 9))
    prob.set_receivers(W.surface_pole_receivers(n, 100))
    mt = torch.tensor(m_true, device="cuda")
    D = prob.forward(mt).clone()
    noise = torch.tensor(np.random.default_rng(1).standard_normal(D.shape), device="cuda")
    d_obs = D + 0.01 * D.abs().mean() * noise
    m0 = torch.full((N,), float(np.log(0.01)), dtype=torch.float64, device="cuda")
    lo, hi = float(np.log(1e-3)), float(np.log(1.0))
    r0 = prob.forward(m0) - d_obs
    misfit0 = 0.5 * float((r0 * r0).sum())
    m, hist = gauss_newton(prob, m0, d_obs, alpha=1e-3 * float((d_obs * d_obs).sum()) / N,
                           bounds=(lo, hi), max_iter=5, cg_iter=10, basis=basis)
    assert len(hist) >= 3
    obj = [h.objective for h in hist]
    assert all(b < a for a, b in zip(obj, obj[1:]))
    assert hist[-1].misfit < 0.5 * misfit0
    assert float(m.min()) >= lo - 1e-12 and float(m.max()) <= hi + 1e-12
    assert float((m - mt).norm()) < float((m0 - mt).norm())
    s = prob.stats()
    assert s.local_noconv == 0 and s.coarse_noconv == 0
    prob.close()
