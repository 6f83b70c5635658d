"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: S_k, A_k, t, D and u within 1e-10 relative, the gradient within
1e-8 relative, as stated for this path; both sides compute in FP64.  t, D
and u are compared source by source and element-wise (``_parity.rows``), the
gradient as a whole and split by source (J^T applied to one source's
residual column at a time), S_k and A_k entry by entry.  Grids span several dual blocks, truncated last coarse cells
(n mod r != 0), empty upper strips (last coarse cell of 1 or 2 cells), both
boundary modes, 2-D and 3-D.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import _parity as PT
import workloads as W
from oracle import Geometry
from oracle import reduced as R

pytestmark = pytest.mark.gpu

CASES = [
    ((13, 11, 9), (4, 4, 4)),     # truncated last cells on every axis
    ((16, 12, 10), (4, 3, 5)),    # mixed coarsening
    ((17, 9, 12), (8, 3, 4)),     # r = 8 with a 1-cell last coarse cell (empty upper strip)
    ((18, 10, 7), (5, 3, 3)),     # 2-cell last coarse cells
    ((40, 36, 34), (16, 16, 16)), # r = 16: a dual block of 15^3 own cells (generic kernels)
    ((33, 33, 17), (16, 16, 16)), # r = 16 with one full 7^3 block among 15 x 15 x 7 ones (both paths)
    ((24, 24, 40), (8, 8, 16)),   # full 7 x 7 faces in the shape-fixed face launch, 7 x 15 faces generic
    ((40, 36), (16, 16)),         # 2-D r = 16: 15^2 own cells, 4 corners (generic kernels)
    ((32, 32), (4, 4)),           # 2-D
    ((23, 17), (5, 6)),           # 2-D truncated
]
MODES = ["reduced", "lagrange"]


def _torch():
    import torch
    return torch


def _problem(n, r, mode, inst, **kw):
    import paper_1707_07598_amd as msfv
    prob = msfv.Problem(n, r, mode, **kw)
    prob.set_sources(inst.sources)
    prob.set_receivers(inst.receivers)
    return prob


def _csr(rp, col, val, shape):
    return sp.csr_matrix((val, col, rp), shape=shape)


@pytest.mark.parametrize("n,r", CASES)
@pytest.mark.parametrize("mode", MODES)
def test_forward_parity(n, r, mode):
    torch = _torch()
    inst = W.small_instance(n, r, seed=11, ns=3, nr=5)
    g = Geometry(n, r)
    st = R.forward(g, inst.m, inst.sources, inst.receivers, mode)
    prob = _problem(n, r, mode, inst)
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    D, u = prob.forward(m, want_u=True)
    # S_k
    rp, col, val = prob.prolongation()
    P = _csr(rp, col, val, (g.ncell, g.ncoarse)).toarray()
    Pref = st.P.toarray()
    assert np.abs(P - Pref).max() < 1e-10
    PT.rows(P.T, Pref.T, 1e-10, "S_k columns")
    # A_k before the pin, row by row
    (krp, kcol, kval), t = prob.coarse()
    K = _csr(krp, kcol, kval, (g.ncoarse, g.ncoarse)).toarray()
    PT.rows(K, st.K, 1e-10, "A_k rows")
    PT.rows(t, st.t.T, 1e-10, "t")
    PT.rows(D.cpu().numpy(), st.D.T, 1e-10, "D")
    PT.rows(u.cpu().numpy(), st.u.T, 1e-10, "u")
    prob.close()


@pytest.mark.parametrize("n,r", CASES)
@pytest.mark.parametrize("mode", MODES)
def test_gradient_parity(n, r, mode):
    torch = _torch()
    inst = W.small_instance(n, r, seed=12, ns=3, nr=5)
    g = Geometry(n, r)
    st = R.forward(g, inst.m, inst.sources, inst.receivers, mode)
    rng = np.random.default_rng(3)
    V = rng.standard_normal(st.D.shape)
    g_ref = R.jtv(st, V)
    prob = _problem(n, r, mode, inst)
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    prob.forward(m)
    gg = prob.jtv(torch.tensor(V.T.copy(), dtype=torch.float64, device="cuda")).cpu().numpy()
    PT.vector(gg, g_ref, 1e-8, "g")
    PT.gradient_per_source(prob, st, V, 1e-8)
    prob.close()


DEGENERATE = [((4, 4, 4), (4, 4, 4)),  # one coarse vertex, and it is fixed: the solution is zero
              ((8, 3, 5), (4, 3, 5)),  # two coarse vertices, one free
              ((5, 5, 5), (4, 4, 4)),  # 2^3 vertices, 1-cell last coarse cells
              ((9, 7), (4, 3))]        # 2-D, 3 x 3 vertices, no dual blocks of 2 open axes beyond faces


@pytest.mark.parametrize("n,r", DEGENERATE)
@pytest.mark.parametrize("mode", MODES)
def test_degenerate_grids_and_sources(n, r, mode):
    """The smallest grids (down to a single coarse vertex, which is fixed),
    with a source column that cancels within one cell, a column with a
    repeated electrode cell and a two-cell receiver: D, t and the gradient
    match the oracle (zero where the oracle's are zero)."""
    torch = _torch()
    import paper_1707_07598_amd as msfv
    g = Geometry(n, r)
    N = g.ncell
    rng = np.random.default_rng(3)
    m = 0.7 * rng.standard_normal(N)
    src = W.explicit_columns([[(1, 1.0), (N - 2, -1.0)], [(2, 1.0), (2, -1.0)],
                              [(0, 0.5), (0, 0.5), (N - 1, -1.0)]])
    rec = W.explicit_columns([[(0, 1.0)], [(N - 1, 1.0)], [(N // 2, 1.0), (N // 3, -1.0)]])
    st = R.forward(g, m, src, rec, mode)
    V = rng.standard_normal(st.D.shape)
    g_ref = R.jtv(st, V)
    prob = msfv.Problem(n, r, mode)
    prob.set_sources(src)
    prob.set_receivers(rec)
    D = prob.forward(torch.tensor(m, dtype=torch.float64, device="cuda")).cpu().numpy()
    _, t = prob.coarse()
    gg = prob.jtv(torch.tensor(V.T.copy(), dtype=torch.float64, device="cuda")).cpu().numpy()
    PT.rows(D, st.D.T, 1e-10, "D")
    PT.rows(t, st.t.T, 1e-10, "t")
    PT.vector(gg, g_ref, 1e-8, "g")
    PT.gradient_per_source(prob, st, V, 1e-8)
    prob.close()


def test_misfit_gradient_parity():
    torch = _torch()
    n, r = (16, 12, 10), (4, 3, 5)
    inst = W.small_instance(n, r, seed=13, ns=4, nr=6)
    g = Geometry(n, r)
    Dobs = R.forward(g, inst.m_obs, inst.sources, inst.receivers).D
    phi_ref, g_ref, _ = R.misfit_grad(g, inst.m, inst.sources, inst.receivers, Dobs)
    prob = _problem(n, r, "reduced", inst)
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    phi, gg = prob.misfit_grad(m, torch.tensor(Dobs.T.copy(), dtype=torch.float64, device="cuda"))
    assert abs(phi.item() - phi_ref) <= 1e-10 * abs(phi_ref)
    PT.vector(gg.cpu().numpy(), g_ref, 1e-8, "g")
    prob.close()


def test_small_2d_workload_parity():
    """The 2-D 32x32, r = 4 workload (one dipole, 16 receivers)."""
    torch = _torch()
    inst = W.workload_small_2d()
    g = Geometry(inst.n, inst.r)
    st = R.forward(g, inst.m, inst.sources, inst.receivers)
    Dobs = R.forward(g, inst.m_obs, inst.sources, inst.receivers).D
    g_ref = R.jtv(st, st.D - Dobs)
    prob = _problem(inst.n, inst.r, "reduced", inst)
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    D = prob.forward(m)
    PT.rows(D.cpu().numpy(), st.D.T, 1e-10, "D")
    gg = prob.jtv(torch.tensor((st.D - Dobs).T.copy(), dtype=torch.float64, device="cuda"))
    PT.vector(gg.cpu().numpy(), g_ref, 1e-8, "g")
    prob.close()


@pytest.mark.parametrize("n,r,ns", [((40, 36, 32), (4, 4, 4), 1),     # 10 x 9 x 8 vertices
                                    ((40, 36, 32), (4, 4, 4), 20),
                                    ((160, 112), (4, 4), 3),          # 2-D 40 x 28: boxes grow to 8 x 4
                                    ((176, 160), (4, 4), 2),          # 2-D 44 x 40: two consecutive rows a thread
                                    ((172, 160), (4, 4), 2),          # 2-D 43 x 40: rows strided (odd Ncx)
                                    ((64, 64), (3, 4), 4),            # 2-D, 22 x 16
                                    ((128, 64), (4, 4), 3),           # 2-D 32 x 16, odd source count
                                    ((32, 32, 24), (4, 4, 4), 5),     # 8 x 8 x 6
                                    ((516, 256), (4, 4), 3),          # 2-D 129 x 64 > 8192: multi-launch
                                    ((52, 52, 52), (4, 4, 4), 3),     # 13^3: 4 rows a thread, 4 does not divide Ncx
                                    ((68, 68, 68), (4, 4, 4), 2),     # 17^3: 6 rows a thread, 6 does not divide Ncx
                                    ((384, 184), (4, 4), 2),          # 2-D 96 x 46: 6 rows a thread, 6 | Ncx
                                    ((340, 340), (4, 4), 2)])         # 2-D 85 x 85: 8 rows a thread, 8 does not divide Ncx
def test_coarse_preconditioners_parity(n, r, ns):
    """The coarse solvers (two-level aggregate correction, plain Jacobi, and
    the multi-launch Jacobi solver of large grids; above 8192 vertices all
    three run multi-launch, two-level with the aggregate correction) give D,
    t and the gradient of the oracle, and agree with each other."""
    torch = _torch()
    inst = W.small_instance(n, r, seed=17, ns=ns, nr=9)
    g = Geometry(n, r)
    st = R.forward(g, inst.m, inst.sources, inst.receivers)
    V = np.random.default_rng(6).standard_normal(st.D.shape)
    g_ref = R.jtv(st, V)
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    Vd = torch.tensor(V.T.copy(), dtype=torch.float64, device="cuda")
    out = {}
    for pc in ("twolevel", "jacobi", "multi"):
        prob = _problem(n, r, "reduced", inst, coarse_precond=pc)
        D = prob.forward(m).cpu().numpy()
        _, t = prob.coarse()
        gg = prob.jtv(Vd).cpu().numpy()
        out[pc] = (D, t, gg, prob.stats().coarse_max_it)
        PT.rows(D, st.D.T, 1e-10, f"D ({pc})")
        PT.rows(t, st.t.T, 1e-10, f"t ({pc})")
        PT.vector(gg, g_ref, 1e-8, f"g ({pc})")
        prob.close()
    for pc in ("jacobi", "multi"):
        PT.rows(out[pc][0], out["twolevel"][0], 1e-11, f"D twolevel vs {pc}")
        PT.vector(out[pc][2], out["twolevel"][2], 1e-9, f"g twolevel vs {pc}")
    assert out["twolevel"][3] < out["jacobi"][3]


@pytest.mark.parametrize("n,r,mode,precond", [
    ((13, 11, 9), (4, 4, 4), "reduced", "twolevel"),
    ((17, 9, 12), (8, 3, 4), "lagrange", "jacobi"),
    ((13, 11, 9), (4, 4, 4), "reduced", "multi"),
    ((23, 17), (5, 6), "reduced", "twolevel"),
])
def test_forward_jtv_joint_coarse_solve(n, r, mode, precond):
    """msfv_forward_jtv (forward and adjoint coarse problems in one launch of
    2 Ns columns) gives D and J^T v bit for bit equal to msfv_forward then
    msfv_jtv, and D, t and g agree with the oracle; with a frozen basis it
    takes the fixed-basis J^T v."""
    torch = _torch()
    inst = W.small_instance(n, r, seed=18, ns=3, nr=5)
    prob = _problem(n, r, mode, inst, coarse_precond=precond)
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    V = np.random.default_rng(19).standard_normal((inst.receivers.count, inst.sources.count))
    v = torch.tensor(V.T.copy(), device="cuda")
    D1 = prob.forward(m).clone()
    g1 = prob.jtv(v).clone()
    D2, g2 = prob.forward_jtv(m, v)
    assert torch.equal(D1, D2) and torch.equal(g1, g2)
    s = prob.stats()
    assert s.local_noconv == 0 and s.coarse_noconv == 0
    geo = Geometry(n, r)
    st = R.forward(geo, inst.m, inst.sources, inst.receivers, mode=mode)
    _, t = prob.coarse()
    PT.rows(t, st.t.T, 1e-10, "t")
    PT.rows(D2.cpu().numpy(), st.D.T, 1e-10, "D")
    PT.vector(g2.cpu().numpy(), R.jtv(st, V), 1e-8, "g")
    # frozen basis: forward with the frozen rows, then the fixed-basis J^T v
    prob.freeze_basis(True)
    m2 = m + 0.05 * torch.tensor(np.random.default_rng(20).standard_normal(m.shape[0]), device="cuda")
    D3 = prob.forward(m2).clone()
    g3 = prob.jtv(v).clone()
    D4, g4 = prob.forward_jtv(m2, v)
    assert torch.equal(D3, D4) and torch.equal(g3, g4)
    prob.freeze_basis(False)
    prob.close()


def test_determinism_and_stats():
    torch = _torch()
    n, r = (13, 11, 9), (4, 4, 4)
    inst = W.small_instance(n, r, seed=14, ns=2, nr=3)
    prob = _problem(n, r, "reduced", inst)
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    v = torch.ones((2, 3), dtype=torch.float64, device="cuda")
    D1 = prob.forward(m).clone()
    g1 = prob.jtv(v).clone()
    D2 = prob.forward(m).clone()
    g2 = prob.jtv(v).clone()
    assert torch.equal(D1, D2) and torch.equal(g1, g2)
    s = prob.stats()
    assert s.local_noconv == 0 and s.coarse_noconv == 0 and s.nonfinite == 0
    assert s.local_max_it > 0 and s.coarse_max_it > 0
    prob.close()


@pytest.mark.parametrize("precond", ["twolevel", "multi"])
def test_residual_stats(precond):
    """msfv_get_stats reports the final relative residuals of the local and
    coarse solves: within the stop tolerance (1e-13) when every solve
    converged, above it (with the cap hits counted) when the caps cut the
    iterations short."""
    torch = _torch()
    import paper_1707_07598_amd as msfv
    n, r = (13, 11, 9), (4, 4, 4)
    inst = W.small_instance(n, r, seed=17, ns=2, nr=3)
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    v = torch.ones((2, 3), dtype=torch.float64, device="cuda")
    prob = _problem(n, r, "reduced", inst, coarse_precond=precond)
    prob.forward(m)
    prob.jtv(v)
    s = prob.stats()
    assert s.local_noconv == 0 and s.coarse_noconv == 0
    assert 0.0 < s.local_max_res <= 1e-13 and 0.0 < s.coarse_max_res <= 1e-13
    prob.close()
    capped = _problem(n, r, "reduced", inst, coarse_precond=precond, local_maxit=2, coarse_maxit=3)
    with pytest.raises(msfv.MsfvError):
        capped.forward(m)
    s = capped.stats()
    assert s.local_noconv > 0 and s.coarse_noconv > 0
    assert s.local_max_res > 1e-13 and s.coarse_max_res > 1e-13
    assert np.isfinite(s.local_max_res) and np.isfinite(s.coarse_max_res)
    capped.close()


def test_error_paths():
    torch = _torch()
    import paper_1707_07598_amd as msfv
    from paper_1707_07598_amd import _lib
    n, r = (13, 11, 9), (4, 4, 4)
    inst = W.small_instance(n, r, seed=15, ns=2, nr=3)
    prob = _problem(n, r, "reduced", inst)
    v = torch.ones((2, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(msfv.MsfvError) as e:
        prob.jtv(v)
    assert e.value.status == _lib.MSFV_ESTATE
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    bad = m.clone()
    bad[7] = float("nan")
    with pytest.raises(msfv.MsfvError) as e:
        prob.forward(bad)
    assert e.value.status == _lib.MSFV_ENONFINITE
    prob.forward(m)  # recovers
    prob.close()
    capped = _problem(n, r, "reduced", inst, local_maxit=1)
    with pytest.raises(msfv.MsfvError) as e:
        capped.forward(m)
    assert e.value.status == _lib.MSFV_ENOCONV
    capped.close()
    with pytest.raises(msfv.MsfvError) as e:
        msfv.Problem((20, 20, 20), (2, 2, 2))
    assert e.value.status == _lib.MSFV_EINVAL


def test_autograd_function():
    torch = _torch()
    import paper_1707_07598_amd as msfv
    n, r = (13, 11, 9), (4, 4, 4)
    inst = W.small_instance(n, r, seed=16, ns=2, nr=4)
    g = Geometry(n, r)
    Dobs = R.forward(g, inst.m_obs, inst.sources, inst.receivers).D
    prob = _problem(n, r, "reduced", inst)
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda", requires_grad=True)
    dobs = torch.tensor(Dobs.T.copy(), dtype=torch.float64, device="cuda")
    phi = msfv.msfv_misfit(m, prob, dobs)
    phi.backward()
    _, g_ref, _ = R.misfit_grad(g, inst.m, inst.sources, inst.receivers, Dobs)
    PT.vector(m.grad.cpu().numpy(), g_ref, 1e-8, "g")
    # directional finite difference through the Function
    e = torch.tensor(np.random.default_rng(5).standard_normal(g.ncell), device="cuda")
    h = 1e-5
    with torch.no_grad():
        fp = msfv.msfv_misfit(m + h * e, prob, dobs).item()
        fm = msfv.msfv_misfit(m - h * e, prob, dobs).item()
    fd = (fp - fm) / (2 * h)
    assert abs(fd - (m.grad * e).sum().item()) <= 1e-5 * abs(fd)
    prob.close()
