"""Pins for the oracle's reduced forward problem and sensitivities.

* Coarsening factor 1 recovers the pinned fine solve (eq. forwardProbFine,
  Sec. 2.2) and the fine adjoint gradient (eq. sens).
* 1-D with sources on vertex cells: the multiscale solution is the fine
  solution (1-D basis functions are exact local solutions).
* A_k: symmetric, A_k 1 = 0 before the pin, 3^d-point pattern; in 1-D it is
  the coarse two-point operator with series transmissibility
  1/T_c = sum 1/T_f (the exact Schur complement).
* Reciprocity of pole data, Galerkin orthogonality of the residual,
  u(m + c 1) = exp(-c) u(m).
* Sensitivities: forward mode (eq. sensred as printed) against central finite
  differences of the forward to 1e-5; transposed form against the forward
  mode (dot test) to 1e-12; the scale identity 1^T g = -sum_j d_j^T v_j;
  fixed-basis forms (eq. senssimple) by dot test; in Lagrange mode with
  every electrode and receiver on the coarse skeleton the adaptive and
  fixed-basis gradients coincide (Y_k vanishes there and S^T A Y_k = 0).
* The fixed-basis surrogate (eq. optredfixed: S_k(m0) held, A_k(m)
  rebuilt) equals the adaptive model at m0, its eq. senssimple derivatives
  match central differences of the surrogate, and its A_k scales with e^c.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import Geometry
from oracle import reduced as R

GRIDS = [((9,), (3,)), ((8, 8), (3, 3)), ((10, 7), (4, 3)), ((7, 5, 6), (3, 2, 3)),
         ((9, 8, 7), (3, 3, 3))]
MODES = ["reduced", "lagrange"]


def _instance(n, r, seed=5):
    return W.small_instance(n, r, seed)


@pytest.mark.parametrize("n", [(9,), (7, 6), (5, 4, 6)])
@pytest.mark.parametrize("mode", MODES)
def test_unit_coarsening_is_fine_solve(n, mode):
    r = (1,) * len(n)
    g = Geometry(n, r)
    inst = _instance(n, r)
    st = R.forward(g, inst.m, inst.sources, inst.receivers, mode)
    fs = R.fine_forward(g, inst.m, inst.sources, inst.receivers)
    np.testing.assert_allclose(st.u, fs.u, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(st.D, fs.D, rtol=1e-12, atol=1e-12)
    V = np.random.default_rng(2).standard_normal(st.D.shape)
    np.testing.assert_allclose(R.jtv(st, V), R.fine_jtv(fs, V), rtol=1e-10, atol=1e-12)


def test_one_dimensional_vertex_sources_exact():
    n, r = (23,), (5,)
    g = Geometry(n, r)
    m = 1.5 * np.random.default_rng(3).standard_normal(23)
    va, vb = g.axes[0].v[0], g.axes[0].v[3]
    src = W.explicit_columns([[(va, 1.0), (vb, -1.0)]])
    rec = W.explicit_columns([[(x, 1.0)] for x in range(23)])
    st = R.forward(g, m, src, rec)
    fs = R.fine_forward(g, m, src, rec)
    np.testing.assert_allclose(st.u, fs.u, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,r", GRIDS)
def test_coarse_operator_structure(n, r):
    g = Geometry(n, r)
    inst = _instance(n, r)
    st = R.forward(g, inst.m, inst.sources, inst.receivers)
    K = st.K
    assert np.abs(K - K.T).max() < 1e-12 * np.abs(K).max()
    assert np.abs(K @ np.ones(g.ncoarse)).max() < 1e-12 * np.abs(K).max()
    vm = g.vertex_multis()
    for a in vm:
        for b in vm:
            far = max(abs(a[k] - b[k]) for k in range(g.d)) > 1
            if far:
                assert K[g.vertex_id(a), g.vertex_id(b)] == 0.0
    # SPD after fixing vertex 0
    assert np.linalg.eigvalsh(K[1:, 1:]).min() > 0


def test_one_dimensional_coarse_operator_is_series_resistance():
    n, r = (29,), (4,)
    g = Geometry(n, r)
    m = 1.5 * np.random.default_rng(9).standard_normal(29)
    s = np.exp(m)
    st = R.forward(g, m, W.explicit_columns([[(3, 1.0), (20, -1.0)]]),
                   W.explicit_columns([[(5, 1.0)]]))
    v = g.axes[0].v
    T = 2 * s[:-1] * s[1:] / (s[:-1] + s[1:])
    Kc = np.zeros((g.ncoarse, g.ncoarse))
    for I in range(g.ncoarse - 1):
        Tc = 1.0 / np.sum(1.0 / T[v[I]:v[I + 1]])
        Kc[I, I] += Tc
        Kc[I + 1, I + 1] += Tc
        Kc[I, I + 1] -= Tc
        Kc[I + 1, I] -= Tc
    np.testing.assert_allclose(st.K, Kc, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("n,r", GRIDS)
@pytest.mark.parametrize("mode", MODES)
def test_reciprocity_orthogonality_scale(n, r, mode):
    g = Geometry(n, r)
    inst = _instance(n, r)
    rng = np.random.default_rng(4)
    a, b = rng.choice(g.ncell, 2, replace=False)
    pa = W.explicit_columns([[(int(a), 1.0)]])
    pb = W.explicit_columns([[(int(b), 1.0)]])
    dab = R.forward(g, inst.m, pa, pb, mode).D[0, 0]
    dba = R.forward(g, inst.m, pb, pa, mode).D[0, 0]
    assert abs(dab - dba) <= 1e-12 * max(1.0, abs(dab))
    st = R.forward(g, inst.m, inst.sources, inst.receivers, mode)
    res = np.asarray(st.Q.todense()) - st.A @ st.u
    orth = np.asarray(st.P.T @ res)[1:]
    assert np.abs(orth).max() < 1e-12 * max(1.0, np.abs(np.asarray(st.Q.todense())).max())
    st2 = R.forward(g, inst.m + 0.8, inst.sources, inst.receivers, mode)
    np.testing.assert_allclose(st2.u, math.exp(-0.8) * st.u, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("n,r", GRIDS)
@pytest.mark.parametrize("mode", MODES)
def test_sensitivity_fd_dot_and_scale(n, r, mode):
    g = Geometry(n, r)
    inst = _instance(n, r)
    rng = np.random.default_rng(6)
    st = R.forward(g, inst.m, inst.sources, inst.receivers, mode)
    V = rng.standard_normal(st.D.shape)
    dm = rng.standard_normal(g.ncell)
    gt = R.jtv(st, V)
    jv = R.jvp(st, dm)
    # forward mode against central differences of the forward map
    eps = 1e-5
    Dp = R.forward(g, inst.m + eps * dm, inst.sources, inst.receivers, mode).D
    Dm = R.forward(g, inst.m - eps * dm, inst.sources, inst.receivers, mode).D
    fd = (Dp - Dm) / (2 * eps)
    assert np.linalg.norm(jv - fd) <= 1e-5 * np.linalg.norm(fd)
    # transposed form against forward mode
    assert abs(np.sum(jv * V) - gt @ dm) <= 1e-12 * max(np.linalg.norm(gt) * np.linalg.norm(dm), 1e-30)
    # scale: S_k is invariant and A, A_k are homogeneous of degree one in e^m
    assert abs(gt.sum() + np.sum(st.D * V)) <= 1e-11 * max(1.0, np.abs(st.D * V).sum())
    # misfit gradient against central differences of the misfit
    Dobs = R.forward(g, inst.m_obs, inst.sources, inst.receivers, mode).D
    phi, grad, _ = R.misfit_grad(g, inst.m, inst.sources, inst.receivers, Dobs, mode)
    e = rng.standard_normal(g.ncell)
    h = 1e-5
    fp = R.misfit(R.forward(g, inst.m + h * e, inst.sources, inst.receivers, mode).D, Dobs)
    fm = R.misfit(R.forward(g, inst.m - h * e, inst.sources, inst.receivers, mode).D, Dobs)
    assert abs((fp - fm) / (2 * h) - grad @ e) <= 1e-5 * abs((fp - fm) / (2 * h))


@pytest.mark.parametrize("n,r", GRIDS)
def test_fixed_basis_and_fine_dot(n, r):
    g = Geometry(n, r)
    inst = _instance(n, r)
    rng = np.random.default_rng(8)
    st = R.forward(g, inst.m, inst.sources, inst.receivers)
    V = rng.standard_normal(st.D.shape)
    dm = rng.standard_normal(g.ncell)
    lhs = np.sum(R.jvp_fixed(st, dm) * V)
    rhs = R.jtv_fixed(st, V) @ dm
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))
    fs = R.fine_forward(g, inst.m, inst.sources, inst.receivers)
    jv = R.fine_jvp(fs, dm)
    eps = 1e-5
    fd = (R.fine_forward(g, inst.m + eps * dm, inst.sources, inst.receivers).D
          - R.fine_forward(g, inst.m - eps * dm, inst.sources, inst.receivers).D) / (2 * eps)
    assert np.linalg.norm(jv - fd) <= 1e-5 * np.linalg.norm(fd)
    assert abs(np.sum(jv * V) - R.fine_jtv(fs, V) @ dm) <= 1e-12 * max(1.0, abs(np.sum(jv * V)))


@pytest.mark.parametrize("n,r", [((13, 10), (4, 3)), ((10, 9, 8), (3, 3, 3))])
def test_lagrange_skeleton_electrodes_adaptive_equals_fixed(n, r):
    g = Geometry(n, r)
    rng = np.random.default_rng(12)
    m = 1.2 * rng.standard_normal(g.ncell)
    skel = [i for i in range(g.ncell)
            if any(g.cell_multi(i)[k] in g.axes[k].v for k in range(g.d))]
    pick = rng.choice(skel, 6, replace=False)
    src = W.explicit_columns([[(int(pick[0]), 1.0), (int(pick[1]), -1.0)],
                              [(int(pick[2]), 1.0), (int(pick[3]), -1.0)]])
    rec = W.explicit_columns([[(int(pick[4]), 1.0)], [(int(pick[5]), 1.0)]])
    st = R.forward(g, m, src, rec, "lagrange")
    V = rng.standard_normal(st.D.shape)
    ga = R.jtv(st, V)
    gf = R.jtv_fixed(st, V)
    np.testing.assert_allclose(ga, gf, rtol=1e-10, atol=1e-12 * np.abs(gf).max())
    # with reduced boundaries the skeleton moves with m and the two differ
    st_r = R.forward(g, m, src, rec, "reduced")
    assert np.abs(R.jtv(st_r, V) - R.jtv_fixed(st_r, V)).max() > 1e-6 * np.abs(gf).max()


@pytest.mark.parametrize("n,r", [((13, 11, 9), (4, 4, 4)), ((20, 14), (5, 4))])
def test_uniform_perturbation_adaptive_equals_fixed(n, r):
    """S_k(m + c 1) = S_k(m), so along dm = c 1 the basis tangent vanishes and
    the adaptive J dm equals the fixed-basis one; both equal -c D (A scales by
    e^c, u by e^-c)."""
    from oracle import Geometry
    from oracle import reduced as R
    import workloads as W
    inst = W.small_instance(n, r, seed=36, ns=2, nr=4)
    g = Geometry(n, r)
    st = R.forward(g, inst.m, inst.sources, inst.receivers)
    dm = -0.001 * np.ones(g.ncell)
    ja, jx = R.jvp(st, dm), R.jvp_fixed(st, dm)
    assert np.allclose(ja, jx, rtol=1e-10, atol=1e-14 * np.abs(ja).max())
    assert np.allclose(ja, 0.001 * st.D, rtol=1e-8, atol=1e-12 * np.abs(st.D).max())


@pytest.mark.parametrize("n,r", GRIDS)
@pytest.mark.parametrize("mode", MODES)
def test_frozen_basis_surrogate(n, r, mode):
    """The fixed-basis surrogate of eq. optredfixed (S_k(m0) held, A_k(m)
    rebuilt): at m = m0 it is the adaptive forward; its exact derivative is
    eq. senssimple with the frozen basis (jvp_fixed against central
    differences of the frozen forward, jtv_fixed by the dot test); and the
    frozen A_k is homogeneous of degree one in e^m."""
    g = Geometry(n, r)
    inst = _instance(n, r)
    rng = np.random.default_rng(14)
    st0 = R.forward(g, inst.m, inst.sources, inst.receivers, mode)
    m1 = inst.m + 0.3 * rng.standard_normal(g.ncell)
    fr = R.forward(g, m1, inst.sources, inst.receivers, mode, basis=st0.basis)
    same = R.forward(g, inst.m, inst.sources, inst.receivers, mode, basis=st0.basis)
    np.testing.assert_array_equal(same.D, st0.D)
    np.testing.assert_array_equal(fr.P.toarray(), st0.P.toarray())
    # an adaptive forward at m1 moves the basis (reduced boundaries or not,
    # the block interiors depend on m), so the two models differ there
    ad = R.forward(g, m1, inst.sources, inst.receivers, mode)
    assert np.abs(ad.D - fr.D).max() > 1e-8 * np.abs(ad.D).max()
    dm = rng.standard_normal(g.ncell)
    eps = 1e-5
    fd = (R.forward(g, m1 + eps * dm, inst.sources, inst.receivers, mode, basis=st0.basis).D
          - R.forward(g, m1 - eps * dm, inst.sources, inst.receivers, mode, basis=st0.basis).D) / (2 * eps)
    jv = R.jvp_fixed(fr, dm)
    assert np.linalg.norm(jv - fd) <= 1e-5 * np.linalg.norm(fd)
    V = rng.standard_normal(fr.D.shape)
    assert abs(np.sum(jv * V) - R.jtv_fixed(fr, V) @ dm) <= 1e-12 * max(1.0, abs(np.sum(jv * V)))
    sc = R.forward(g, m1 + 0.7, inst.sources, inst.receivers, mode, basis=st0.basis)
    np.testing.assert_allclose(sc.K, math.exp(0.7) * fr.K, rtol=1e-12, atol=1e-14 * np.abs(fr.K).max())
