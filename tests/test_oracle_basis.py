"""Pins for the oracle's multiscale basis S_k(m) (Sec. 3.2) and its
derivatives (Sec. 4.5).

* Partition of unity S_k 1 = 1 and reproduction of constants (the local
  operators annihilate constants and the vertex data sum to one).
* s_c(vertex c') = delta_cc'; 0 <= s <= 1 (the local matrices are M-matrices,
  so the discrete maximum principle holds); support inside the closed dual
  blocks around c.
* Constant conductivity: the basis is the multilinear interpolant in index
  coordinates, built here from the vertex positions alone.
* 1-D: the closed form s_lo(i) = R(i -> hi) / R(lo -> hi) with R the sum of
  face resistances 1/T.
* Reduced boundaries with layered sigma(x): s = psi(x) * (multilinear in the
  other axes) with psi the 1-D closed form; Lagrange boundaries do not have
  this product form, which tells the two modes apart.
* S_k(m + c 1) = S_k(m); Lagrange skeleton values do not depend on m.
* Tangent against central finite differences; reverse sweep against the
  tangent (dot test).
* A build restricted to a few entities reproduces the full build's rows of
  those entities (it is what checks single entities of large grids).
"""
import numpy as np
import pytest

from oracle import Geometry
from oracle.basis import basis_tangent, basis_vjp, build_basis, tangent_csr

GRIDS = [((9,), (3,)), ((11,), (4,)), ((8, 8), (3, 3)), ((10, 7), (4, 3)),
         ((7, 5, 6), (3, 2, 3)), ((13, 11, 9), (4, 4, 4)), ((6, 6, 6), (2, 3, 2))]
MODES = ["reduced", "lagrange"]


def _model(g, seed, kind="random"):
    rng = np.random.default_rng(seed)
    if kind == "random":
        return 1.5 * rng.standard_normal(g.ncell)
    if kind == "const":
        return np.full(g.ncell, 0.7)
    raise ValueError(kind)


@pytest.mark.parametrize("n,r", GRIDS)
@pytest.mark.parametrize("mode", MODES)
def test_partition_of_unity_and_bounds(n, r, mode):
    g = Geometry(n, r)
    b = build_basis(g, _model(g, 3), mode)
    P = b.csr()
    np.testing.assert_allclose(P @ np.ones(g.ncoarse), 1.0, atol=1e-13)
    assert P.data.min() >= -1e-14 and P.data.max() <= 1 + 1e-14
    # reproduction of constants: u = S 1*c is constant c
    np.testing.assert_allclose(P @ np.full(g.ncoarse, 2.5), 2.5, atol=1e-12)


@pytest.mark.parametrize("n,r", GRIDS)
def test_vertex_delta_and_support(n, r):
    g = Geometry(n, r)
    b = build_basis(g, _model(g, 4), "reduced")
    P = b.csr().toarray()
    for multi in g.vertex_multis():
        cell = g.vertex_cell(multi)
        row = np.zeros(g.ncoarse)
        row[g.vertex_id(multi)] = 1.0
        np.testing.assert_array_equal(P[cell], row)
    # support of s_c: cells whose coordinates lie within the closed segments
    # adjacent to c's planes on every axis
    coords = np.array([g.cell_multi(i) for i in range(g.ncell)])
    for multi in g.vertex_multis():
        c = g.vertex_id(multi)
        inside = np.ones(g.ncell, dtype=bool)
        for k in range(g.d):
            ax = g.axes[k]
            I = multi[k]
            lo = ax.v[I - 1] if I > 0 else 0
            hi = ax.v[I + 1] if I + 1 < ax.nc else ax.n - 1
            inside &= (coords[:, k] >= lo) & (coords[:, k] <= hi)
        assert np.all(P[~inside, c] == 0.0)


def _hat(g, multi, coords):
    """Multilinear hat of vertex ``multi`` in index coordinates: linear
    between neighbouring vertex planes, flat out to the domain boundary."""
    val = np.ones(coords.shape[0])
    for k in range(g.d):
        ax = g.axes[k]
        I = multi[k]
        x = coords[:, k].astype(float)
        vI = ax.v[I]
        f = np.zeros_like(x)
        f[x == vI] = 1.0
        if I > 0:
            lo = ax.v[I - 1]
            sel = (x > lo) & (x < vI)
            f[sel] = (x[sel] - lo) / (vI - lo)
        else:
            f[x < vI] = 1.0
        if I + 1 < ax.nc:
            hi = ax.v[I + 1]
            sel = (x > vI) & (x < hi)
            f[sel] = (hi - x[sel]) / (hi - vI)
        else:
            f[x > vI] = 1.0
        val *= f
    return val


@pytest.mark.parametrize("n,r", GRIDS)
@pytest.mark.parametrize("mode", MODES)
def test_constant_conductivity_is_multilinear(n, r, mode):
    g = Geometry(n, r)
    b = build_basis(g, _model(g, 0, "const"), mode)
    P = b.csr().toarray()
    coords = np.array([g.cell_multi(i) for i in range(g.ncell)])
    for multi in g.vertex_multis():
        np.testing.assert_allclose(P[:, g.vertex_id(multi)], _hat(g, multi, coords), atol=1e-13)


def _resistance_profile(sigma_line):
    T = 2 * sigma_line[:-1] * sigma_line[1:] / (sigma_line[:-1] + sigma_line[1:])
    return np.concatenate([[0.0], np.cumsum(1.0 / T)])


def _psi(ax, sigma_x, I):
    """1-D reduced basis of vertex I along one axis (closed form)."""
    n = ax.n
    out = np.zeros(n)
    vI = ax.v[I]
    Rcum = _resistance_profile(sigma_x)
    out[vI] = 1.0
    if I > 0:
        lo = ax.v[I - 1]
        for x in range(lo + 1, vI):
            out[x] = (Rcum[x] - Rcum[lo]) / (Rcum[vI] - Rcum[lo])
    else:
        out[:vI] = 1.0
    if I + 1 < ax.nc:
        hi = ax.v[I + 1]
        for x in range(vI + 1, hi):
            out[x] = (Rcum[hi] - Rcum[x]) / (Rcum[hi] - Rcum[vI])
    else:
        out[vI + 1:] = 1.0
    return out


@pytest.mark.parametrize("n,r", [((23,), (5,)), ((12,), (4,)), ((9,), (2,))])
def test_one_dimensional_closed_form(n, r):
    g = Geometry(n, r)
    m = _model(g, 5)
    P = build_basis(g, m, "reduced").csr().toarray()
    for I in range(g.nc[0]):
        np.testing.assert_allclose(P[:, I], _psi(g.axes[0], np.exp(m), I), atol=1e-14)


@pytest.mark.parametrize("n,r", [((13, 9), (4, 3)), ((11, 7, 9), (4, 3, 4))])
def test_layered_reduced_is_tensor_product(n, r):
    g = Geometry(n, r)
    rng = np.random.default_rng(11)
    sig_x = np.exp(1.5 * rng.standard_normal(n[0]))
    coords = np.array([g.cell_multi(i) for i in range(g.ncell)])
    m = np.log(sig_x[coords[:, 0]])
    P = build_basis(g, m, "reduced").csr().toarray()
    for multi in g.vertex_multis():
        psi = _psi(g.axes[0], sig_x, multi[0])[coords[:, 0]]
        rest = np.ones(g.ncell)
        if g.d > 1:
            # multilinear in the remaining axes: hat with axis 0 frozen at 1
            sub = coords.copy()
            sub[:, 0] = g.axes[0].v[multi[0]]
            rest = _hat(g, multi, sub)
        np.testing.assert_allclose(P[:, g.vertex_id(multi)], psi * rest, atol=1e-13)
    # the Lagrange boundary data are linear along x, so the product form fails
    PL = build_basis(g, m, "lagrange").csr().toarray()
    assert np.abs(PL - P).max() > 1e-3


@pytest.mark.parametrize("n,r", GRIDS)
@pytest.mark.parametrize("mode", MODES)
def test_scale_invariance(n, r, mode):
    g = Geometry(n, r)
    m = _model(g, 6)
    P0 = build_basis(g, m, mode).csr().toarray()
    P1 = build_basis(g, m + 2.3, mode).csr().toarray()
    np.testing.assert_allclose(P1, P0, atol=1e-13)


@pytest.mark.parametrize("n,r", [((10, 7), (4, 3)), ((7, 5, 6), (3, 2, 3))])
def test_lagrange_skeleton_independent_of_m(n, r):
    g = Geometry(n, r)
    b1 = build_basis(g, _model(g, 1), "lagrange")
    b2 = build_basis(g, _model(g, 2), "lagrange")
    for e in g.entities:
        if e.dim < g.d:
            ids = g.cell_ids(e.cell_ranges)
            np.testing.assert_array_equal(b1.vals[ids], b2.vals[ids])


@pytest.mark.parametrize("n,r", GRIDS)
@pytest.mark.parametrize("mode", MODES)
def test_tangent_fd_and_reverse_dot(n, r, mode):
    g = Geometry(n, r)
    rng = np.random.default_rng(7)
    m = _model(g, 8)
    dm = rng.standard_normal(g.ncell)
    b = build_basis(g, m, mode)
    dP = tangent_csr(b, basis_tangent(b, dm)).toarray()
    eps = 1e-6
    Pp = build_basis(g, m + eps * dm, mode).csr().toarray()
    Pm = build_basis(g, m - eps * dm, mode).csr().toarray()
    fd = (Pp - Pm) / (2 * eps)
    scale = max(1.0, np.abs(fd).max())
    assert np.abs(dP - fd).max() <= 1e-7 * scale
    V = rng.standard_normal((g.ncoarse, 3))
    Z = rng.standard_normal((g.ncell, 3))
    lhs = basis_vjp(b, V, Z) @ dm
    rhs = np.sum(Z * (dP @ V))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs))


@pytest.mark.parametrize("mode", MODES)
def test_restricted_build_matches_full(mode):
    n, r = (17, 13, 11), (4, 4, 3)
    g = Geometry(n, r)
    m = np.random.default_rng(8).standard_normal(g.ncell)
    full = build_basis(g, m, mode)
    rng = np.random.default_rng(9)
    picks = []
    for d in (1, 2, 3):
        cand = [i for i, e in enumerate(g.entities) if e.dim == d]
        picks += [cand[0], cand[-1]] + list(rng.choice(cand, 2, replace=False))
    part = build_basis(g, m, mode, only=picks)
    for i in picks:
        cells = g.cell_ids(g.entities[i].cell_ranges)
        assert np.array_equal(part.cols[cells], full.cols[cells])
        assert np.array_equal(part.vals[cells], full.vals[cells])
    # rows outside every picked closure stay empty, vertex rows aside
    covered = np.zeros(g.ncell, dtype=bool)
    for i in picks:
        covered[g.cell_ids(g.entities[i].closure_ranges)] = True
    for multi in g.vertex_multis():
        covered[g.vertex_cell(multi)] = True
    assert (part.cols[~covered] < 0).all()
    assert (~covered).sum() > g.ncell // 2
