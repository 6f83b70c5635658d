"""Pins for the oracle's geometry and fine operator.

* Vertex placement and the coarse sizes the workloads name (8x8 at 32^2/r=4,
  8^3 at 64^3/r=8, 16^3 at 128^3/r=8).
* Every cell belongs to exactly one entity; entity counts and the sparsity of
  the basis against per-axis closed forms (nnz(S_k) = prod_k (Nc_k + w_k),
  blocks = prod_k (#segments)).
* A(m): symmetric, A 1 = 0, equal to the textbook graph Laplacian for
  sigma = 1 (built here as a Kronecker sum of path Laplacians), 1-D solve
  equal to the closed form of cumulative flux times resistance.
* The flux derivatives against central finite differences.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import Geometry
from oracle.operator import (fine_operator, harmonic_T, harmonic_dT,
                             operator_derivative_jvp, operator_derivative_vjp)


def _w_open(n, r):
    nc = -(-n // r)
    v = [I * r + min(r, n - I * r) // 2 for I in range(nc)]
    w = v[0]                       # lower strip cells count once
    w += (n - 1 - v[-1])           # upper strip
    for s in range(1, nc):
        w += 2 * (v[s] - v[s - 1] - 1)
    return nc, v, w


@pytest.mark.parametrize("n,r,expect", [(32, 4, [2, 6, 10, 14, 18, 22, 26, 30]),
                                        (128, 8, list(range(4, 128, 8))),
                                        (13, 4, [2, 6, 10, 12]),
                                        (9, 1, list(range(9)))])
def test_vertex_positions(n, r, expect):
    g = Geometry((n,), (r,))
    assert g.axes[0].v == expect


@pytest.mark.parametrize("n,r,nc", [((32, 32), (4, 4), 64), ((64,) * 3, (8,) * 3, 512),
                                    ((128,) * 3, (8,) * 3, 4096)])
def test_coarse_sizes(n, r, nc):
    assert Geometry(n, r).ncoarse == nc


@pytest.mark.parametrize("n,r", [((9,), (3,)), ((8, 8), (3, 3)), ((10, 7), (4, 3)),
                                 ((7, 5, 6), (3, 2, 3)), ((13, 11, 9), (4, 4, 4)),
                                 ((64,) * 3, (8,) * 3), ((49, 50, 51), (8, 8, 8))])
def test_entity_partition_and_counts(n, r):
    g = Geometry(n, r)
    owner = np.zeros(g.ncell, dtype=np.int64)
    nnz = 0
    for e in g.entities:
        ids = g.cell_ids(e.cell_ranges)
        np.add.at(owner, ids, 1)
        nnz += ids.size * len(e.corners)
        assert len(e.corners) == 2 ** sum(
            1 for k in e.open_axes if g.axes[k].segments[e.key[k][1]].kind == "bounded")
    assert np.all(owner == 1)
    expect_nnz, expect_blocks = 1, 1
    for k in range(g.d):
        nc, v, w = _w_open(n[k], r[k])
        expect_nnz *= nc + w
        expect_blocks *= nc + 1
    assert nnz == expect_nnz
    nonempty_blocks = sum(1 for e in g.entities if e.dim == g.d)
    assert nonempty_blocks <= expect_blocks


def test_appendix_counts_128():
    """nnz of the basis at 128^3 / r = 8 from the per-axis closed form."""
    nc, v, w = _w_open(128, 8)
    assert (nc, w) == (16, 217)
    assert (nc + w) ** 3 == 12_649_337
    g = Geometry((128,) * 3, (8,) * 3)
    assert sum(1 for e in g.entities if e.dim == 3) == 17 ** 3


def _path_laplacian(n):
    if n == 1:
        return sp.csr_matrix((1, 1))
    main = np.full(n, 2.0)
    main[0] = main[-1] = 1.0
    return sp.diags([main, -np.ones(n - 1), -np.ones(n - 1)], [0, -1, 1]).tocsr()


@pytest.mark.parametrize("n", [(7,), (5, 4), (4, 3, 5)])
def test_unit_conductivity_is_graph_laplacian(n):
    g = Geometry(n, (1,) * len(n))
    A = fine_operator(g, np.zeros(g.ncell)).toarray()
    L = None
    for k in range(len(n)):
        term = _path_laplacian(n[k])
        for j in range(len(n)):
            if j == k:
                continue
            eye = sp.identity(n[j])
            term = sp.kron(eye, term) if j > k else sp.kron(term, eye)
        L = term if L is None else L + term
    np.testing.assert_allclose(A, L.toarray(), atol=1e-14)


@pytest.mark.parametrize("n", [(9,), (6, 5), (4, 5, 3)])
def test_operator_symmetric_and_annihilates_constants(n, rng):
    g = Geometry(n, (1,) * len(n))
    m = rng.standard_normal(g.ncell) * 2
    A = fine_operator(g, m)
    assert abs(A - A.T).max() < 1e-13
    assert np.abs(A @ np.ones(g.ncell)).max() < 1e-12
    # constant conductivity scales the Laplacian
    A0 = fine_operator(g, np.zeros(g.ncell))
    A3 = fine_operator(g, np.full(g.ncell, np.log(3.0)))
    np.testing.assert_allclose(A3.toarray(), 3.0 * A0.toarray(), rtol=1e-14, atol=1e-14)


def test_one_dimensional_solve_closed_form(rng):
    n = 17
    g = Geometry((n,), (1,))
    m = rng.standard_normal(n)
    sigma = np.exp(m)
    q = np.zeros(n)
    q[3], q[12] = 1.0, -1.0
    # flux across face i+1/2 is the cumulative source; the potential drops by
    # flux times resistance 1/T; fix u at cell 0
    T = 2 * sigma[:-1] * sigma[1:] / (sigma[:-1] + sigma[1:])
    flux = np.cumsum(q)[:-1]
    u = np.concatenate([[0.0], -np.cumsum(flux / T)])
    A = fine_operator(g, m).toarray()
    keep = np.arange(1, n)
    u_solve = np.zeros(n)
    u_solve[keep] = np.linalg.solve(A[np.ix_(keep, keep)], q[keep])
    np.testing.assert_allclose(u_solve, u, rtol=1e-12, atol=1e-12)


def test_transmissibility_derivative_fd(rng):
    sa, sb = np.exp(rng.standard_normal(5)), np.exp(rng.standard_normal(5))
    dTa, dTb = harmonic_dT(sa, sb)
    eps = 1e-6
    fa = (harmonic_T(sa * np.exp(eps), sb) - harmonic_T(sa * np.exp(-eps), sb)) / (2 * eps)
    fb = (harmonic_T(sa, sb * np.exp(eps)) - harmonic_T(sa, sb * np.exp(-eps))) / (2 * eps)
    np.testing.assert_allclose(dTa, fa, rtol=1e-8)
    np.testing.assert_allclose(dTb, fb, rtol=1e-8)


@pytest.mark.parametrize("n", [(8,), (5, 6), (3, 4, 5)])
def test_operator_derivative_fd_and_dot(n, rng):
    g = Geometry(n, (1,) * len(n))
    m = rng.standard_normal(g.ncell)
    u = rng.standard_normal((g.ncell, 2))
    z = rng.standard_normal((g.ncell, 2))
    dm = rng.standard_normal(g.ncell)
    eps = 1e-6
    fd = (fine_operator(g, m + eps * dm) @ u - fine_operator(g, m - eps * dm) @ u) / (2 * eps)
    jv = operator_derivative_jvp(g, m, u, dm)
    np.testing.assert_allclose(jv, fd, rtol=1e-7, atol=1e-8)
    vj = operator_derivative_vjp(g, m, u, z)
    assert abs(vj @ dm - np.sum(z * jv)) < 1e-12 * max(1.0, abs(vj @ dm))
