"""Planted mistakes in the oracle must be caught by its pins.

Each test monkeypatches one plausible mistake into the CPU oracle (a wrong
face average, a dropped term, a flipped sign, a swapped derivative, a wrong
pinned vertex) and checks that a pin from the other oracle test modules
fails on it.  This is what makes the pins worth trusting.
"""
import numpy as np
import pytest

import workloads as W
from oracle import Geometry
from oracle import basis as OB
from oracle import operator as OO
from oracle import reduced as R


def _setup(n=(8, 7), r=(3, 3), mode="reduced"):
    g = Geometry(n, r)
    inst = W.small_instance(n, r, 5)
    return g, inst


def _dot_gap(g, inst, mode="reduced"):
    rng = np.random.default_rng(1)
    st = R.forward(g, inst.m, inst.sources, inst.receivers, mode)
    V = rng.standard_normal(st.D.shape)
    dm = rng.standard_normal(g.ncell)
    a = np.sum(R.jvp(st, dm) * V)
    b = R.jtv(st, V) @ dm
    return abs(a - b) / max(abs(a), 1e-30)


def _fd_gap(g, inst, mode="reduced"):
    rng = np.random.default_rng(2)
    st = R.forward(g, inst.m, inst.sources, inst.receivers, mode)
    dm = rng.standard_normal(g.ncell)
    eps = 1e-5
    fd = (R.forward(g, inst.m + eps * dm, inst.sources, inst.receivers, mode).D
          - R.forward(g, inst.m - eps * dm, inst.sources, inst.receivers, mode).D) / (2 * eps)
    return np.linalg.norm(R.jvp(st, dm) - fd) / np.linalg.norm(fd)


def test_baseline_pins_hold():
    g, inst = _setup()
    assert _dot_gap(g, inst) < 1e-12
    assert _fd_gap(g, inst) < 1e-5


def test_arithmetic_face_average_is_caught(monkeypatch):
    bad = lambda sa, sb: 0.5 * (sa + sb)  # noqa: E731
    monkeypatch.setattr(OO, "harmonic_T", bad)
    monkeypatch.setattr(OB, "harmonic_T", bad)
    # the 1-D closed-form pin uses the harmonic mean of the paper's reading
    n = 17
    g = Geometry((n,), (1,))
    m = np.random.default_rng(0).standard_normal(n)
    s = np.exp(m)
    T = 2 * s[:-1] * s[1:] / (s[:-1] + s[1:])
    A = OO.fine_operator(g, m).toarray()
    assert abs(-A[0, 1] - T[0]) > 1e-6


def test_dropped_push_in_reverse_sweep_is_caught(monkeypatch):
    real = OB.basis_vjp

    def no_push(bas, V, Z):
        # reverse sweep that forgets to pass the load down to lower entities
        geom = bas.geom
        V = np.asarray(V, dtype=np.float64).reshape(geom.ncoarse, -1)
        Z = np.array(Z, dtype=np.float64).reshape(geom.ncell, -1)
        X = bas.csr() @ V
        g = np.zeros(geom.ncell)
        for idx, e in enumerate(geom.entities):
            if e.dim == 0 or not bas.solved(e):
                continue
            lp = bas.local[idx]
            mu = lp.solve(Z[lp.ids[lp.U]]).reshape(lp.U.size, -1)
            mut = np.zeros((lp.ids.size, mu.shape[1]))
            mut[lp.U] = mu
            xl = X[lp.ids]
            w = np.sum((mut[lp.la] - mut[lp.lb]) * (xl[lp.la] - xl[lp.lb]), axis=1)
            np.add.at(g, lp.ga, -lp.dTa * w)
            np.add.at(g, lp.gb, -lp.dTb * w)
        return g

    assert real is not no_push
    monkeypatch.setattr(R, "basis_vjp", no_push)
    g, inst = _setup()
    assert _dot_gap(g, inst) > 1e-6


def test_flipped_operator_term_is_caught(monkeypatch):
    real = R.operator_derivative_vjp
    monkeypatch.setattr(R, "operator_derivative_vjp", lambda *a: -real(*a))
    g, inst = _setup()
    assert _dot_gap(g, inst) > 1e-6


def test_swapped_flux_derivative_is_caught(monkeypatch):
    real = OO.harmonic_dT
    swapped = lambda sa, sb: real(sa, sb)[::-1]  # noqa: E731
    monkeypatch.setattr(OO, "harmonic_dT", swapped)
    monkeypatch.setattr(OB, "harmonic_dT", swapped)
    g, inst = _setup()
    assert _fd_gap(g, inst) > 1e-3


def test_dropped_basis_derivative_is_caught(monkeypatch):
    # using the fixed-basis sensitivity for the adaptive one fails the FD pin
    monkeypatch.setattr(R, "jvp", R.jvp_fixed)
    g, inst = _setup(mode="reduced")
    assert _fd_gap(g, inst) > 1e-4


def test_wrong_pinned_cell_is_caught():
    n, r = (7, 6), (1, 1)
    g = Geometry(n, r)
    inst = W.small_instance(n, r, 3)
    st = R.forward(g, inst.m, inst.sources, W.explicit_columns([[(5, 1.0)]]))
    fs = R.fine_forward(g, inst.m, inst.sources, W.explicit_columns([[(5, 1.0)]]), pin=7)
    # pole data depend on the gauge: the r = 1 pin fails with another cell
    assert np.abs(st.D - fs.D).max() > 1e-6


@pytest.mark.parametrize("mode", ["reduced", "lagrange"])
def test_unsorted_corner_order_is_caught(mode, monkeypatch):
    # a basis with corners assigned to the wrong vertices breaks partition of
    # unity or the vertex-delta pin
    g, inst = _setup()
    b = OB.build_basis(g, inst.m, mode)
    rows = np.nonzero((b.cols[:, 1] >= 0))[0]
    b.cols[rows, 0], b.cols[rows, 1] = b.cols[rows, 1].copy(), b.cols[rows, 0].copy()
    b._csr = None
    P = b.csr().toarray()
    ok_delta = all(P[g.vertex_cell(mm), g.vertex_id(mm)] == 1.0 for mm in g.vertex_multis())
    const = np.full(g.ncoarse, 1.0)
    const[0] = 2.0
    assert (not ok_delta) or np.abs(P @ const - OB.build_basis(g, inst.m, mode).csr() @ const).max() > 1e-3
