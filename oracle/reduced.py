"""Reduced forward problem, sensitivities and the fine-mesh reference
(oracle; test infrastructure only).

Reduced forward (eq. fwdProbRed, eq. reducedPDE): with the Galerkin choice
R = S_k^T,

    A_k(m) = S_k(m)^T A(m) S_k(m),   t_j = A_k^{-1} S_k^T q_j,
    u_j = S_k t_j,                   D = Rx^T U.

The potential is fixed at one grid point (Sec. 2.2); on the coarse level
this is coarse vertex 0 (t_0 = 0, the basis without its first column), and
the fine reference fixes the cell of that vertex.

Adaptive sensitivities (Sec. 4.3).  Differentiating eq. redField gives
dt/dm = A_k^{-1} ( X_k(q - A S t) - S^T (G + A Y_k(t)) ) and eq. sensred
J_k = Rx^T ( Y_k(t) + S dt/dm ), with G = grad_m(A(m) S u) (eq. G).
``jvp`` evaluates J_k dm in exactly that form (forward mode, using the
basis tangent dS so that Y_k(v) dm = dS v and X_k(w) dm = dS^T w).
``jtv`` evaluates J_k^T v for every source by transposing the same
expression term by term, with lambda_j = A_k^{-1} S^T Rx v_j:

    J_k^T v = sum_j [ Y_k(t_j)^T (Rx v_j - A S lambda_j)
                      + Y_k(lambda_j)^T (q_j - A S t_j)
                      - G_j^T S lambda_j ],

using X_k(w)^T y = Y_k(y)^T w (both are grad_m of w^T S(m) y).  The
misfit gradient of Sec. 4.1 is J_k^T (D - D_obs).

Fixed basis (eq. senssimple): J_k = -Rx^T S A_k^{-1} S^T G.

Fine reference (eq. forwardProbFine, eq. sens): u = A^{-1} q with the
potential fixed at one cell, J = -Rx^T A^{-1} G.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .basis import Basis, basis_tangent, basis_vjp, build_basis, tangent_csr
from .geometry import Geometry
from .operator import fine_operator, operator_derivative_jvp, operator_derivative_vjp


def columns_matrix(ncell: int, cols) -> sp.csc_matrix:
    """Sparse N x count matrix from CSR-over-columns arrays (ptr, cell, val)
    or any object with those attributes."""
    ptr = np.asarray(cols.ptr, dtype=np.int64)
    cell = np.asarray(cols.cell, dtype=np.int64)
    val = np.asarray(cols.val, dtype=np.float64)
    return sp.csc_matrix((val, cell, ptr), shape=(ncell, ptr.size - 1))


def coarse_operator(P: sp.csr_matrix, A: sp.csr_matrix) -> np.ndarray:
    """A_k = S_k^T A S_k (eq. reducedPDE), dense."""
    return np.asarray((P.T @ (A @ P)).todense())


class PinnedCoarse:
    """A_k with vertex 0 removed (t_0 = 0), factorised by dense Cholesky."""

    def __init__(self, K: np.ndarray):
        self.K = K
        self.n = K.shape[0]
        self.chol = sla.cho_factor(K[1:, 1:], lower=True) if self.n > 1 else None

    def solve(self, B: np.ndarray) -> np.ndarray:
        B = np.asarray(B, dtype=np.float64)
        out = np.zeros_like(B)
        if self.n > 1:
            out[1:] = sla.cho_solve(self.chol, B[1:])
        return out


@dataclasses.dataclass
class ReducedState:
    geom: Geometry
    m: np.ndarray
    basis: Basis
    A: sp.csr_matrix
    P: sp.csr_matrix
    K: np.ndarray
    coarse: PinnedCoarse
    Q: sp.csc_matrix
    Rx: sp.csc_matrix
    t: np.ndarray   # Nc x Ns
    u: np.ndarray   # N x Ns
    D: np.ndarray   # Nr x Ns


def forward(geom: Geometry, m: np.ndarray, sources, receivers, mode: str = "reduced",
            basis: Optional[Basis] = None) -> ReducedState:
    """F_k(m) = Rx^T S_k A_k^{-1} S_k^T Q (eq. fwdProbRed).

    With ``basis`` given (a basis built at another model m0), the basis is
    held fixed and only A_k(m) = S_k(m0)^T A(m) S_k(m0) is rebuilt: the
    fixed-basis surrogate of eq. optredfixed, whose exact sensitivities are
    those of eq. senssimple (``jvp_fixed``, ``jtv_fixed``)."""
    m = np.asarray(m, dtype=np.float64)
    bas = build_basis(geom, m, mode) if basis is None else basis
    A = fine_operator(geom, m)
    P = bas.csr()
    K = coarse_operator(P, A)
    coarse = PinnedCoarse(K)
    Q = sources if sp.issparse(sources) else columns_matrix(geom.ncell, sources)
    Rx = receivers if sp.issparse(receivers) else columns_matrix(geom.ncell, receivers)
    b = np.asarray((P.T @ Q).todense())
    t = coarse.solve(b)
    u = P @ t
    D = np.asarray(Rx.T @ u)
    return ReducedState(geom, m, bas, A, P, K, coarse, Q, Rx, t, u, D)


def jtv(st: ReducedState, V: np.ndarray) -> np.ndarray:
    """J_k(m)^T V for the adaptive basis (transpose of eq. sensred)."""
    V = np.asarray(V, dtype=np.float64).reshape(st.D.shape)
    W = np.asarray(st.Rx @ V)                        # Rx v_j
    lam = st.coarse.solve(np.asarray(st.P.T @ W))    # A_k^{-1} S^T Rx v_j
    Plam = st.P @ lam
    a = W - st.A @ Plam                              # Rx v_j - A S lambda_j
    b = np.asarray(st.Q.todense()) - st.A @ st.u     # q_j - A S t_j
    g = basis_vjp(st.basis, np.hstack([st.t, lam]), np.hstack([a, b]))
    g -= operator_derivative_vjp(st.geom, st.m, st.u, Plam)
    return g


def jvp(st: ReducedState, dm: np.ndarray) -> np.ndarray:
    """J_k(m) dm for the adaptive basis, eq. sensred in forward mode."""
    dm = np.asarray(dm, dtype=np.float64)
    dS = tangent_csr(st.basis, basis_tangent(st.basis, dm))
    Yt = dS @ st.t                                     # Y_k(t) dm
    Gdm = operator_derivative_jvp(st.geom, st.m, st.u, dm)   # G dm
    resid = np.asarray(st.Q.todense()) - st.A @ st.u   # q - A S t
    Xr = np.asarray(dS.T @ resid)                      # X_k(q - A S t) dm
    dt = st.coarse.solve(Xr - np.asarray(st.P.T @ (Gdm + st.A @ Yt)))
    return np.asarray(st.Rx.T @ (Yt + st.P @ dt))


def jtv_fixed(st: ReducedState, V: np.ndarray) -> np.ndarray:
    """J_k^T V with the basis held fixed (transpose of eq. senssimple)."""
    V = np.asarray(V, dtype=np.float64).reshape(st.D.shape)
    lam = st.coarse.solve(np.asarray(st.P.T @ (st.Rx @ V)))
    return -operator_derivative_vjp(st.geom, st.m, st.u, st.P @ lam)


def jvp_fixed(st: ReducedState, dm: np.ndarray) -> np.ndarray:
    """J_k dm with the basis held fixed (eq. senssimple)."""
    Gdm = operator_derivative_jvp(st.geom, st.m, st.u, np.asarray(dm, dtype=np.float64))
    dt = st.coarse.solve(np.asarray(st.P.T @ Gdm))
    return -np.asarray(st.Rx.T @ (st.P @ dt))


def misfit(D: np.ndarray, D_obs: np.ndarray) -> float:
    """SSD misfit 1/2 ||D_pred - D_obs||_F^2 (Sec. 2.2)."""
    r = np.asarray(D) - np.asarray(D_obs)
    return 0.5 * float(np.sum(r * r))


def misfit_grad(geom: Geometry, m: np.ndarray, sources, receivers, D_obs: np.ndarray,
                mode: str = "reduced"):
    """(phi, grad phi) with grad phi = J_k^T (D - D_obs) (Sec. 4.1)."""
    st = forward(geom, m, sources, receivers, mode)
    return misfit(st.D, D_obs), jtv(st, st.D - D_obs), st


# ---------------------------------------------------------------------------
# fine-mesh reference
# ---------------------------------------------------------------------------

def pin_cell(geom: Geometry) -> int:
    """The cell of coarse vertex 0; both levels fix the potential there."""
    return geom.vertex_cell((0,) * geom.d)


@dataclasses.dataclass
class FineState:
    geom: Geometry
    m: np.ndarray
    A: sp.csr_matrix
    keep: np.ndarray
    lu: object
    Q: sp.csc_matrix
    Rx: sp.csc_matrix
    u: np.ndarray
    D: np.ndarray

    def solve(self, B: np.ndarray) -> np.ndarray:
        out = np.zeros((self.geom.ncell, B.shape[1]))
        out[self.keep] = self.lu.solve(np.ascontiguousarray(B[self.keep]))
        return out


def fine_forward(geom: Geometry, m: np.ndarray, sources, receivers,
                 pin: Optional[int] = None) -> FineState:
    """F(m) = Rx^T A(m)^{-1} Q with u fixed to 0 at one cell
    (eq. forwardProbFine and Sec. 2.2)."""
    m = np.asarray(m, dtype=np.float64)
    A = fine_operator(geom, m)
    pin = pin_cell(geom) if pin is None else pin
    keep = np.ones(geom.ncell, dtype=bool)
    keep[pin] = False
    lu = spla.splu(A[keep][:, keep].tocsc())
    Q = sources if sp.issparse(sources) else columns_matrix(geom.ncell, sources)
    Rx = receivers if sp.issparse(receivers) else columns_matrix(geom.ncell, receivers)
    st = FineState(geom, m, A, keep, lu, Q, Rx, None, None)
    st.u = st.solve(np.asarray(Q.todense()))
    st.D = np.asarray(Rx.T @ st.u)
    return st


def fine_jtv(st: FineState, V: np.ndarray) -> np.ndarray:
    """J^T V with J = -Rx^T A^{-1} grad_m(A(m) u) (eq. sens)."""
    lam = st.solve(np.asarray(st.Rx @ np.asarray(V).reshape(st.D.shape)))
    return -operator_derivative_vjp(st.geom, st.m, st.u, lam)


def fine_jvp(st: FineState, dm: np.ndarray) -> np.ndarray:
    """J dm for the fine mesh (eq. sens)."""
    Gdm = operator_derivative_jvp(st.geom, st.m, st.u, np.asarray(dm, dtype=np.float64))
    return -np.asarray(st.Rx.T @ st.solve(Gdm))
