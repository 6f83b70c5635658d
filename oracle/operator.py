"""Conductivity, two-point fluxes and the fine operator A(m) (oracle; test
infrastructure only).

Sec. 2.1 models the field by the steady diffusion equation with conductivity
sigma(m), e.g. sigma = exp(m), no-flux boundaries, and the potential fixed at
one grid point (Sec. 2.2).  This oracle uses the SPD sign convention
-div(sigma grad u) = q and a cell-centred finite-volume discretisation on a
uniform grid with h = 1: every pair of face-adjacent cells (a, b) is joined
by the harmonic-mean transmissibility T_ab = 2 s_a s_b / (s_a + s_b), and

    A(m) = sum_f T_f (e_a - e_b)(e_a - e_b)^T,

which is symmetric positive semi-definite with A 1 = 0 (no-flux boundary).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np
import scipy.sparse as sp


def conductivity(m: np.ndarray) -> np.ndarray:
    """sigma(m) = exp(m) (Sec. 2.1)."""
    return np.exp(np.asarray(m, dtype=np.float64))


def harmonic_T(sa: np.ndarray, sb: np.ndarray) -> np.ndarray:
    """Two-point transmissibility of one face with unit spacing."""
    return 2.0 * sa * sb / (sa + sb)


def harmonic_dT(sa: np.ndarray, sb: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """(dT/dm_a, dT/dm_b) for sigma = exp(m):
    dT/dm_a = sigma_a * dT/dsigma_a = 2 s_a s_b^2 / (s_a + s_b)^2."""
    den = (sa + sb) ** 2
    return 2.0 * sa * sb * sb / den, 2.0 * sb * sa * sa / den


def fine_faces(geom, m: np.ndarray):
    """All face-adjacent cell pairs (a, b = a + e_k) of the fine grid with
    their transmissibilities and derivatives.  Returns (a, b, T, dTa, dTb)."""
    sigma = conductivity(m)
    aa, bb = [], []
    for k in range(geom.d):
        ranges = [np.arange(geom.n[j]) for j in range(geom.d)]
        ranges[k] = np.arange(geom.n[k] - 1)
        if geom.n[k] < 2:
            continue
        a = geom.cell_ids(ranges)
        aa.append(a)
        bb.append(a + geom.strides[k])
    if not aa:
        e = np.zeros(0, dtype=np.int64)
        z = np.zeros(0)
        return e, e, z, z, z
    a = np.concatenate(aa)
    b = np.concatenate(bb)
    T = harmonic_T(sigma[a], sigma[b])
    dTa, dTb = harmonic_dT(sigma[a], sigma[b])
    return a, b, T, dTa, dTb


def assemble(nrow: int, a: np.ndarray, b: np.ndarray, T: np.ndarray) -> sp.csr_matrix:
    """sum_f T_f (e_a - e_b)(e_a - e_b)^T as a sparse matrix."""
    rows = np.concatenate([a, b, a, b])
    cols = np.concatenate([a, b, b, a])
    data = np.concatenate([T, T, -T, -T])
    return sp.csr_matrix((data, (rows, cols)), shape=(nrow, nrow))


def fine_operator(geom, m: np.ndarray) -> sp.csr_matrix:
    """The fine operator A(m) of Sec. 2.2 (before fixing the potential)."""
    a, b, T, _, _ = fine_faces(geom, m)
    return assemble(geom.ncell, a, b, T)


def operator_derivative_vjp(geom, m: np.ndarray, U: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """grad_m sum_cols Z[:, j]^T A(m) U[:, j]
    = sum_f dT_f/dm (U_a - U_b)(Z_a - Z_b), the transpose of the matrix G of
    eq. G applied to Z (the product rule term d(A(m)u)/dm)."""
    a, b, _, dTa, dTb = fine_faces(geom, m)
    U = U.reshape(geom.ncell, -1)
    Z = Z.reshape(geom.ncell, -1)
    w = np.sum((U[a] - U[b]) * (Z[a] - Z[b]), axis=1)
    g = np.zeros(geom.ncell)
    np.add.at(g, a, dTa * w)
    np.add.at(g, b, dTb * w)
    return g


def operator_derivative_jvp(geom, m: np.ndarray, U: np.ndarray, dm: np.ndarray) -> np.ndarray:
    """(d/dm A(m) U) dm = G dm of eq. G for each column of U."""
    a, b, _, dTa, dTb = fine_faces(geom, m)
    U = U.reshape(geom.ncell, -1)
    dT = dTa * dm[a] + dTb * dm[b]
    flux = dT[:, None] * (U[a] - U[b])
    out = np.zeros_like(U)
    np.add.at(out, a, flux)
    np.add.at(out, b, -flux)
    return out
