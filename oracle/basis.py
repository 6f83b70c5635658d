"""The parameter-dependent multiscale basis S_k(m), its tangent and its
reverse-mode derivative (oracle; test infrastructure only).

Construction (Sec. 3.2, steps 1-3, eq. multiscaleBasis_step3).  Every basis
function belongs to one coarse vertex c and equals delta_{c c'} at the
vertex cells.  Entities are processed in increasing dimension; on each entity
E and for each corner c of E the values on E solve the local problem

    A^E_EE s_c|E = - A^E_{E,dE} s_c|dE       (q = 0, Dirichlet data s_bc),

where A^E keeps only the two-point fluxes along E's open axes between cells
of E's closure (the reduced, tangential operator of classic MSFV), and s_c|dE
are the already-computed values on the lower-dimensional entities bounding E.
For a dual block (dimension d) A^E is the full operator on the closed block,
which is exactly eq. multiscaleBasis_step3 with Dirichlet data on the block
boundary.  Strip ends have no cell beyond the domain, so they carry the
physical no-flux condition of Sec. 2.1.  s_c is zero on entities that do
not have c as a corner.

Two choices of boundary data are provided (Sec. 3.2 "Piecewise Lagrange
Polynomials" and the reduced-boundary localisation of classic MSFV):

* ``mode="lagrange"``: on entities of dimension < d the values are the
  products of 1-D linear Lagrange factors in index coordinates (1 along a
  strip); only dual blocks are solved.
* ``mode="reduced"``: edges, then faces, then blocks are all solved with
  their reduced operators, so the boundary data depend on m.

Derivatives (Sec. 4.5, eq. reducedDiscreteMSBasisPDE and the expression for
grad x following it): with x = S_k(m) v, differentiating the local problem of
every entity gives

    dx_E = -(A^E_EE)^{-1} [ (dA^E x)_E + A^E_{E,dE} dx_dE ],

swept in increasing dimension (``basis_tangent``), and its transpose swept
in decreasing dimension (``basis_vjp``), which is Y_k(v, m)^T of eq. Y
applied to a fine vector.  In Lagrange mode only the dual blocks contribute,
because the boundary values do not depend on m (Sec. 4.5).
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .geometry import Entity, Geometry
from .operator import assemble, conductivity, harmonic_T, harmonic_dT

MODES = ("reduced", "lagrange")


class LocalProblem:
    """The reduced operator A^E of one entity on its closure."""

    def __init__(self, geom: Geometry, ent: Entity, sigma: np.ndarray):
        d = geom.d
        self.ids = geom.cell_ids(ent.closure_ranges)
        shape = [len(rg) for rg in ent.closure_ranges]
        loc = np.arange(self.ids.size).reshape(shape, order="F")
        la, lb = [], []
        for k in ent.open_axes:
            if shape[k] < 2:
                continue
            sa = [slice(None)] * d
            sb = [slice(None)] * d
            sa[k] = slice(0, shape[k] - 1)
            sb[k] = slice(1, shape[k])
            la.append(loc[tuple(sa)].reshape(-1, order="F"))
            lb.append(loc[tuple(sb)].reshape(-1, order="F"))
        la = np.concatenate(la) if la else np.zeros(0, np.int64)
        lb = np.concatenate(lb) if lb else np.zeros(0, np.int64)
        masks = [np.isin(ent.closure_ranges[k], ent.cell_ranges[k]) for k in range(d)]
        unk = masks[0]
        for k in range(1, d):
            unk = np.multiply.outer(unk, masks[k])
        unk = np.asarray(unk, dtype=bool).reshape(-1, order="F")
        # keep the fluxes that touch the entity's own cells
        touch = unk[la] | unk[lb]
        self.la, self.lb = la[touch], lb[touch]
        self.ga, self.gb = self.ids[self.la], self.ids[self.lb]
        self.T = harmonic_T(sigma[self.ga], sigma[self.gb])
        self.dTa, self.dTb = harmonic_dT(sigma[self.ga], sigma[self.gb])
        self.U = np.nonzero(unk)[0]
        self.B = np.nonzero(~unk)[0]
        A = assemble(self.ids.size, self.la, self.lb, self.T).tocsr()
        self.A_UU = A[self.U][:, self.U].tocsc()
        self.A_UB = A[self.U][:, self.B].tocsr()
        self.A_BU = A[self.B][:, self.U].tocsr()
        self.lu = spla.splu(self.A_UU) if self.U.size else None

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        rhs = np.asarray(rhs, dtype=np.float64)
        if rhs.ndim == 1:
            return self.lu.solve(rhs)
        return self.lu.solve(np.ascontiguousarray(rhs))


class Basis:
    """S_k(m) stored row-wise: row i lists the corners of the entity that
    owns cell i (ascending vertex id) and the basis values there."""

    def __init__(self, geom: Geometry, m: np.ndarray, mode: str):
        if mode not in MODES:
            raise ValueError(f"mode must be one of {MODES}")
        self.geom = geom
        self.mode = mode
        self.m = np.asarray(m, dtype=np.float64).copy()
        self.sigma = conductivity(self.m)
        width = 2 ** geom.d
        self.cols = -np.ones((geom.ncell, width), dtype=np.int64)
        self.vals = np.zeros((geom.ncell, width))
        self.local: Dict[int, LocalProblem] = {}
        self._csr = None

    # -- helpers ---------------------------------------------------------
    def solved(self, ent: Entity) -> bool:
        if ent.dim == 0:
            return False
        return self.mode == "reduced" or ent.dim == self.geom.d

    def entity_list(self) -> List[int]:
        return [i for i, e in enumerate(self.geom.entities) if e.dim > 0]

    def values_at(self, cells: np.ndarray, corners: np.ndarray, vals=None) -> np.ndarray:
        """phi_c(cell) for every cell in ``cells`` and corner in ``corners``."""
        vals = self.vals if vals is None else vals
        c = self.cols[cells]                      # (k, W)
        v = vals[cells]                           # (k, W)
        hit = c[:, :, None] == corners[None, None, :]
        return np.einsum("kw,kwc->kc", v, hit.astype(np.float64))

    def csr(self) -> sp.csr_matrix:
        if self._csr is None:
            g = self.geom
            rows, cols, vals = [], [], []
            for w in range(self.cols.shape[1]):
                sel = self.cols[:, w] >= 0
                rows.append(np.nonzero(sel)[0])
                cols.append(self.cols[sel, w])
                vals.append(self.vals[sel, w])
            self._csr = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                      shape=(g.ncell, g.ncoarse))
            self._csr.sort_indices()
        return self._csr


def _lagrange_values(geom: Geometry, ent: Entity) -> np.ndarray:
    """Products of 1-D linear Lagrange factors (index coordinates) on the
    cells of ``ent`` for each of its corners; 1 along strips and planes."""
    grids = np.meshgrid(*ent.cell_ranges, indexing="ij")
    coords = [g.reshape(-1, order="F").astype(np.float64) for g in grids]
    out = np.ones((coords[0].size, len(ent.corners)))
    for j, multi in enumerate(ent.corner_index):
        for k in ent.open_axes:
            seg_idx = ent.key[k][1]
            seg = geom.axes[k].segments[seg_idx]
            if seg.kind != "bounded":
                continue
            lo, hi = seg.closure
            if multi[k] == seg.corners[0]:
                out[:, j] *= (hi - coords[k]) / (hi - lo)
            else:
                out[:, j] *= (coords[k] - lo) / (hi - lo)
    return out


def build_basis(geom: Geometry, m: np.ndarray, mode: str = "reduced",
                only: Optional[Sequence[int]] = None) -> Basis:
    """S_k(m) (Sec. 3.2) for every coarse vertex.

    With ``only`` (indices into ``geom.entities``), just the rows of those
    entities are built, together with the rows of every entity inside their
    closures, which is all their boundary data depends on; other rows stay
    empty.  Used to check single entities of grids too large to build whole.
    """
    bas = Basis(geom, m, mode)
    for multi in geom.vertex_multis():
        cell = geom.vertex_cell(multi)
        bas.cols[cell, 0] = geom.vertex_id(multi)
        bas.vals[cell, 0] = 1.0
    mark = None
    if only is not None:
        mark = np.zeros(geom.ncell, dtype=bool)
        for i in only:
            mark[geom.cell_ids(geom.entities[i].closure_ranges)] = True
    for idx, ent in enumerate(geom.entities):
        if ent.dim == 0:
            continue
        cells = geom.cell_ids(ent.cell_ranges)
        if mark is not None and not mark[cells].all():
            continue
        nc = len(ent.corners)
        if bas.solved(ent):
            lp = LocalProblem(geom, ent, bas.sigma)
            bas.local[idx] = lp
            phi_b = bas.values_at(lp.ids[lp.B], ent.corners)
            x = lp.solve(-(lp.A_UB @ phi_b))
            x = x.reshape(lp.U.size, nc)
        else:
            x = _lagrange_values(geom, ent)
        bas.cols[cells, :nc] = ent.corners[None, :]
        bas.vals[cells, :nc] = x
    return bas


def basis_tangent(bas: Basis, dm: np.ndarray) -> np.ndarray:
    """dS_k = (d/dm S_k(m)) dm, returned row-aligned with ``bas.cols``."""
    geom = bas.geom
    dm = np.asarray(dm, dtype=np.float64)
    dvals = np.zeros_like(bas.vals)
    for idx, ent in enumerate(geom.entities):
        if ent.dim == 0 or not bas.solved(ent):
            continue
        lp = bas.local[idx]
        phi = bas.values_at(lp.ids, ent.corners)
        dphi_b = bas.values_at(lp.ids[lp.B], ent.corners, dvals)
        dT = lp.dTa * dm[lp.ga] + lp.dTb * dm[lp.gb]
        flux = dT[:, None] * (phi[lp.la] - phi[lp.lb])
        dA_phi = np.zeros_like(phi)
        np.add.at(dA_phi, lp.la, flux)
        np.add.at(dA_phi, lp.lb, -flux)
        rhs = -(dA_phi[lp.U] + lp.A_UB @ dphi_b)
        dx = lp.solve(rhs).reshape(lp.U.size, -1)
        cells = lp.ids[lp.U]
        dvals[cells, :len(ent.corners)] = dx
    return dvals


def tangent_csr(bas: Basis, dvals: np.ndarray) -> sp.csr_matrix:
    """Tangent values in the sparsity of S_k as a sparse matrix."""
    g = bas.geom
    rows, cols, vals = [], [], []
    for w in range(bas.cols.shape[1]):
        sel = bas.cols[:, w] >= 0
        rows.append(np.nonzero(sel)[0])
        cols.append(bas.cols[sel, w])
        vals.append(dvals[sel, w])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(g.ncell, g.ncoarse))


def basis_vjp(bas: Basis, V: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """sum_j grad_m ( Z[:, j]^T S_k(m) V[:, j] ) = sum_j Y_k(V_j, m)^T Z_j.

    Reverse sweep over entities in decreasing dimension: mu = (A^E_EE)^{-1}
    z_E, the flux derivative term -dT_f (mu_a - mu_b)(x_a - x_b) on every flux
    of A^E (mu = 0 off E), and z_dE <- z_dE - A^E_{dE,E} mu."""
    geom = bas.geom
    V = np.asarray(V, dtype=np.float64).reshape(geom.ncoarse, -1)
    Z = np.array(Z, dtype=np.float64).reshape(geom.ncell, -1)
    X = bas.csr() @ V
    g = np.zeros(geom.ncell)
    order = sorted([i for i, e in enumerate(geom.entities) if e.dim > 0 and bas.solved(e)],
                   key=lambda i: -geom.entities[i].dim)
    for idx in order:
        lp = bas.local[idx]
        mu = lp.solve(Z[lp.ids[lp.U]]).reshape(lp.U.size, -1)
        mut = np.zeros((lp.ids.size, mu.shape[1]))
        mut[lp.U] = mu
        xl = X[lp.ids]
        w = np.sum((mut[lp.la] - mut[lp.lb]) * (xl[lp.la] - xl[lp.lb]), axis=1)
        np.add.at(g, lp.ga, -lp.dTa * w)
        np.add.at(g, lp.gb, -lp.dTb * w)
        Z[lp.ids[lp.B]] -= lp.A_BU @ mu
    return g
