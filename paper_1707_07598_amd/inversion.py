"""Projected Gauss-Newton-PCG for the reduced parameter estimation problem.

Sec. 2.2 (eq. optfull): minimise
    phi(m) = 1/2 ||D(m) - D_obs||_F^2 + alpha/2 ||L (m - m_ref)||^2
subject to m_L <= m <= m_H, where D(m) is the multiscale forward model of a
``Problem`` (eq. optredadapt) and L the forward-difference gradient of the
cell-centred grid.  Each Gauss-Newton step solves
    (J^T J + alpha L^T L) s = -grad phi
on the variables that are not held at a bound, by a few conjugate-gradient
iterations (J s and J^T w from the library), then takes a projected Armijo
line search.  ``basis="adaptive"`` (eq. optredadapt) rebuilds S_k(m) at
every forward and differentiates through it (Sec. 4.3); ``basis="fixed"``
is the fixed-basis surrogate of eq. optredfixed: S_k is built once at the
starting model and frozen, only A_k(m) is rebuilt, and J is eq. senssimple.  The driver
only orchestrates: every model-dependent operation (basis, Galerkin
operator, coarse solves, sensitivities) runs in the HIP library, and the
vector algebra in device tensors.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence, Tuple


def _torch():
    import torch
    return torch


class GradientRegularizer:
    """L = forward differences between face neighbours along every axis of
    an n[0] x n[1] (x n[2]) cell grid (cell id x fastest); L^T L is the
    graph Laplacian with no-flux ends."""

    def __init__(self, n: Sequence[int]):
        self.n = tuple(int(v) for v in n)

    def _grid(self, v):
        return v.view(*reversed(self.n))  # (nz, ny, nx) or (ny, nx)

    def norm2(self, v) -> float:
        g = self._grid(v)
        s = 0.0
        for ax in range(g.dim()):
            d = g.diff(dim=ax)
            s += float((d * d).sum())
        return s

    def apply_ltl(self, v):
        torch = _torch()
        g = self._grid(v)
        out = torch.zeros_like(g)
        for ax in range(g.dim()):
            d = g.diff(dim=ax)              # d_i = v_{i+1} - v_i
            lo = [slice(None)] * g.dim()
            hi = [slice(None)] * g.dim()
            lo[ax] = slice(0, g.shape[ax] - 1)
            hi[ax] = slice(1, g.shape[ax])
            out[tuple(lo)] -= d
            out[tuple(hi)] += d
        return out.reshape(-1)


@dataclasses.dataclass
class GNIteration:
    misfit: float
    regularizer: float
    objective: float
    grad_norm: float
    cg_iterations: int
    step: float
    active: int


def _objective(prob, m, d_obs, reg, alpha, m_ref):
    D = prob.forward(m)
    r = D - d_obs
    phi_d = 0.5 * float((r * r).sum())
    phi_r = 0.5 * alpha * reg.norm2(m - m_ref)
    return phi_d + phi_r, phi_d, phi_r, r


def gauss_newton(prob, m0, d_obs, alpha: float, m_ref=None,
                 bounds: Tuple[float, float] = (-float("inf"), float("inf")),
                 max_iter: int = 10, cg_iter: int = 15, cg_tol: float = 1e-2,
                 basis: str = "adaptive", max_backtrack: int = 8,
                 callback: Optional[Callable[[int, GNIteration], None]] = None):
    """Run projected Gauss-Newton-PCG from m0; returns (m, history).  The
    problem is left with an adaptive basis."""
    if basis not in ("adaptive", "fixed"):
        raise ValueError("basis must be 'adaptive' or 'fixed'")
    fixed = basis == "fixed"
    lo, hi = bounds
    reg = GradientRegularizer(prob.n)
    m = m0.clone().clamp_(lo, hi)
    m_ref = m.clone() if m_ref is None else m_ref
    history: List[GNIteration] = []
    prob.freeze_basis(False)
    f, phi_d, phi_r, r = _objective(prob, m, d_obs, reg, alpha, m_ref)
    if fixed:
        prob.freeze_basis(True)  # S_k(m0) from the forward just run
    try:
        return _gn_loop(prob, m, d_obs, reg, alpha, m_ref, lo, hi, max_iter, cg_iter, cg_tol,
                        max_backtrack, callback, history, f, phi_d, phi_r, r)
    finally:
        prob.freeze_basis(False)


def _gn_loop(prob, m, d_obs, reg, alpha, m_ref, lo, hi, max_iter, cg_iter, cg_tol, max_backtrack,
             callback, history, f, phi_d, phi_r, r):
    torch = _torch()
    for it in range(max_iter):
        # gradient at the current forward state
        gd = prob.jtv(r)
        g = gd + alpha * reg.apply_ltl(m - m_ref)
        eps = 1e-12
        active = ((m <= lo + eps) & (g > 0)) | ((m >= hi - eps) & (g < 0))
        free = (~active).to(m.dtype)

        def hess(v):
            v = v * free
            return prob.jtv(prob.jvp(v)) * free + alpha * reg.apply_ltl(v) * free

        # conjugate gradients on the free variables for H s = -g
        b = -g * free
        s = torch.zeros_like(m)
        res = b.clone()
        p = res.clone()
        rr = float((res * res).sum())
        rr0 = rr
        k = 0
        while k < cg_iter and rr > (cg_tol ** 2) * rr0 and rr0 > 0:
            hp = hess(p)
            php = float((p * hp).sum())
            if php <= 0:
                break
            a = rr / php
            s += a * p
            res -= a * hp
            rr_new = float((res * res).sum())
            p = res + (rr_new / rr) * p
            rr = rr_new
            k += 1
        if float((s * g).sum()) >= 0:  # not a descent direction: fall back to the gradient
            s = -g * free
        # projected Armijo line search
        t = 1.0
        accepted = False
        for _ in range(max_backtrack + 1):
            m_new = (m + t * s).clamp(lo, hi)
            f_new, pd_new, pr_new, r_new = _objective(prob, m_new, d_obs, reg, alpha, m_ref)
            if f_new <= f + 1e-4 * float((g * (m_new - m)).sum()):
                accepted = True
                break
            t *= 0.5
        if not accepted:
            prob.forward(m)  # restore the state of the current model
            history.append(GNIteration(phi_d, phi_r, f, float(g.norm()), k, 0.0, int(active.sum())))
            break
        m, f, phi_d, phi_r, r = m_new, f_new, pd_new, pr_new, r_new
        rec = GNIteration(phi_d, phi_r, f, float(g.norm()), k, t, int(active.sum()))
        history.append(rec)
        if callback is not None:
            callback(it, rec)
    return m, history
