"""Per-source and element-wise comparisons of device results with the oracle.

The bar for this path: the coarse coefficients t, the data D and the field u
within 1e-10 relative, the gradient within 1e-8 relative, both sides in
FP64.  A single relative norm over all sources would let a wrong
low-magnitude source column (or a local error far below the global norm)
pass, so every comparison here is made

* per source: the relative 2-norm error of each source's row, and
* element-wise: every entry of a row within ``rtol`` times the largest
  magnitude of that row of the reference.

A reference row that is exactly zero (a source cancelling inside one cell,
a grid whose only coarse vertex is fixed) must come out within ``rtol``
times the largest magnitude of the whole reference, and exactly zero when
the whole reference is zero.

Arrays are in the binding's layout: one row per source, ``(Ns, k)``.
"""
from __future__ import annotations

import numpy as np


def rows(got, ref, rtol: float, what: str = "") -> float:
    """Per-source rows of ``got`` against ``ref``; returns the worst
    relative row error (for reports)."""
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    if ref.ndim == 1:
        ref = ref[None, :]
        got = got[None, :]
    whole = float(np.abs(ref).max()) if ref.size else 0.0
    worst = 0.0
    for j in range(ref.shape[0]):
        r, d = ref[j], got[j] - ref[j]
        assert np.all(np.isfinite(got[j])), (what, j, "non-finite")
        nr = float(np.linalg.norm(r))
        if nr > 0.0:
            rel = float(np.linalg.norm(d)) / nr
            worst = max(worst, rel)
            assert rel <= rtol, f"{what}: source {j}: relative error {rel:.3e} > {rtol:.1e}"
            scale = float(np.abs(r).max())
        else:
            scale = whole
        dmax = float(np.abs(d).max()) if d.size else 0.0
        assert dmax <= rtol * scale, \
            f"{what}: source {j}: max |error| {dmax:.3e} > {rtol:.1e} x {scale:.3e}"
    return worst


def vector(got, ref, rtol: float, what: str = "") -> float:
    """One vector (a gradient, an operator): relative 2-norm error and
    every entry within ``rtol`` times the largest reference magnitude."""
    return rows(np.ravel(got), np.ravel(ref), rtol, what)


def gradient_per_source(prob, st, V, rtol: float, sources=None, fixed: bool = False) -> float:
    """J^T v split by source: for each source j, the device's J^T applied to
    V with every other source's column zeroed, against the oracle's.

    ``V`` is the oracle's (Nr, Ns) layout; ``prob`` has run its forward at
    ``st.m``.  ``fixed`` compares the fixed-basis J^T instead of the
    adaptive one."""
    import torch

    from oracle import reduced as R

    jtv_ref = R.jtv_fixed if fixed else R.jtv
    jtv_dev = prob.jtv_fixed if fixed else prob.jtv
    V = np.asarray(V, dtype=np.float64)
    ns = V.shape[1]
    worst = 0.0
    for j in (range(ns) if sources is None else sources):
        Vj = np.zeros_like(V)
        Vj[:, j] = V[:, j]
        ref = jtv_ref(st, Vj)
        got = jtv_dev(torch.tensor(Vj.T.copy(), dtype=torch.float64, device=prob.device)).cpu().numpy()
        worst = max(worst, vector(got, ref, rtol, f"gradient of source {j}"))
    return worst
