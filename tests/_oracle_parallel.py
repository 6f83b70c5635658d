"""The oracle's basis built block-parallel over worker processes (test
infrastructure for the largest parity cases).

Each worker builds the oracle's basis rows of a contiguous run of dual
blocks -- with ``build_basis(..., only=...)``, which also builds the faces
and edges in those blocks' closures -- and the rows are merged into one
basis.  Entities built by several workers come out identical (each is the
same local solve on the same data), and the merged basis feeds the oracle's
forward as a given basis.  Only the forward uses it: the oracle's J^T v needs
the local factorisations of every entity in one process.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np


def _chunk(args):
    from oracle import Geometry
    from oracle.basis import build_basis

    n, r, m, mode, only = args
    bas = build_basis(Geometry(n, r), m, mode, only=only)
    rows = np.nonzero((bas.cols >= 0).any(axis=1))[0]
    return rows, bas.cols[rows], bas.vals[rows]


def parallel_basis(geom, m, mode: str = "reduced", workers: int = 0):
    """The oracle's S_k(m) (``oracle.basis.Basis``) built over a process pool."""
    from oracle.basis import Basis

    workers = workers or min(16, len(os.sched_getaffinity(0)))
    blocks = [i for i, e in enumerate(geom.entities) if e.dim == geom.d]
    cuts = [len(blocks) * k // workers for k in range(workers + 1)]
    chunks = [blocks[cuts[k]:cuts[k + 1]] for k in range(workers)]
    with mp.get_context("spawn").Pool(workers) as pool:
        parts = pool.map(_chunk, [(geom.n, geom.r, np.asarray(m, dtype=np.float64), mode, c)
                                  for c in chunks if c])
    bas = Basis(geom, m, mode)
    for rows, cols, vals in parts:
        bas.cols[rows] = cols
        bas.vals[rows] = vals
    assert (bas.cols[:, 0] >= 0).all(), "a cell without basis values"
    return bas
