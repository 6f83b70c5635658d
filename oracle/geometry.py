"""Fine grid, coarse vertices, segments and entities (oracle; test
infrastructure only).

Sec. 3.2 step 1 partitions the fine mesh into a nested coarse mesh.  In the
cell-centred setting used here the coarse mesh is the vertex / dual-block
complex of classic MSFV:

* Per axis with n cells and coarsening r there are Nc = ceil(n/r) coarse
  vertices.  Coarse cell I covers cells [I*r, I*r + L_I) with
  L_I = min(r, n - I*r); its vertex sits at v_I = I*r + floor(L_I/2).
* A cell is either *on* a vertex plane v_I or *open* in a segment: the lower
  strip [0, v_0), a bounded segment (v_{s-1}, v_s), or the upper strip
  (v_last, n-1].  The closure of a segment adds its bounding vertex planes;
  a strip has one bounding plane (its other end is the domain boundary).
* An entity is the tuple over axes of (plane I) or (segment s).  Its
  dimension is the number of open axes: 0 vertex, 1 edge, 2 face, 3 interior
  (a dual block).  Every cell belongs to exactly one entity.
* The corners of an entity are the coarse vertices in its closure,
  2^(number of bounded open axes) of them.

Vertex ids are I0 + Nc0*(I1 + Nc1*I2); cell ids are i0 + n0*(i1 + n1*i2).
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import List, Sequence, Tuple

import numpy as np

PLANE = "P"
SEG = "S"


@dataclasses.dataclass(frozen=True)
class Segment:
    kind: str                 # "low", "bounded" or "high"
    first: int                # first open cell (inclusive)
    last: int                 # last open cell (inclusive); last < first if empty
    closure: Tuple[int, int]  # closed cell range [lo, hi]
    corners: Tuple[int, ...]  # vertex indices bounding the segment

    @property
    def empty(self) -> bool:
        return self.last < self.first

    def cells(self) -> np.ndarray:
        return np.arange(self.first, self.last + 1, dtype=np.int64)


class Axis:
    """Vertex planes and segments along one axis."""

    def __init__(self, n: int, r: int):
        if n < 1 or r < 1:
            raise ValueError("n and r must be positive")
        self.n = int(n)
        self.r = int(r)
        self.nc = -(-self.n // self.r)
        self.v = [I * self.r + min(self.r, self.n - I * self.r) // 2 for I in range(self.nc)]
        v = self.v
        segs = [Segment("low", 0, v[0] - 1, (0, v[0]), (0,))]
        for s in range(1, self.nc):
            segs.append(Segment("bounded", v[s - 1] + 1, v[s] - 1, (v[s - 1], v[s]), (s - 1, s)))
        segs.append(Segment("high", v[-1] + 1, self.n - 1, (v[-1], self.n - 1), (self.nc - 1,)))
        self.segments = segs

    def status(self) -> List[Tuple[str, int]]:
        """Per cell: (PLANE, I) or (SEG, s)."""
        out: List[Tuple[str, int]] = [None] * self.n  # type: ignore
        for I, pos in enumerate(self.v):
            out[pos] = (PLANE, I)
        for s, seg in enumerate(self.segments):
            for i in range(seg.first, seg.last + 1):
                out[i] = (SEG, s)
        return out


@dataclasses.dataclass
class Entity:
    key: Tuple[Tuple[str, int], ...]
    dim: int
    open_axes: Tuple[int, ...]
    cell_ranges: List[np.ndarray]      # per axis, the entity's own cells
    closure_ranges: List[np.ndarray]   # per axis, the closed range
    corner_choices: List[Tuple[int, ...]]  # per axis, vertex indices
    corners: np.ndarray                # vertex ids, ascending
    corner_index: List[Tuple[int, ...]]  # per corner, its multi-index

    def ncells(self) -> int:
        return int(np.prod([len(r) for r in self.cell_ranges]))


class Geometry:
    """Fine grid of n cells per axis with coarsening r per axis."""

    def __init__(self, n: Sequence[int], r: Sequence[int]):
        if len(n) != len(r) or not 1 <= len(n) <= 3:
            raise ValueError("n and r must have the same length 1..3")
        self.n = tuple(int(x) for x in n)
        self.r = tuple(int(x) for x in r)
        self.d = len(self.n)
        self.axes = [Axis(self.n[k], self.r[k]) for k in range(self.d)]
        self.nc = tuple(ax.nc for ax in self.axes)
        self.ncell = int(np.prod(self.n))
        self.ncoarse = int(np.prod(self.nc))
        self.strides = [int(np.prod(self.n[:k])) for k in range(self.d)]
        self.vstrides = [int(np.prod(self.nc[:k])) for k in range(self.d)]
        self.entities = self._enumerate()

    # -- ids -------------------------------------------------------------
    def cell_ids(self, ranges: Sequence[np.ndarray]) -> np.ndarray:
        """Global cell ids of the box given by per-axis index ranges,
        flattened with axis 0 fastest."""
        grids = np.meshgrid(*[np.asarray(rg, dtype=np.int64) for rg in ranges], indexing="ij")
        ids = np.zeros(grids[0].shape, dtype=np.int64)
        for k in range(self.d):
            ids += grids[k] * self.strides[k]
        return ids.reshape(-1, order="F")

    def vertex_id(self, multi: Sequence[int]) -> int:
        return int(sum(int(multi[k]) * self.vstrides[k] for k in range(self.d)))

    def vertex_cell(self, multi: Sequence[int]) -> int:
        return int(sum(self.axes[k].v[int(multi[k])] * self.strides[k] for k in range(self.d)))

    def cell_multi(self, cell: int) -> Tuple[int, ...]:
        out = []
        for k in range(self.d):
            out.append((cell // self.strides[k]) % self.n[k])
        return tuple(out)

    # -- entities --------------------------------------------------------
    def _enumerate(self) -> List[Entity]:
        per_axis = []
        for ax in self.axes:
            items = [(PLANE, I) for I in range(ax.nc)]
            items += [(SEG, s) for s in range(len(ax.segments)) if not ax.segments[s].empty]
            per_axis.append(items)
        ents: List[Entity] = []
        for key in itertools.product(*per_axis):
            cell_ranges, closure_ranges, choices, open_axes = [], [], [], []
            for k, (kind, idx) in enumerate(key):
                ax = self.axes[k]
                if kind == PLANE:
                    pos = np.array([ax.v[idx]], dtype=np.int64)
                    cell_ranges.append(pos)
                    closure_ranges.append(pos)
                    choices.append((idx,))
                else:
                    seg = ax.segments[idx]
                    open_axes.append(k)
                    cell_ranges.append(seg.cells())
                    closure_ranges.append(np.arange(seg.closure[0], seg.closure[1] + 1, dtype=np.int64))
                    choices.append(seg.corners)
            corner_multi = list(itertools.product(*choices))
            vids = [self.vertex_id(c) for c in corner_multi]
            order = np.argsort(vids)
            ents.append(Entity(key=tuple(key), dim=len(open_axes), open_axes=tuple(open_axes),
                               cell_ranges=cell_ranges, closure_ranges=closure_ranges,
                               corner_choices=choices,
                               corners=np.asarray(vids, dtype=np.int64)[order],
                               corner_index=[corner_multi[i] for i in order]))
        ents.sort(key=lambda e: e.dim)
        return ents

    def entities_of_dim(self, dim: int) -> List[Entity]:
        return [e for e in self.entities if e.dim == dim]

    def vertex_multis(self) -> List[Tuple[int, ...]]:
        return list(itertools.product(*[range(nc) for nc in self.nc]))
