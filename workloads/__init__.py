"""Seeded synthetic inputs for the MSFV diffusion / DC-resistivity problem.

This module only draws inputs: log-conductivity fields, electrode and receiver
layouts, and the per-workload recipes.  It holds none of the method's
arithmetic (no operator, basis, coarse solve or derivative), so both the CPU
oracle's tests and the GPU path's tests and benchmark may use it.

Conventions
-----------
* cell id = i + nx*(j + ny*k)  (x fastest); 2-D grids use (nx, ny).
* The "surface" is k == 0 in 3-D and j == 0 in 2-D (the electrodes and
  receivers of a DC-resistivity survey sit on the ground surface, Sec. 2.1).
* Sources and receivers are sparse columns given as CSR over columns:
  ptr[n+1], cell[ptr[n]], val[ptr[n]].  A dipole is (+1, -1) at two cells, a
  pole receiver is a single 1 at one cell.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 170707598


# ---------------------------------------------------------------------------
# index helpers
# ---------------------------------------------------------------------------

def cell_id(n: Sequence[int], ijk: Sequence[int]) -> int:
    """Linear cell id, x fastest."""
    idx = 0
    stride = 1
    for k in range(len(n)):
        idx += int(ijk[k]) * stride
        stride *= int(n[k])
    return idx


def num_cells(n: Sequence[int]) -> int:
    return int(np.prod([int(x) for x in n]))


# ---------------------------------------------------------------------------
# random fields
# ---------------------------------------------------------------------------

def gaussian_random_field(shape: Sequence[int], std: float, corr_len: float,
                          seed: int) -> np.ndarray:
    """Stationary Gaussian random field, flattened in cell-id order.

    White noise drawn with ``default_rng(seed).standard_normal`` on the grid
    padded by ceil(3*corr_len) cells per side is smoothed by FFT convolution
    with a Gaussian kernel whose standard deviation is ``corr_len`` cells,
    cropped, and standardised to mean 0 and standard deviation ``std``.
    The correlation length is that kernel width (the paper does not define
    one; the workloads only name it).
    """
    shape = tuple(int(s) for s in shape)
    pad = int(math.ceil(3.0 * corr_len)) if corr_len > 0 else 0
    padded = tuple(s + 2 * pad for s in shape)
    rng = np.random.default_rng(seed)
    # draw in (z, y, x) C-order so that the flattened field is x-fastest
    noise = rng.standard_normal(padded[::-1])
    if corr_len > 0:
        spec = np.fft.rfftn(noise)
        kernel_hat = None
        axes_shape = noise.shape
        for ax, size in enumerate(axes_shape):
            freq = (np.fft.rfftfreq(size) if ax == len(axes_shape) - 1
                    else np.fft.fftfreq(size))
            g = np.exp(-2.0 * (math.pi * corr_len * freq) ** 2)
            bshape = [1] * len(axes_shape)
            bshape[ax] = g.size
            g = g.reshape(bshape)
            kernel_hat = g if kernel_hat is None else kernel_hat * g
        field = np.fft.irfftn(spec * kernel_hat, s=axes_shape,
                              axes=list(range(len(axes_shape))))
    else:
        field = noise
    if pad:
        sl = tuple(slice(pad, pad + s) for s in shape[::-1])
        field = field[sl]
    field = field - field.mean()
    sd = field.std()
    if sd > 0:
        field = field * (std / sd)
    return np.ascontiguousarray(field).reshape(-1).astype(np.float64)


def add_box(m: np.ndarray, n: Sequence[int], lo: Sequence[int],
            hi: Sequence[int], value: float) -> np.ndarray:
    """Add ``value`` to m on the half-open box [lo, hi) (in place; returned)."""
    grid = m.reshape(tuple(int(x) for x in n[::-1]))
    sl = tuple(slice(int(lo[k]), int(hi[k])) for k in range(len(n)))[::-1]
    grid[sl] += value
    return m


# ---------------------------------------------------------------------------
# electrodes and receivers
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SparseColumns:
    """Sparse columns in CSR-over-columns form (host arrays)."""
    ptr: np.ndarray   # int32 [count+1]
    cell: np.ndarray  # int32 [nnz]
    val: np.ndarray   # float64 [nnz]

    @property
    def count(self) -> int:
        return int(self.ptr.size - 1)

    def dense(self, ncell: int) -> np.ndarray:
        out = np.zeros((ncell, self.count))
        for j in range(self.count):
            for p in range(self.ptr[j], self.ptr[j + 1]):
                out[self.cell[p], j] += self.val[p]
        return out


def _columns(cols: List[List[Tuple[int, float]]]) -> SparseColumns:
    ptr = [0]
    cells: List[int] = []
    vals: List[float] = []
    for col in cols:
        for c, v in col:
            cells.append(int(c))
            vals.append(float(v))
        ptr.append(len(cells))
    return SparseColumns(np.asarray(ptr, np.int32), np.asarray(cells, np.int32),
                         np.asarray(vals, np.float64))


def _spread(lo: int, hi: int, k: int) -> List[int]:
    return [lo + int(math.floor((hi - lo) * (i + 0.5) / k)) for i in range(k)]


def _grid_factor(count: int) -> Tuple[int, int]:
    """count = ax * ay with ay the largest divisor <= sqrt(count)."""
    ay = 1
    for d in range(1, int(math.isqrt(count)) + 1):
        if count % d == 0:
            ay = d
    return count // ay, ay


def surface_dipoles(n: Sequence[int], count: int) -> SparseColumns:
    """Dipole sources on the surface: A electrodes on an ax-by-ay grid over
    the central [n/8, 7n/8) of the surface, B offset by +max(1, n/8) in x."""
    d = len(n)
    nx = int(n[0])
    cols = []
    if d == 2:
        off = max(1, nx // 8)
        xs = _spread(nx // 8, 7 * nx // 8, count)
        for x in xs:
            a = cell_id(n, (x, 0))
            b = cell_id(n, (min(x + off, nx - 1), 0))
            cols.append([(a, 1.0), (b, -1.0)])
        return _columns(cols)
    ny = int(n[1])
    off = max(1, nx // 8)
    ax, ay = _grid_factor(count)
    xs = _spread(nx // 8, 7 * nx // 8, ax)
    ys = _spread(ny // 8, 7 * ny // 8, ay)
    for y in ys:
        for x in xs:
            a = cell_id(n, (x, y, 0))
            b = cell_id(n, (min(x + off, nx - 1), y, 0))
            cols.append([(a, 1.0), (b, -1.0)])
    return _columns(cols[:count])


def surface_pole_receivers(n: Sequence[int], count: int) -> SparseColumns:
    """Pole receivers on a sqrt(count) x sqrt(count) surface grid over
    [n/16, 15n/16) (2-D: ``count`` receivers along the surface line)."""
    d = len(n)
    nx = int(n[0])
    cols = []
    if d == 2:
        for x in _spread(nx // 16, 15 * nx // 16, count):
            cols.append([(cell_id(n, (x, 0)), 1.0)])
        return _columns(cols)
    ny = int(n[1])
    side = int(math.isqrt(count))
    if side * side != count:
        ax, ay = _grid_factor(count)
    else:
        ax = ay = side
    for y in _spread(ny // 16, 15 * ny // 16, ay):
        for x in _spread(nx // 16, 15 * nx // 16, ax):
            cols.append([(cell_id(n, (x, y, 0)), 1.0)])
    return _columns(cols)


def explicit_columns(cols: List[List[Tuple[int, float]]]) -> SparseColumns:
    return _columns(cols)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Instance:
    """One synthetic DC-resistivity instance."""
    name: str
    n: Tuple[int, ...]
    r: Tuple[int, ...]
    m: np.ndarray
    sources: SparseColumns
    receivers: SparseColumns
    seed: int
    m_obs: Optional[np.ndarray] = None  # model that produced observed data

    @property
    def ncell(self) -> int:
        return num_cells(self.n)


def config_seed(config: int, instance: int = 0) -> int:
    return BASE_SEED + 10 * config + instance


def workload_small_2d(seed_offset: int = 0) -> Instance:
    """2-D 32x32, r=4 (8x8 coarse), log-sigma GRF(std 1, corr 4), one dipole
    (+1 at (8,0), -1 at (24,0)), 16 surface receivers at x = 1, 3, ..., 31."""
    n = (32, 32)
    seed = config_seed(1, seed_offset)
    m = gaussian_random_field(n, 1.0, 4.0, seed)
    src = _columns([[(cell_id(n, (8, 0)), 1.0), (cell_id(n, (24, 0)), -1.0)]])
    rec = _columns([[(cell_id(n, (x, 0)), 1.0)] for x in range(1, 32, 2)])
    m_obs = m + 0.5 * gaussian_random_field(n, 1.0, 4.0, seed + 1)
    return Instance("2d-32x32-r4", n, (4, 4), m, src, rec, seed, m_obs)


def workload_64(seed_offset: int = 0) -> Instance:
    """3-D 64^3, r=8 (8^3 coarse): GRF(std 1, corr 8) plus a 10x box and a
    0.1x box, 16 surface dipoles, 256 surface pole receivers."""
    n = (64, 64, 64)
    seed = config_seed(2, seed_offset)
    m = gaussian_random_field(n, 1.0, 8.0, seed)
    add_box(m, n, (16, 24, 8), (28, 40, 20), math.log(10.0))
    add_box(m, n, (36, 24, 8), (48, 40, 20), -math.log(10.0))
    src = surface_dipoles(n, 16)
    rec = surface_pole_receivers(n, 256)
    m_obs = m + 0.5 * gaussian_random_field(n, 1.0, 8.0, seed + 1)
    return Instance("3d-64-r8", n, (8, 8, 8), m, src, rec, seed, m_obs)


def workload_128(seed_offset: int = 0, n_side: int = 128) -> Instance:
    """3-D 128^3, r=8 (16^3 coarse): GRF(std 1.5, corr 16) clipped to a
    conductivity contrast of 1e3, 32 surface dipoles, 1024 receivers."""
    n = (n_side,) * 3
    seed = config_seed(3, seed_offset)
    clip = 0.5 * math.log(1e3)
    m = np.clip(gaussian_random_field(n, 1.5, 16.0, seed), -clip, clip)
    src = surface_dipoles(n, 32)
    rec = surface_pole_receivers(n, 1024)
    m_obs = m + 0.5 * gaussian_random_field(n, 1.0, 16.0, seed + 1)
    return Instance(f"3d-{n_side}-r8", n, (8, 8, 8), m, src, rec, seed, m_obs)


def workload_batch(count: int = 64, seed_offset: int = 0,
                   n_range: Tuple[int, int] = (48, 160),
                   r_choices: Sequence[int] = (4, 8, 16),
                   ns_range: Tuple[int, int] = (1, 32)) -> List[Instance]:
    """Mixed batch: cubic n ~ U{48..160} resampled until n mod r != 0,
    r ~ U{4,8,16}, Ns ~ U{1..32}, GRF(std 1, corr 8), 16x16 receivers."""
    out = []
    for i in range(count):
        seed = config_seed(4, seed_offset + i)
        rng = np.random.default_rng(seed)
        r = int(rng.choice(np.asarray(r_choices)))
        while True:
            nn = int(rng.integers(n_range[0], n_range[1] + 1))
            if nn % r != 0:
                break
        ns = int(rng.integers(ns_range[0], ns_range[1] + 1))
        n = (nn, nn, nn)
        m = gaussian_random_field(n, 1.0, 8.0, seed)
        out.append(Instance(f"batch-{i}-{nn}-r{r}", n, (r, r, r), m,
                            surface_dipoles(n, ns), surface_pole_receivers(n, 256),
                            seed, m + 0.5 * gaussian_random_field(n, 1.0, 8.0, seed + 1)))
    return out


@dataclasses.dataclass
class Job:
    """A synthetic inversion job for the serving workload: a base model that
    is perturbed by 1 % GRF steps at each optimiser iteration."""
    name: str
    n: Tuple[int, ...]
    r: Tuple[int, ...]
    m0: np.ndarray
    receivers: SparseColumns
    seed: int

    def model(self, iteration: int) -> np.ndarray:
        m = self.m0.copy()
        for it in range(iteration):
            m += 0.01 * gaussian_random_field(self.n, 1.0, 8.0, self.seed * 1000 + it + 1)
        return m

    def sources(self, iteration: int, ns_range: Tuple[int, int] = (1, 64)) -> SparseColumns:
        rng = np.random.default_rng(self.seed * 7919 + iteration)
        ns = int(rng.integers(ns_range[0], ns_range[1] + 1))
        return surface_dipoles(self.n, ns)


def workload_serving(jobs: int = 16, seed_offset: int = 0,
                     n_range: Tuple[int, int] = (32, 192), r: int = 8) -> List[Job]:
    """16 inversion jobs with n ~ U{32..192}, r = 8."""
    out = []
    for k in range(jobs):
        seed = config_seed(5, seed_offset + k)
        rng = np.random.default_rng(seed)
        nn = int(rng.integers(n_range[0], n_range[1] + 1))
        n = (nn, nn, nn)
        out.append(Job(f"job-{k}-{nn}", n, (r, r, r),
                       gaussian_random_field(n, 1.0, 8.0, seed),
                       surface_pole_receivers(n, 256), seed))
    return out


def small_instance(n: Sequence[int], r: Sequence[int], seed: int, std: float = 1.0,
                   corr: float = 2.0, ns: int = 2, nr: int = 4) -> Instance:
    """Tiny instance for tests: GRF model, ``ns`` surface dipoles and ``nr``
    pole receivers."""
    n = tuple(int(x) for x in n)
    m = gaussian_random_field(n, std, corr, seed)
    d = len(n)
    if d == 1:
        nx = n[0]
        src = _columns([[(nx // 5, 1.0), (4 * nx // 5, -1.0)]])
        rec = _columns([[(x, 1.0)] for x in _spread(0, nx, nr)])
    else:
        src = surface_dipoles(n, ns)
        rec = surface_pole_receivers(n, nr)
    m_obs = m + 0.5 * gaussian_random_field(n, 1.0, corr, seed + 1)
    return Instance(f"small-{'x'.join(map(str, n))}", n, tuple(int(x) for x in r),
                    m, src, rec, seed, m_obs)
