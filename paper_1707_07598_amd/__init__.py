"""MI355X-native adaptive multiscale finite volume (MSFV) hot path.

Implements, as hand-written HIP kernels for gfx950 behind the C ABI of
include/msfv.h, the per-iteration rebuild of the parameter-dependent
prolongation S_k(m) (Sec. 3.2), the Galerkin reduced solve (eq. reducedPDE,
eq. fwdProbRed) and the explicit misfit gradient through the change of basis
(Sec. 4.3, eq. sensred; Sec. 4.5) of Wu Fung & Ruthotto (arXiv:1707.07598).

This module only marshals arguments: torch provides device memory and the
stream, every arithmetic step runs in libmsfv.so.

Layouts: m and g are flat (N,) float64 CUDA tensors in cell-id order
(x fastest); data D, residuals v and observed data are (Ns, Nr) float64
tensors (row j = source j), i.e. the column-contiguous Nr x Ns layout of
the C ABI.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import (MSFV_BC_LAGRANGE, MSFV_BC_REDUCED, MSFV_COARSE_JACOBI,  # noqa: F401
                   MSFV_COARSE_TWOLEVEL, MsfvError)

__all__ = ["Problem", "Batch", "Server", "MSFVForward", "msfv_misfit", "MsfvError"]

_MODES = {"reduced": MSFV_BC_REDUCED, "lagrange": MSFV_BC_LAGRANGE}
_COARSE_PRECONDS = {"twolevel": MSFV_COARSE_TWOLEVEL, "jacobi": MSFV_COARSE_JACOBI,
                    "multi": _lib.MSFV_COARSE_MULTI}


def _torch():
    import torch
    return torch


def _dptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _ivec(a) -> Tuple[np.ndarray, object]:
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _dvec(a) -> Tuple[np.ndarray, object]:
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Problem:
    """One MSFV problem (grid, coarsening, boundary mode) with its device
    state: plan, S_k, A_k, coarse coefficients and workspace stay resident
    between calls."""

    def __init__(self, n: Sequence[int], r: Sequence[int], bc_mode: str = "reduced",
                 local_rtol: float = 1e-13, local_maxit: int = 1000,
                 coarse_rtol: float = 1e-13, coarse_maxit: int = 20000,
                 coarse_precond: str = "twolevel", device: int = 0, stream=None):
        torch = _torch()
        self.lib = _lib.load()
        n = tuple(int(x) for x in n)
        r = tuple(int(x) for x in r)
        if len(n) not in (2, 3) or len(r) != len(n):
            raise ValueError("n and r must both have length 2 or 3")
        self.n, self.r, self.dim = n, r, len(n)
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        cfg = _lib.MsfvConfig()
        cfg.dim = self.dim
        for k in range(3):
            cfg.n[k] = n[k] if k < self.dim else 1
            cfg.r[k] = r[k] if k < self.dim else 1
        cfg.bc_mode = _MODES[bc_mode]
        cfg.local_rtol = local_rtol
        cfg.local_maxit = local_maxit
        cfg.coarse_rtol = coarse_rtol
        cfg.coarse_maxit = coarse_maxit
        if coarse_precond not in _COARSE_PRECONDS:
            raise ValueError(f"coarse_precond must be one of {sorted(_COARSE_PRECONDS)}")
        cfg.coarse_precond = _COARSE_PRECONDS[coarse_precond]
        self.bc_mode = bc_mode
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self.lib.msfv_create(ctypes.byref(cfg), ctypes.c_void_p(stream.cuda_stream),
                                            ctypes.byref(handle)), "msfv_create")
        self._h = handle
        self.generation = 0
        self.frozen = False
        self.last_m = None
        self._ns = 0
        self._nr = 0

    # -- lifetime ----------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            self.lib.msfv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- inputs ------------------------------------------------------------
    def set_sources(self, cols) -> None:
        ptr, pp = _ivec(cols.ptr)
        cell, cp = _ivec(cols.cell)
        val, vp = _dvec(cols.val)
        _lib.check(self.lib.msfv_set_sources(self._h, int(ptr.size - 1), pp, cp, vp), "msfv_set_sources")
        self._ns = int(ptr.size - 1)

    def set_receivers(self, cols) -> None:
        ptr, pp = _ivec(cols.ptr)
        cell, cp = _ivec(cols.cell)
        val, vp = _dvec(cols.val)
        _lib.check(self.lib.msfv_set_receivers(self._h, int(ptr.size - 1), pp, cp, vp), "msfv_set_receivers")
        self._nr = int(ptr.size - 1)

    @property
    def ns(self) -> int:
        return self._ns

    @property
    def nr(self) -> int:
        return self._nr

    def _check_tensor(self, t, numel: int, name: str):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if not t.is_contiguous() or t.numel() != numel:
            raise ValueError(f"{name} must be contiguous with {numel} elements")

    # -- the path ----------------------------------------------------------
    def forward(self, m, want_u: bool = False, out=None, sync: bool = True):
        """D = Rx^T S_k(m) A_k(m)^{-1} S_k(m)^T Q as an (Ns, Nr) tensor; with
        ``want_u`` also u = S_k t as an (Ns, N) tensor."""
        torch = _torch()
        ncell = int(np.prod(self.n))
        self._check_tensor(m, ncell, "m")
        D = out if out is not None else torch.empty((self._ns, self._nr), dtype=torch.float64, device=m.device)
        u = torch.empty((self._ns, ncell), dtype=torch.float64, device=m.device) if want_u else None
        _lib.check(self.lib.msfv_forward(self._h, _dptr(m), _dptr(D), _dptr(u) if u is not None else None),
                   "msfv_forward")
        self.generation += 1
        self.last_m = m
        if sync:
            self.sync()
        return (D, u) if want_u else D

    def forward_jtv(self, m, v, sync: bool = True):
        """(D, g): the forward at m and g = J_k(m)^T v for a v known before
        the forward, with both coarse problems solved in one launch; the
        same results as ``forward(m)`` then ``jtv(v)``."""
        torch = _torch()
        ncell = int(np.prod(self.n))
        self._check_tensor(m, ncell, "m")
        self._check_tensor(v, self._ns * self._nr, "v")
        D = torch.empty((self._ns, self._nr), dtype=torch.float64, device=m.device)
        g = torch.empty(ncell, dtype=torch.float64, device=m.device)
        _lib.check(self.lib.msfv_forward_jtv(self._h, _dptr(m), _dptr(v), _dptr(D), _dptr(g)),
                   "msfv_forward_jtv")
        self.generation += 1
        self.last_m = m
        if sync:
            self.sync()
        return D, g

    def jtv(self, v, out=None, sync: bool = True):
        """g = J_k(m)^T v at the m of the last forward; v is (Ns, Nr)."""
        torch = _torch()
        self._check_tensor(v, self._ns * self._nr, "v")
        ncell = int(np.prod(self.n))
        g = out if out is not None else torch.empty(ncell, dtype=torch.float64, device=v.device)
        _lib.check(self.lib.msfv_jtv(self._h, _dptr(v), _dptr(g)), "msfv_jtv")
        if sync:
            self.sync()
        return g

    def jvp(self, dm, out=None, sync: bool = True, fixed: bool = False):
        """dD = J_k(m) dm at the m of the last forward, as an (Ns, Nr) tensor;
        ``fixed`` holds the basis S_k fixed (dS = 0)."""
        torch = _torch()
        self._check_tensor(dm, int(np.prod(self.n)), "dm")
        dd = out if out is not None else torch.empty((self._ns, self._nr), dtype=torch.float64, device=dm.device)
        fn = self.lib.msfv_jvp_fixed if fixed else self.lib.msfv_jvp
        _lib.check(fn(self._h, _dptr(dm), _dptr(dd)), "msfv_jvp_fixed" if fixed else "msfv_jvp")
        if sync:
            self.sync()
        return dd

    def freeze_basis(self, frozen: bool = True) -> None:
        """Keep the basis S_k of the last forward for the following forwards
        (only A_k(m) is rebuilt; eq. optredfixed), whose J^T v and J dm are
        then the fixed-basis sensitivities of eq. senssimple; ``False``
        returns to rebuilding S_k(m) at every forward."""
        _lib.check(self.lib.msfv_set_basis(self._h, 1 if frozen else 0), "msfv_set_basis")
        self.frozen = bool(frozen)

    def jtv_fixed(self, v, out=None, sync: bool = True):
        """g = J_k^T v with the basis S_k held fixed, at the m of the last forward."""
        torch = _torch()
        self._check_tensor(v, self._ns * self._nr, "v")
        g = out if out is not None else torch.empty(int(np.prod(self.n)), dtype=torch.float64, device=v.device)
        _lib.check(self.lib.msfv_jtv_fixed(self._h, _dptr(v), _dptr(g)), "msfv_jtv_fixed")
        if sync:
            self.sync()
        return g

    def misfit_grad(self, m, d_obs, sync: bool = True):
        """(phi, g): phi = 1/2 ||D(m) - d_obs||_F^2 and g = J_k^T (D - d_obs)."""
        torch = _torch()
        ncell = int(np.prod(self.n))
        self._check_tensor(m, ncell, "m")
        self._check_tensor(d_obs, self._ns * self._nr, "d_obs")
        phi = torch.empty(1, dtype=torch.float64, device=m.device)
        g = torch.empty(ncell, dtype=torch.float64, device=m.device)
        _lib.check(self.lib.msfv_misfit_grad(self._h, _dptr(m), _dptr(d_obs), _dptr(phi), _dptr(g)),
                   "msfv_misfit_grad")
        self.generation += 1
        self.last_m = m
        if sync:
            self.sync()
        return phi, g

    def misfit_grad_noalloc(self, m, d_obs, phi, g, sync: bool = True):
        """``misfit_grad`` into caller-allocated ``phi`` (1 value) and ``g``
        (N values) through the library's allocation-free entry point: the
        residual lives in a fixed device array (Nr * Ns <= 65536), and the
        problem must have run a forward since its sources or receivers were
        set."""
        ncell = int(np.prod(self.n))
        self._check_tensor(m, ncell, "m")
        self._check_tensor(d_obs, self._ns * self._nr, "d_obs")
        self._check_tensor(phi, 1, "phi")
        self._check_tensor(g, ncell, "g")
        _lib.check(self.lib.msfv_misfit_grad_noalloc(self._h, _dptr(m), _dptr(d_obs), _dptr(phi), _dptr(g)),
                   "msfv_misfit_grad_noalloc")
        self.generation += 1
        self.last_m = m
        if sync:
            self.sync()
        return phi, g

    def sync(self) -> None:
        _lib.check(self.lib.msfv_sync(self._h), "msfv_sync")

    # -- introspection -----------------------------------------------------
    def profile_enable(self, enable: bool = True) -> None:
        """Bracket every stage with HIP events on the problem's stream."""
        _lib.check(self.lib.msfv_profile_enable(self._h, 1 if enable else 0), "msfv_profile_enable")

    def profile_read(self) -> dict:
        """Per-stage summed milliseconds and launch counts since the last
        read, and the work counters; resets them."""
        pr = _lib.MsfvProfile()
        _lib.check(self.lib.msfv_profile_read(self._h, ctypes.byref(pr)), "msfv_profile_read")
        stages = {}
        for i in range(_lib.NSTAGE):
            if pr.count[i]:
                name = self.lib.msfv_stage_name(i).decode()
                stages[name] = {"ms": pr.ms[i], "count": pr.count[i]}
        work = {"block_fwd_cell_its": pr.work[0], "block_adj_cell_its": pr.work[1],
                "face_fwd_cell_its": pr.work[2], "face_adj_cell_its": pr.work[3],
                "coarse_fwd_row_its": pr.work[4], "coarse_adj_row_its": pr.work[5]}
        return {"stages": stages, "work": work}

    def sizes(self) -> _lib.MsfvSizes:
        s = _lib.MsfvSizes()
        _lib.check(self.lib.msfv_get_sizes(self._h, ctypes.byref(s)), "msfv_get_sizes")
        return s

    def stats(self) -> _lib.MsfvStats:
        s = _lib.MsfvStats()
        _lib.check(self.lib.msfv_get_stats(self._h, ctypes.byref(s)), "msfv_get_stats")
        return s

    def prolongation(self):
        """S_k as (row_ptr, col, val) host arrays (CSR by fine cell)."""
        sz = self.sizes()
        rp = np.empty(sz.ncell + 1, np.int32)
        col = np.empty(sz.nnz_p, np.int32)
        val = np.empty(sz.nnz_p, np.float64)
        _lib.check(self.lib.msfv_get_prolongation(
            self._h, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            col.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            val.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "msfv_get_prolongation")
        return rp, col, val

    def coarse(self):
        """A_k (before fixing vertex 0) as (row_ptr, col, val) and the coarse
        coefficients t as an (Ns, Nc) array."""
        sz = self.sizes()
        rp = np.empty(sz.ncoarse + 1, np.int32)
        col = np.empty(sz.nnz_k, np.int32)
        val = np.empty(sz.nnz_k, np.float64)
        t = np.empty((max(self._ns, 1), sz.ncoarse), np.float64)
        _lib.check(self.lib.msfv_get_coarse(
            self._h, rp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            col.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            val.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "msfv_get_coarse")
        return (rp, col, val), t[: self._ns]


def _make_function():
    torch = _torch()

    class MSFVForward(torch.autograd.Function):
        """D = F_k(m) with backward g = J_k(m)^T grad_D (Sec. 4.1, eq. Jk).

        ``MSFVForward.apply(m, problem)`` returns the (Ns, Nr) data; the
        backward runs the library's adjoint at the same m (it re-runs the
        forward first if the problem has been used at another m since)."""

        @staticmethod
        def forward(ctx, m, problem):
            D = problem.forward(m.detach().contiguous())
            ctx.problem = problem
            ctx.generation = problem.generation
            ctx.save_for_backward(m)
            return D

        @staticmethod
        def backward(ctx, grad_D):
            (m,) = ctx.saved_tensors
            problem = ctx.problem
            if problem.generation != ctx.generation:
                problem.forward(m.detach().contiguous())
                ctx.generation = problem.generation
            g = problem.jtv(grad_D.contiguous())
            return g, None

    return MSFVForward


class _Lazy:
    _fn = None

    def __get__(self, obj, objtype=None):
        if _Lazy._fn is None:
            _Lazy._fn = _make_function()
        return _Lazy._fn


class _Namespace:
    MSFVForward = _Lazy()


def __getattr__(name):
    if name == "MSFVForward":
        return _Namespace.MSFVForward
    raise AttributeError(name)


def msfv_misfit(m, problem, d_obs):
    """phi(m) = 1/2 ||F_k(m) - d_obs||_F^2 through the autograd Function."""
    D = _Namespace.MSFVForward.apply(m, problem)
    return 0.5 * ((D - d_obs) ** 2).sum()


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr()
    return arr


class Batch:
    """forward + J^T v of many problems at once (``msfv_batch_*``): problems
    are issued largest first over a pool of HIP streams, each replaying its
    captured kernel sequence as a HIP graph.  Outputs D[i] (Ns_i, Nr_i) and
    g[i] (N_i) are allocated once and reused."""

    def __init__(self, problems: Sequence["Problem"], stream=None):
        torch = _torch()
        self.lib = _lib.load()
        self.problems = list(problems)
        if not self.problems:
            raise ValueError("empty batch")
        dev = self.problems[0].device
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        handles = (ctypes.c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        h = ctypes.c_void_p()
        _lib.check(self.lib.msfv_batch_create(len(self.problems), handles,
                                              ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)),
                   "msfv_batch_create")
        self._h = h
        self.D = [torch.empty((p._ns, p._nr), dtype=torch.float64, device=dev) for p in self.problems]
        self.g = [torch.empty(int(np.prod(p.n)), dtype=torch.float64, device=dev) for p in self.problems]
        self._dp = _ptr_array(self.D)
        self._gp = _ptr_array(self.g)

    def _check_inputs(self, ms, vs):
        torch = _torch()
        if len(ms) != len(self.problems) or len(vs) != len(self.problems):
            raise ValueError("one m and one v per problem")
        for p, m, v in zip(self.problems, ms, vs):
            p._check_tensor(m, int(np.prod(p.n)), "m")
            p._check_tensor(v, p._ns * p._nr, "v")
        # a problem's sources or receivers may have changed since the last
        # call: the library writes Nr * Ns values into D[i]
        stale = False
        for i, p in enumerate(self.problems):
            if tuple(self.D[i].shape) != (p._ns, p._nr):
                self.D[i] = torch.empty((p._ns, p._nr), dtype=torch.float64, device=self.D[i].device)
                stale = True
        if stale:
            self._dp = _ptr_array(self.D)

    def forward_jtv(self, ms, vs, sync: bool = True):
        """D_i = F(m_i) and g_i = J(m_i)^T v_i for every problem i."""
        self._check_inputs(ms, vs)
        self._keep = (ms, vs)
        _lib.check(self.lib.msfv_batch_forward_jtv(self._h, _ptr_array(ms), _ptr_array(vs),
                                                   self._dp, self._gp), "msfv_batch_forward_jtv")
        if sync:
            self.sync()
        return self.D, self.g

    def sync(self):
        _lib.check(self.lib.msfv_batch_sync(self._h), "msfv_batch_sync")

    def set_options(self, streams: int, graphs: bool, shared: int = 0):
        """Streams of the pool, HIP graphs for the per-problem path, and the
        number of pipelines of shared launches of the local solves across
        problems (0: per-problem path)."""
        _lib.check(self.lib.msfv_batch_set_options(self._h, int(streams), int(bool(graphs)), int(shared)),
                   "msfv_batch_set_options")

    def options(self):
        s, g, sh = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _lib.check(self.lib.msfv_batch_get_options(self._h, ctypes.byref(s), ctypes.byref(g), ctypes.byref(sh)),
                   "msfv_batch_get_options")
        return s.value, bool(g.value), sh.value

    def autotune(self, ms, vs):
        """Time each candidate (shared launches in 1, 2, 4 or 8 pipelines, or
        the per-problem path with or without graphs, times the stream count)
        once and keep the fastest; returns (streams, graphs, shared)."""
        self._check_inputs(ms, vs)
        s, g, sh = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _lib.check(self.lib.msfv_batch_autotune(self._h, _ptr_array(ms), _ptr_array(vs), self._dp,
                                                self._gp, ctypes.byref(s), ctypes.byref(g), ctypes.byref(sh)),
                   "msfv_batch_autotune")
        return s.value, bool(g.value), sh.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.msfv_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving runtime (``msfv_server_*``): forward + J^T v requests of
    registered jobs, admitted first come first served as jobs, in-flight
    slots (``max_inflight``) and the device-memory budget (``hbm_budget``
    bytes; None = the device's memory) allow; each job's requests are
    prepared and issued by a native worker thread of its own on the job's
    stream."""

    def __init__(self, max_inflight: int = 8, hbm_budget: Optional[float] = None):
        self.lib = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(self.lib.msfv_server_create(int(max_inflight), float(hbm_budget or 0.0), ctypes.byref(h)),
                   "msfv_server_create")
        self._h = h
        self._jobs = []
        self._live = {}
        self.device_times = {}

    def add_job(self, problem: "Problem", max_sources: int = 64) -> int:
        """Register ``problem`` for requests of up to ``max_sources`` sources."""
        j = ctypes.c_int()
        _lib.check(self.lib.msfv_server_add_job(self._h, problem._h, int(max_sources), ctypes.byref(j)),
                   "msfv_server_add_job")
        self._jobs.append(problem)
        return j.value

    def request_bytes(self, job: int, ns: int) -> Tuple[int, int]:
        """(resident bytes of the job, admission bytes of a request of ns sources)."""
        res, req = ctypes.c_longlong(), ctypes.c_longlong()
        _lib.check(self.lib.msfv_server_request_bytes(self._h, int(job), int(ns), ctypes.byref(res),
                                                      ctypes.byref(req)), "msfv_server_request_bytes")
        return res.value, req.value

    def submit(self, job: int, sources, m, v, d_out, g_out, stream=None) -> int:
        """Queue forward + J^T v of job ``job`` with these sources (host
        CSR-over-columns ptr/cell/val), ordered after the work queued so far
        on ``stream`` (default: the current stream); tensors stay referenced
        until the request is done."""
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(m.device)
        ptr = np.ascontiguousarray(sources.ptr, dtype=np.int32)
        cell = np.ascontiguousarray(sources.cell, dtype=np.int32)
        val = np.ascontiguousarray(sources.val, dtype=np.float64)
        rid = ctypes.c_longlong()
        _lib.check(self.lib.msfv_server_submit(
            self._h, int(job), int(ptr.size - 1),
            ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            cell.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            val.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            _dptr(m), _dptr(v), _dptr(d_out), _dptr(g_out), ctypes.c_void_p(stream.cuda_stream),
            ctypes.byref(rid)), "msfv_server_submit")
        self._live[rid.value] = (m, v, d_out, g_out)
        return rid.value

    def wait(self, req: int) -> float:
        """Block until request ``req`` is done; its latency in ms.  The device
        times (ms since the server's creation) of its first and last kernel
        are kept in ``device_times[req]``."""
        lat, t0, t1 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        try:
            _lib.check(self.lib.msfv_server_wait(self._h, ctypes.c_longlong(req), ctypes.byref(lat),
                                                 ctypes.byref(t0), ctypes.byref(t1)), "msfv_server_wait")
            self.device_times[req] = (t0.value, t1.value)
        finally:
            self._live.pop(req, None)
        return lat.value

    def drain(self):
        _lib.check(self.lib.msfv_server_drain(self._h), "msfv_server_drain")
        self._live.clear()

    def stats(self, reset: bool = False) -> dict:
        st = _lib.MsfvServeStats()
        _lib.check(self.lib.msfv_server_stats(self._h, ctypes.byref(st), int(bool(reset))),
                   "msfv_server_stats")
        return {k: getattr(st, k) for k, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.msfv_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
