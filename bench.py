#!/usr/bin/env python3
"""MSFV forward + J^T v throughput on one MI355X.

Workload: 3-D 128^3 cell-centred diffusion grid, coarsening 8 (16^3 coarse
vertices), log-conductivity = Gaussian random field (std 1.5, correlation
length 16 cells, contrast clipped at 1e3), 32 surface dipole sources, 1024
surface pole receivers, reduced-boundary multiscale basis, FP64.

One step = one misfit-gradient evaluation: rebuild of the basis S_k(m), the
Galerkin coarse operator, the coarse solves for all 32 sources, the data,
the residual against observed data, and J_k^T of that residual through the
change of basis (one "solve" in solves/s).  Inputs are resident in HBM before
the timed region.  Prints one JSON line.

Besides the headline, the line carries (unless --no-extra) compact figures
of the other workloads measured in the same run: forward only at 64^3 (r 8,
16 dipoles, 256 receivers), the 64-instance mixed batch through the batch
entry points against the same instances one after another, and the serving
loop (16 jobs, Poisson arrivals at 0.5x, 1x and 2x its measured capacity,
200 GB admission budget).  --workload batch / serve print the full lines of
those workloads instead.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MSFV forward+J^T v solves/s at 128^3 r=8; % HBM roofline; serve p50/p99 latency"
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector peak
HBM_PEAK_BPS = 8e12          # MI355X HBM3E peak
LDS_PEAK_TBS = 78.6          # 256 CUs x 128 B/clk x 2.4 GHz
# algorithmic flops of one conjugate-gradient cell-iteration of the local
# solves (6 neighbour FMAs of the scaled operator, 5 vector FMAs) and of one
# coarse row-iteration (27 FMAs of the stencil, 5 vector FMAs)
FLOPS_PER_LOCAL_CELL_IT = 22.0
FLOPS_PER_COARSE_ROW_IT = 64.0
LDS_BYTES_PER_LOCAL_CELL_IT = 40.0  # 4 neighbour reads + 1 write of the search direction

STAGE_WORK = {
    "block_fwd": ("block_fwd_cell_its", FLOPS_PER_LOCAL_CELL_IT),
    "block_adj": ("block_adj_cell_its", FLOPS_PER_LOCAL_CELL_IT),
    "face_fwd": ("face_fwd_cell_its", FLOPS_PER_LOCAL_CELL_IT),
    "face_adj": ("face_adj_cell_its", FLOPS_PER_LOCAL_CELL_IT),
    "coarse_fwd": ("coarse_fwd_row_its", FLOPS_PER_COARSE_ROW_IT),
    "coarse_adj": ("coarse_adj_row_its", FLOPS_PER_COARSE_ROW_IT),
}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_128cubed_r8.json")
SERVE_HBM_BUDGET = 200e9  # admission budget of the serving workload (bytes)


def measured_traffic(kernel_stage: str):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter runs, or None when they were taken on a
    different kernel source than the one built now."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get("stages", {}).get(kernel_stage)
    if not ent:
        return None
    src = os.path.join(ROOT, "paper_1707_07598_amd", "csrc", ent["source"])
    try:
        with open(src, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if digest != ent["source_sha256"]:
        return None
    return ent["bytes_per_launch"]


def _basis_chunk(args):
    """Worker of the block-parallel CPU basis build: the oracle's basis rows
    of a chunk of dual blocks (and of the faces and edges in their
    closures, which each worker builds again for itself)."""
    import numpy as np

    from oracle import Geometry
    from oracle.basis import build_basis

    n, r, m, only = args
    g = Geometry(n, r)
    t0 = time.perf_counter()
    bas = build_basis(g, m, "reduced", only=only)
    rows = np.nonzero((bas.cols >= 0).any(axis=1))[0]
    return rows, bas.cols[rows], bas.vals[rows], time.perf_counter() - t0


def cpu_baseline(inst, parallel: bool = True) -> dict:
    """The CPU oracle on the whole benchmarked workload (no sample scaling):
    forward + J^T v once in one process (NumPy/SciPy, BLAS threads = cores),
    its basis build timed on its own; then the basis build block-parallel
    over a pool of one worker process per core (the worker parallelism of
    the paper's Table 3), checked against the one-process basis."""
    import numpy as np

    from oracle import Geometry
    from oracle import reduced as R
    from oracle.basis import build_basis

    cores = len(os.sched_getaffinity(0))
    g = Geometry(inst.n, inst.r)
    t0 = time.perf_counter()
    bas = build_basis(g, inst.m, "reduced")
    t1 = time.perf_counter()
    st = R.forward(g, inst.m, inst.sources, inst.receivers, basis=bas)
    R.jtv(st, np.ones_like(st.D))
    t2 = time.perf_counter()
    dt = t2 - t0
    out = {"value": 1.0 / dt, "unit": "solves/s", "cores": cores, "kind": "oracle",
           "sample": f"oracle forward + J^T v on the whole 128^3 workload (r=8, 32 dipoles, 1024 "
                     f"receivers), once: {dt:.1f} s, of which the basis build {t1 - t0:.1f} s; one "
                     "process, NumPy/SciPy with BLAS threads = cores",
           "seconds": dt, "basis_build_s": t1 - t0}
    if parallel:
        import multiprocessing as mp
        blocks = [i for i, e in enumerate(g.entities) if e.dim == g.d]
        # contiguous runs of blocks (slabs of the grid): only the faces and
        # edges on slab boundaries are built twice
        cuts = [len(blocks) * k // cores for k in range(cores + 1)]
        chunks = [blocks[cuts[k]:cuts[k + 1]] for k in range(cores)]
        ctx = mp.get_context("spawn")  # fresh interpreters: nothing of this process's device state
        with ctx.Pool(cores) as pool:
            t3 = time.perf_counter()
            parts = pool.map(_basis_chunk, [(inst.n, inst.r, inst.m, c) for c in chunks])
            t4 = time.perf_counter()
        cols = -np.ones_like(bas.cols)
        vals = np.zeros_like(bas.vals)
        for rows, c, v, _ in parts:
            cols[rows] = c
            vals[rows] = v
        agree = bool(np.array_equal(cols, bas.cols) and np.abs(vals - bas.vals).max() <= 1e-12)
        out["parallel_basis_build"] = {
            "workers": cores, "seconds": t4 - t3, "speedup_vs_one_process": (t1 - t0) / (t4 - t3),
            "worker_seconds_max": max(p[3] for p in parts), "matches_one_process": agree,
            "note": "dual blocks in contiguous runs (slabs) per worker; each also builds the faces "
                    "and edges in its blocks' closures; the reduced solve and J^T v stay in one "
                    "process"}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle leg (profiling runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="default workload only: skip the forward-only 64^3, batch and serving figures "
                         "appended to its line")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without per-stage events")
    ap.add_argument("--workload", choices=["c3", "batch", "serve"], default="c3",
                    help="c3: the 128^3 single-instance step (default); batch: 64 mixed "
                         "instances per call through the batch API; serve: 16 jobs, Poisson "
                         "arrivals at 0.5x, 1x and 2x the measured capacity")
    ap.add_argument("--serve-jobs", type=int, default=16)
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests per load point")
    ap.add_argument("--serve-inflight", type=int, default=8)
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run 3 device copies of 512 MiB (a kernel of known "
                         "traffic for scaling the HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one MI355X: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1707_07598_amd as msfv
    import workloads as W

    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "serve":
        sv = run_serve(args.serve_jobs, args.serve_requests, args.serve_inflight)
        one = sv["load_points"]["1.0"]
        out = {"metric": "MSFV serve p99 latency at 1x measured capacity (forward + J^T v requests)",
               "value": one["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": args.serve_requests,
               "warmup": args.serve_jobs, "ms_per_step": one["mean_ms"], "higher_is_better": False,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": f"serve-{sv['jobs']}-jobs-n32..192-r8-ns1..64-poisson"},
               "serve": sv}
        print(json.dumps(out), flush=True)
        return 0

    inst = W.workload_128()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    prob = msfv.Problem(inst.n, inst.r, "reduced")
    prob.set_sources(inst.sources)
    prob.set_receivers(inst.receivers)
    m = torch.tensor(inst.m, dtype=torch.float64, device=dev)
    m_obs = torch.tensor(inst.m_obs, dtype=torch.float64, device=dev)
    d_obs = prob.forward(m_obs).clone()

    for _ in range(args.warmup):
        prob.misfit_grad(m, d_obs, sync=False)
    prob.sync()
    if not args.no_profile:
        prob.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        phi, g = prob.misfit_grad(m, d_obs, sync=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prob.sync()  # raises on a non-converged or non-finite step
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps / elapsed
    stats = prob.stats()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3d-128^3-r8-32dipoles-1024rx-forward+JTv",
                   "n": list(inst.n), "r": list(inst.r), "sources": int(prob.ns),
                   "receivers": int(prob.nr), "bc_mode": "reduced",
                   "local_rtol": 1e-13, "coarse_rtol": 1e-13},
        "source_solves_per_s": value * prob.ns,
        "local_cg_max_it": stats.local_max_it,
        "coarse_cg_max_it": stats.coarse_max_it,
    }

    if not args.no_profile:
        prof = prob.profile_read()
        stages = prof["stages"]
        work = prof["work"]
        out["stages_ms_per_step"] = {k: v["ms"] / args.steps for k, v in
                                     sorted(stages.items(), key=lambda kv: -kv[1]["ms"])}
        dom = max((k for k in stages if k in STAGE_WORK), key=lambda k: stages[k]["ms"])
        launches = stages[dom]["count"]
        avg_s = stages[dom]["ms"] / launches / 1e3
        key, flops_per_unit = STAGE_WORK[dom]
        units_per_launch = work[key] / launches
        achieved = flops_per_unit * units_per_launch / avg_s / 1e12
        out["roofline"] = {
            "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS, "traffic": measured_traffic(dom),
            "kernel": dom, "avg_launch_ms": avg_s * 1e3, "units_per_launch": units_per_launch,
            "unit_kind": key, "flops_per_unit": flops_per_unit,
        }
        sz = prob.sizes()
        if dom.startswith(("block", "face")):
            lds = LDS_BYTES_PER_LOCAL_CELL_IT * units_per_launch / avg_s / 1e12
            out["roofline"]["lds_tb_per_s"] = lds
            out["roofline"]["lds_frac"] = lds / LDS_PEAK_TBS
            # iteration-independent figures of the same launch: (own cell,
            # corner) pairs solved per second, and the algorithmic HBM bytes
            # (m read, one S_k value written per pair) against the HBM peak
            pairs = sz.pairs_block if dom.startswith("block") else sz.pairs_face
            alg = 8 * sz.ncell + 8 * pairs
            out["roofline"]["pairs_per_launch"] = pairs
            out["roofline"]["pair_solves_per_s"] = pairs / avg_s
            out["roofline"]["algorithmic_bytes_per_launch"] = alg
            out["roofline"]["algorithmic_hbm_frac"] = alg / avg_s / HBM_PEAK_BPS
        # the streaming kernels against the HBM peak: g from the flux weights
        # (every step) and u = S_k t (one extra forward with the fields)
        streaming = {}
        if "gfinal" in stages:
            gms = stages["gfinal"]["ms"] / stages["gfinal"]["count"]
            b = 40 * sz.ncell  # m and 3 flux weights read, g written: 8 B each per cell
            streaming["gfinal"] = {"ms": gms, "algorithmic_bytes": b,
                                   "gb_per_s": b / (gms / 1e3) / 1e9,
                                   "frac_of_hbm_peak": b / (gms / 1e3) / HBM_PEAK_BPS}
        prob.profile_enable(True)
        _, u = prob.forward(m, want_u=True)
        pst = prob.profile_read()["stages"]
        del u
        if "prolong" in pst:
            pms = pst["prolong"]["ms"] / pst["prolong"]["count"]
            b = 12 * sz.nnz_p + 4 * (sz.ncell + 1) + 8 * sz.ncell * prob.ns
            streaming["prolong"] = {"ms": pms, "algorithmic_bytes": b,
                                    "gb_per_s": b / (pms / 1e3) / 1e9,
                                    "frac_of_hbm_peak": b / (pms / 1e3) / HBM_PEAK_BPS,
                                    "note": "S_k values and columns (12 B a nonzero) and row "
                                            "pointers read once, u written (8 B per cell and source)"}
        out["streaming"] = streaming
        # HBM view of the whole step: its algorithmic bytes
        hbm_bytes = 8 * sz.ncell * 3 + 12 * sz.nnz_p * 2
        out["hbm_algorithmic_bytes_per_step"] = hbm_bytes
        out["hbm_frac_of_step"] = hbm_bytes / (ms_per_step / 1e3) / HBM_PEAK_BPS

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst)
    prob.close()
    if not args.no_extra:
        # the other workloads, compact: forward only at 64^3, the 64-instance
        # batch (autotuned form against one instance after another) and the
        # serving loop (capacity, latency percentiles at 0.5x, 1x, 2x load)
        torch.cuda.synchronize()
        out["forward_only_64"] = forward_only_64()
        out["batch"] = measure_batch(8, 1, args.batch_count, sweep=False)
        sv = run_serve(args.serve_jobs, args.serve_requests, args.serve_inflight)
        out["serve"] = {"jobs": sv["jobs"], "requests_per_point": sv["requests_per_point"],
                        "hbm_budget_bytes": sv["hbm_budget_bytes"], "capacity_per_s": sv["capacity_per_s"],
                        "load_points": {k: {kk: v[kk] for kk in ("served_per_s", "p50_ms", "p99_ms", "failed")}
                                        for k, v in sv["load_points"].items()}}
    print(json.dumps(out), flush=True)
    return 0


def run_serve(jobs: int, nreq: int, inflight: int, log=sys.stderr) -> dict:
    """Serving: inversion jobs with n ~ U{32..192}, r = 8, 16 x 16 receivers;
    request i of a job is forward + J^T v at model m_i (m_0, or m_0 plus a 1 %
    GRF step, alternating) with Ns ~ U{1..64} dipoles.  Capacity is the
    closed-loop rate of nreq requests submitted at once; then Poisson arrivals
    at 0.5x, 1x and 2x that rate, nreq requests each, latency from
    submission to completion."""
    import numpy as np
    import torch

    import paper_1707_07598_amd as msfv
    import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    js = W.workload_serving(jobs)
    srv = msfv.Server(max_inflight=inflight, hbm_budget=SERVE_HBM_BUDGET)
    state = []
    rng = np.random.default_rng(W.config_seed(5, 999))
    for k, job in enumerate(js):
        p = msfv.Problem(job.n, job.r, "reduced", stream=torch.cuda.Stream(dev))
        p.set_receivers(job.receivers)
        srv.add_job(p)
        m0 = torch.tensor(job.m0, dtype=torch.float64, device=dev)
        m1 = torch.tensor(job.model(1), dtype=torch.float64, device=dev)
        nr = job.receivers.count
        v = torch.tensor(rng.standard_normal((64, nr)), dtype=torch.float64, device=dev)
        d = torch.empty((64, nr), dtype=torch.float64, device=dev)
        g = torch.empty(int(np.prod(job.n)), dtype=torch.float64, device=dev)
        state.append({"p": p, "m": (m0, m1), "v": v, "d": d, "g": g, "it": 0, "job": job})
        print(f"job {k}: n={job.n[0]}", file=log, flush=True)
    setup_s = time.perf_counter() - t0

    def submit_one():
        k = int(rng.integers(0, len(state)))
        s = state[k]
        i = s["it"]
        s["it"] += 1
        src = s["job"].sources(i)
        ns = src.count
        return srv.submit(k, src, s["m"][i % 2], s["v"][:ns], s["d"][:ns], s["g"])

    # warm-up: every job once (builds electrode tables, first-touch allocations)
    for k in range(len(state)):
        s = state[k]
        src = s["job"].sources(0)
        srv.wait(srv.submit(k, src, s["m"][0], s["v"][:src.count], s["d"][:src.count], s["g"]))
    srv.stats(reset=True)
    # capacity: closed loop
    t1 = time.perf_counter()
    ids = [submit_one() for _ in range(nreq)]
    for rid in ids:
        srv.wait(rid)
    cap = nreq / (time.perf_counter() - t1)
    closed = srv.stats(reset=True)
    points = {}
    for f in (0.5, 1.0, 2.0):
        lam = f * cap
        gaps = rng.exponential(1.0 / lam, nreq)
        ids = []
        t_next = time.perf_counter()
        for gap in gaps:
            t_next += gap
            while True:
                dt = t_next - time.perf_counter()
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.002))
            ids.append(submit_one())
        for rid in ids:
            srv.wait(rid)
        st = srv.stats(reset=True)
        points[str(f)] = {"offered_per_s": lam, "served_per_s": st["throughput"],
                          "p50_ms": st["p50_ms"], "p90_ms": st["p90_ms"], "p99_ms": st["p99_ms"],
                          "mean_ms": st["mean_ms"], "failed": st["failed"]}
        print(f"load {f}: {points[str(f)]}", file=log, flush=True)
    srv.close()
    for s in state:
        s["p"].close()
    return {"jobs": len(js), "requests_per_point": nreq, "max_inflight": inflight,
            "hbm_budget_bytes": SERVE_HBM_BUDGET,
            "capacity_per_s": cap, "closed_loop_p50_ms": closed["p50_ms"],
            "closed_loop_p99_ms": closed["p99_ms"], "load_points": points, "setup_s": setup_s,
            "job_sizes": [j.n[0] for j in js]}


def measure_batch(steps: int, warmup: int, count: int, sweep: bool = True) -> dict:
    """Mixed batch: cubic n ~ U{48..160} (n mod r != 0), r ~ U{4, 8, 16},
    Ns ~ U{1..32} dipoles, 16 x 16 receivers; one solve = forward + J^T v of
    one instance.  The plain form runs the instances one after another on
    one stream; the batch form issues them through msfv_batch_* with the
    autotuned options.  With ``sweep`` each form is also timed at its best
    stream count."""
    import numpy as np
    import torch

    import paper_1707_07598_amd as msfv
    import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    insts = W.workload_batch(count)
    probs, ms, vs = [], [], []
    for k, inst in enumerate(insts):
        p = msfv.Problem(inst.n, inst.r, "reduced")
        p.set_sources(inst.sources)
        p.set_receivers(inst.receivers)
        m = torch.tensor(inst.m, dtype=torch.float64, device=dev)
        d_obs = p.forward(torch.tensor(inst.m_obs, dtype=torch.float64, device=dev)).clone()
        v = (p.forward(m) - d_obs).contiguous()
        probs.append(p)
        ms.append(m)
        vs.append(v)
        print(f"instance {k}: n={inst.n[0]} r={inst.r[0]} ns={inst.sources.count}", file=sys.stderr,
              flush=True)
    setup_s = time.perf_counter() - t0
    cells = sum(int(np.prod(i.n)) for i in insts)

    # plain form: one instance after another on one stream, no graphs
    for p, m, v in zip(probs, ms, vs):
        p.forward(m, sync=False)
        p.jtv(v, sync=False)
    torch.cuda.synchronize()
    reps = max(1, steps // 10)
    t0 = time.perf_counter()
    for _ in range(reps):
        for p, m, v in zip(probs, ms, vs):
            p.forward(m, sync=False)
            p.jtv(v, sync=False)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / reps
    for p in probs:
        p.sync()

    b = msfv.Batch(probs)

    def timed(nsteps):
        for _ in range(warmup):
            b.forward_jtv(ms, vs, sync=False)
        b.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            b.forward_jtv(ms, vs, sync=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.sync()
        return dt

    n = len(probs)
    # each form at its best stream count: the per-problem path (graphs) and
    # the shared launches of the local solves across problems
    forms = {}
    if sweep:
        for name, graphs, shared in (("streams+graphs", True, 0), ("shared launches, 1 pipeline", False, 1),
                                     ("shared launches, 2 pipelines", False, 2),
                                     ("shared launches, 4 pipelines", False, 4),
                                     ("shared launches, 8 pipelines", False, 8)):
            best = None
            for sc in (4, 8, 16):
                if sc < 2 * shared:
                    continue
                b.set_options(sc, graphs, shared)
                dt = timed(max(1, steps // 4))
                if best is None or dt < best[0]:
                    best = (dt, sc)
            forms[name] = {"streams": best[1], "solves_per_s": n * max(1, steps // 4) / best[0]}
    streams, graphs, shared = b.autotune(ms, vs)
    elapsed = timed(steps)
    value = n * steps / elapsed
    out = {
        "solves_per_s": value, "steps": steps, "ms_per_step": 1e3 * elapsed / steps,
        "workload": f"batch-{n}-mixed-n48..160-r4/8/16-ns1..32", "instances": n,
        "fine_cells": cells, "sources": int(sum(i.sources.count for i in insts)),
        "plain_solves_per_s": n / plain_s, "speedup_vs_plain": value / (n / plain_s),
        "autotuned": {"streams": streams, "graphs": graphs, "shared": shared}, "setup_s": setup_s,
    }
    if sweep:
        out["forms"] = forms
    b.close()
    for p in probs:
        p.close()
    return out


def run_batch(args) -> int:
    bt = measure_batch(args.steps, args.warmup, args.batch_count, sweep=True)
    out = {
        "metric": "MSFV forward+J^T v solves/s, batch of mixed instances (one solve = one instance)",
        "value": bt["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": bt["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": bt["workload"], "instances": bt["instances"], "fine_cells": bt["fine_cells"],
                   "sources": bt["sources"], "bc_mode": "reduced"},
        "plain_solves_per_s": bt["plain_solves_per_s"], "speedup_vs_plain": bt["speedup_vs_plain"],
        "forms": bt["forms"], "autotuned": bt["autotuned"], "setup_s": bt["setup_s"],
    }
    print(json.dumps(out), flush=True)
    return 0


def forward_only_64(steps: int = 10) -> dict:
    """The 64^3 workload (r = 8, 16 dipoles, 256 receivers, two box
    anomalies): forward only, one instance per call."""
    import torch

    import paper_1707_07598_amd as msfv
    import workloads as W

    inst = W.workload_64()
    dev = torch.device("cuda", 0)
    prob = msfv.Problem(inst.n, inst.r, "reduced")
    prob.set_sources(inst.sources)
    prob.set_receivers(inst.receivers)
    m = torch.tensor(inst.m, dtype=torch.float64, device=dev)
    for _ in range(2):
        prob.forward(m, sync=False)
    prob.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prob.forward(m, sync=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prob.sync()
    prob.close()
    return {"workload": "3d-64^3-r8-16dipoles-256rx-forward", "forward_solves_per_s": steps / dt,
            "ms_per_forward": 1e3 * dt / steps}


if __name__ == "__main__":
    sys.exit(main())
