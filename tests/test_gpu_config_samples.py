"""Sampled instances of the many-problem (batch) and serving workloads at
their full sizes, through the batch and serving entry points, against the
oracle (same bars as everywhere: t and D within 1e-10 per source and
element-wise, J^T v within 1e-8).

* batch instance 27: 133^3, r = 16 (dual blocks of 15^3 own cells: the
  generic workgroup-per-entity kernels), 14 dipoles -- t and D, and a
  central finite difference for J^T v (the oracle's J^T v at this size
  takes minutes; r = 16 gradients are compared with the oracle on the
  smaller parity grids);
* batch instance 60: 85^3, r = 8 (85 mod 8 = 5: truncated last coarse
  cells), 11 dipoles -- t, D and J^T v, J^T v also split by source;
* batch instance 29: 85^3, r = 4, 27 dipoles, 22^3 = 10648 coarse vertices
  (above 8192: the multi-launch coarse solver) -- t and D against the
  oracle's forward on a block-parallel oracle basis, and a central finite
  difference of the misfit for J^T v;
* serving job 11: 156^3, r = 8, its first request of 27 dipoles served
  among requests of two other jobs -- D per source against the oracle
  (block-parallel basis), and D and g bit for bit equal to the same
  problem's eager call.

The batch runs the three instances in one msfv_batch_forward_jtv call with
shared launches of the local solves across the three problems.
"""
import numpy as np
import pytest

import _parity as PT
import workloads as W
from _oracle_parallel import parallel_basis
from oracle import Geometry
from oracle import reduced as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch_run():
    import torch
    import paper_1707_07598_amd as msfv
    insts = W.workload_batch(64)
    picks = [27, 60, 29]
    probs, ms, vs, Vs = [], [], [], []
    for k in picks:
        inst = insts[k]
        p = msfv.Problem(inst.n, inst.r, "reduced")
        p.set_sources(inst.sources)
        p.set_receivers(inst.receivers)
        probs.append(p)
        ms.append(torch.tensor(inst.m, dtype=torch.float64, device="cuda"))
        V = np.random.default_rng(500 + k).standard_normal((inst.receivers.count, inst.sources.count))
        Vs.append(V)
        vs.append(torch.tensor(V.T.copy(), device="cuda"))
    b = msfv.Batch(probs)
    b.autotune(ms, vs)
    # the results compared below come from the shared launches of the local
    # solves (one launch per stage and kernel class over all three problems)
    b.set_options(8, False, 1)
    D, g = b.forward_jtv(ms, vs)
    out = {"insts": [insts[k] for k in picks], "probs": probs, "ms": ms, "Vs": Vs,
           "D": [d.cpu().numpy() for d in D], "g": [x.cpu().numpy() for x in g],
           "t": [p.coarse()[1] for p in probs], "batch": b}
    yield out
    b.close()
    for p in probs:
        p.close()


def _fd_check(batch_run, idx, seed):
    """J^T v of the batch against a central difference of <v, D(m)>."""
    import torch
    prob, m = batch_run["probs"][idx], batch_run["ms"][idx]
    V = torch.tensor(batch_run["Vs"][idx].T.copy(), device="cuda")
    e = torch.tensor(np.random.default_rng(seed).standard_normal(m.numel()), device="cuda")
    h = 1e-5
    fp = float((prob.forward(m + h * e) * V).sum())
    fm = float((prob.forward(m - h * e) * V).sum())
    fd = (fp - fm) / (2 * h)
    dd = float((torch.tensor(batch_run["g"][idx], device="cuda") * e).sum())
    assert abs(fd - dd) <= 1e-5 * abs(dd)


def test_batch_r16_instance_against_oracle(batch_run):
    inst = batch_run["insts"][0]
    geo = Geometry(inst.n, inst.r)
    st = R.forward(geo, inst.m, inst.sources, inst.receivers, basis=parallel_basis(geo, inst.m))
    PT.rows(batch_run["t"][0], st.t.T, 1e-10, "t")
    PT.rows(batch_run["D"][0], st.D.T, 1e-10, "D")
    _fd_check(batch_run, 0, 76)


def test_batch_r8_instance_against_oracle(batch_run):
    inst = batch_run["insts"][1]
    geo = Geometry(inst.n, inst.r)
    st = R.forward(geo, inst.m, inst.sources, inst.receivers)
    PT.rows(batch_run["t"][1], st.t.T, 1e-10, "t")
    PT.rows(batch_run["D"][1], st.D.T, 1e-10, "D")
    V = batch_run["Vs"][1]
    PT.vector(batch_run["g"][1], R.jtv(st, V), 1e-8, "g")
    prob = batch_run["probs"][1]
    prob.forward(batch_run["ms"][1])
    PT.gradient_per_source(prob, st, V, 1e-8, sources=(0, V.shape[1] - 1))


def test_batch_large_coarse_instance_against_oracle(batch_run):
    inst = batch_run["insts"][2]
    geo = Geometry(inst.n, inst.r)
    assert geo.ncoarse > 8192
    st = R.forward(geo, inst.m, inst.sources, inst.receivers, basis=parallel_basis(geo, inst.m))
    PT.rows(batch_run["t"][2], st.t.T, 1e-10, "t")
    PT.rows(batch_run["D"][2], st.D.T, 1e-10, "D")
    _fd_check(batch_run, 2, 77)


def test_served_request_on_a_large_job_against_oracle():
    import torch
    import paper_1707_07598_amd as msfv
    jobs = W.workload_serving(16)
    picks = [11, 0, 12]           # 156^3 and two small jobs served alongside
    assert jobs[11].n[0] >= 150
    srv = msfv.Server(max_inflight=4)
    state = []
    for k in picks:
        job = jobs[k]
        p = msfv.Problem(job.n, job.r, "reduced", stream=torch.cuda.Stream())
        p.set_receivers(job.receivers)
        srv.add_job(p, max_sources=64)
        src = job.sources(0)
        m = torch.tensor(job.m0, dtype=torch.float64, device="cuda")
        v = torch.tensor(np.random.default_rng(600 + k).standard_normal((src.count, job.receivers.count)),
                         device="cuda")
        state.append((job, p, src, m, v))
    reqs = []
    for i, (job, p, src, m, v) in enumerate(state):
        d = torch.empty((src.count, job.receivers.count), dtype=torch.float64, device="cuda")
        g = torch.empty(m.numel(), dtype=torch.float64, device="cuda")
        reqs.append((srv.submit(i, src, m, v, d, g), d, g))
    for rid, _, _ in reqs:
        srv.wait(rid)
    job, p, src, m, v = state[0]
    d, g = reqs[0][1], reqs[0][2]
    q = msfv.Problem(job.n, job.r, "reduced")
    q.set_receivers(job.receivers)
    q.set_sources(src)
    assert torch.equal(q.forward(m), d) and torch.equal(q.jtv(v), g)
    q.close()
    geo = Geometry(job.n, job.r)
    st = R.forward(geo, job.m0, src, job.receivers, basis=parallel_basis(geo, job.m0))
    PT.rows(d.cpu().numpy(), st.D.T, 1e-10, "D of the served request")
    srv.close()
    for s in state:
        s[1].close()
