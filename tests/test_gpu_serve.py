"""Serving runtime (msfv_server_*): interleaved requests of several jobs,
each with its own source set, give bit for bit what the same problem
computes eagerly (and the oracle, for one of them); statistics count every
request; bad arguments are rejected.  Admission by memory budget: with a
budget that fits one request at a time the committed bytes never exceed it
and the requests run one after another; a request that can never fit is
rejected; a job whose resident state does not fit is refused.  Without
that limit two jobs' requests overlap on the device.  A request is ordered
after the caller's stream; several threads may wait for one request."""
import time

import numpy as np
import pytest

import _parity as PT
import workloads as W
from oracle import Geometry
from oracle import reduced as R

pytestmark = pytest.mark.gpu

JOBS = [((13, 11, 9), (4, 4, 4)), ((24, 22, 20), (8, 8, 8)), ((32, 32), (4, 4))]
NR = 6


def test_server_requests_match_eager_and_oracle():
    import torch
    import paper_1707_07598_amd as msfv
    srv = msfv.Server(max_inflight=2)
    probs, refs, ms = [], [], []
    for k, (n, r) in enumerate(JOBS):
        inst = W.small_instance(n, r, seed=60 + k, ns=1, nr=NR)
        p = msfv.Problem(n, r, "reduced", stream=torch.cuda.Stream())
        p.set_receivers(inst.receivers)
        q = msfv.Problem(n, r, "reduced")
        q.set_receivers(inst.receivers)
        assert srv.add_job(p) == k
        probs.append(p)
        refs.append((q, inst))
        ms.append(torch.tensor(inst.m, dtype=torch.float64, device="cuda"))
    rng = np.random.default_rng(7)
    reqs = []
    for i in range(4):
        for k, (n, r) in enumerate(JOBS):
            ns = int(rng.integers(1, 6))
            src = W.surface_dipoles(n, ns)
            v = torch.tensor(rng.standard_normal((ns, NR)), device="cuda")
            d = torch.empty((ns, NR), dtype=torch.float64, device="cuda")
            g = torch.empty(int(np.prod(n)), dtype=torch.float64, device="cuda")
            reqs.append((srv.submit(k, src, ms[k], v, d, g), k, src, v, d, g))
    for rid, *_ in reqs:
        assert srv.wait(rid) > 0.0
    st = srv.stats(reset=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert 0.0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    for idx, (rid, k, src, v, d, g) in enumerate(reqs):
        q, inst = refs[k]
        q.set_sources(src)
        D = q.forward(ms[k])
        gg = q.jtv(v)
        assert torch.equal(D, d) and torch.equal(gg, g), idx
        if idx == 1:
            geo = Geometry(inst.n, inst.r)
            ref = R.forward(geo, inst.m, src, inst.receivers)
            PT.rows(d.cpu().numpy(), ref.D.T, 1e-10, "D")
            PT.vector(g.cpu().numpy(), R.jtv(ref, v.cpu().numpy().T), 1e-8, "g")
    srv.close()
    for p in probs:
        p.close()
    for q, _ in refs:
        q.close()


def test_server_errors():
    import torch
    import paper_1707_07598_amd as msfv
    from paper_1707_07598_amd import _lib
    srv = msfv.Server(max_inflight=1)
    inst = W.small_instance((13, 11, 9), (4, 4, 4), seed=70, ns=1, nr=3)
    p = msfv.Problem(inst.n, inst.r)
    with pytest.raises(msfv.MsfvError) as e:
        srv.add_job(p)  # no receivers yet
    assert e.value.status == _lib.MSFV_ESTATE
    p.set_receivers(inst.receivers)
    job = srv.add_job(p)
    with pytest.raises(msfv.MsfvError) as e:
        srv.add_job(p)
    assert e.value.status == _lib.MSFV_EINVAL
    m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
    v = torch.ones((1, 3), dtype=torch.float64, device="cuda")
    d = torch.empty((1, 3), dtype=torch.float64, device="cuda")
    g = torch.empty(m.numel(), dtype=torch.float64, device="cuda")
    with pytest.raises(msfv.MsfvError) as e:
        srv.submit(job + 1, inst.sources, m, v, d, g)
    assert e.value.status == _lib.MSFV_EINVAL
    bad = m.clone()
    bad[3] = float("nan")
    rid = srv.submit(job, inst.sources, bad, v, d, g)
    with pytest.raises(msfv.MsfvError) as e:
        srv.wait(rid)
    assert e.value.status == _lib.MSFV_ENONFINITE
    rid = srv.submit(job, inst.sources, m, v, d, g)  # the job recovers
    srv.wait(rid)
    srv.close()
    p.close()


def _jobs(srv, specs, seed0):
    import torch
    import paper_1707_07598_amd as msfv
    out = []
    for k, (n, r, ns) in enumerate(specs):
        inst = W.small_instance(n, r, seed=seed0 + k, ns=ns, nr=NR)
        p = msfv.Problem(n, r, "reduced", stream=torch.cuda.Stream())
        p.set_receivers(inst.receivers)
        job = srv.add_job(p, max_sources=ns) if srv is not None else None
        m = torch.tensor(inst.m, dtype=torch.float64, device="cuda")
        v = torch.tensor(np.random.default_rng(seed0 + 50 + k).standard_normal((ns, NR)), device="cuda")
        out.append({"p": p, "inst": inst, "job": job, "m": m, "v": v, "ns": ns})
    return out


def _eager(j):
    import paper_1707_07598_amd as msfv
    q = msfv.Problem(j["inst"].n, j["inst"].r, "reduced")
    q.set_receivers(j["inst"].receivers)
    q.set_sources(j["inst"].sources)
    D = q.forward(j["m"]).clone()
    g = q.jtv(j["v"]).clone()
    q.close()
    return D, g


def _submit(srv, j):
    import torch
    d = torch.empty((j["ns"], NR), dtype=torch.float64, device="cuda")
    g = torch.empty(j["m"].numel(), dtype=torch.float64, device="cuda")
    return srv.submit(j["job"], j["inst"].sources, j["m"], j["v"], d, g), d, g


def test_server_budget_admits_one_at_a_time():
    import torch
    import paper_1707_07598_amd as msfv
    # jobs of about the same size, so that no two requests fit together
    specs = [((24, 22, 20), (8, 8, 8), 4), ((22, 24, 20), (4, 4, 4), 3), ((20, 22, 24), (5, 5, 5), 2)]
    # size the budget from the jobs' own figures: all resident state plus
    # 1.5 times the largest request
    probe = msfv.Server(max_inflight=8)
    js = _jobs(probe, specs, 90)
    res = sum(probe.request_bytes(j["job"], j["ns"])[0] for j in js)
    req = max(probe.request_bytes(j["job"], j["ns"])[1] for j in js)
    probe.close()
    for j in js:
        j["p"].close()
    # requests hold at least m and g (16 bytes a cell): no two fit together
    smallest = sorted(16 * int(np.prod(n)) for n, _, _ in specs)
    budget = res + 1.5 * req
    assert budget < res + smallest[0] + smallest[1]
    srv = msfv.Server(max_inflight=8, hbm_budget=budget)
    js = _jobs(srv, specs, 90)
    refs = [_eager(j) for j in js]
    subs = []
    for rep in range(3):
        for k, j in enumerate(js):
            subs.append((k,) + _submit(srv, j))
    for k, rid, d, g in subs:
        srv.wait(rid)
        assert torch.equal(d, refs[k][0]) and torch.equal(g, refs[k][1]), (k, rid)
    st = srv.stats()
    assert st["completed"] == len(subs) and st["failed"] == 0 and st["rejected"] == 0
    assert st["budget_bytes"] == budget
    assert st["resident_bytes"] + req <= st["peak_committed_bytes"] <= st["budget_bytes"]
    # one request at a time: the device intervals do not overlap
    iv = sorted(srv.device_times[rid] for _, rid, _, _ in subs)
    assert all(b[0] >= a[1] for a, b in zip(iv, iv[1:]))
    srv.close()
    for j in js:
        j["p"].close()


def test_server_rejects_what_cannot_fit():
    import torch
    import paper_1707_07598_amd as msfv
    from paper_1707_07598_amd import _lib
    specs = [((24, 22, 20), (8, 8, 8), 4)]
    probe = msfv.Server(max_inflight=2)
    js = _jobs(probe, specs, 95)
    res, req = probe.request_bytes(js[0]["job"], 4)
    probe.close()
    js[0]["p"].close()
    # the job fits, a request never does: rejected at submission
    srv = msfv.Server(max_inflight=2, hbm_budget=res + req // 2)
    js = _jobs(srv, specs, 95)
    with pytest.raises(msfv.MsfvError) as e:
        _submit(srv, js[0])
    assert e.value.status == _lib.MSFV_ENOMEM
    assert srv.stats()["rejected"] == 1
    # more sources than the job was registered for
    with pytest.raises(msfv.MsfvError) as e:
        srv.submit(js[0]["job"], W.surface_dipoles(js[0]["inst"].n, 5), js[0]["m"],
                   torch.zeros((5, NR), dtype=torch.float64, device="cuda"),
                   torch.zeros((5, NR), dtype=torch.float64, device="cuda"), torch.empty_like(js[0]["m"]))
    assert e.value.status == _lib.MSFV_EINVAL
    srv.close()
    js[0]["p"].close()
    # a job whose resident state does not fit is not added
    tiny = msfv.Server(max_inflight=1, hbm_budget=res // 4)
    p = msfv.Problem((24, 22, 20), (8, 8, 8), "reduced")
    p.set_receivers(W.surface_pole_receivers((24, 22, 20), NR))
    with pytest.raises(msfv.MsfvError) as e:
        tiny.add_job(p, max_sources=4)
    assert e.value.status == _lib.MSFV_ENOMEM
    tiny.close()
    p.close()


def test_server_requests_overlap_on_the_device():
    """Two jobs of a few milliseconds of device work each, submitted
    together with room for both: their device intervals overlap, and each
    result equals the job's eager result."""
    import torch
    import paper_1707_07598_amd as msfv
    specs = [((48, 48, 40), (8, 8, 8), 16), ((48, 44, 40), (8, 8, 8), 16)]
    srv = msfv.Server(max_inflight=4)
    js = _jobs(srv, specs, 97)
    refs = [_eager(j) for j in js]
    for j in js:  # first request of each job builds its electrode tables
        srv.wait(_submit(srv, j)[0])
    subs = []
    for rep in range(4):
        for k, j in enumerate(js):
            subs.append((k,) + _submit(srv, j))
    for k, rid, d, g in subs:
        srv.wait(rid)
        assert torch.equal(d, refs[k][0]) and torch.equal(g, refs[k][1]), (k, rid)
    t = {k: [srv.device_times[rid] for kk, rid, _, _ in subs if kk == k] for k in (0, 1)}
    overlaps = sum(1 for a in t[0] for b in t[1] if a[0] < b[1] and b[0] < a[1])
    assert overlaps > 0, t
    srv.close()
    for j in js:
        j["p"].close()


def test_server_orders_after_the_callers_stream_and_shared_waits():
    """m is rewritten on the caller's stream behind a long kernel just before
    submission: the request sees the new m.  Two threads wait for the same
    request while a third drains."""
    import threading
    import torch
    import paper_1707_07598_amd as msfv
    specs = [((24, 22, 20), (8, 8, 8), 3)]
    srv = msfv.Server(max_inflight=2)
    js = _jobs(srv, specs, 99)
    j = js[0]
    m_new = j["m"] + 0.3 * torch.sin(torch.arange(j["m"].numel(), dtype=torch.float64, device="cuda"))
    jn = dict(j, m=m_new)
    ref = _eager(jn)
    srv.wait(_submit(srv, j)[0])
    dev_m = j["m"].clone()
    x = torch.rand((3072, 3072), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    for _ in range(6):  # milliseconds of work on the caller's stream before m changes
        x = (x @ x) / 3072.0
    dev_m.copy_(m_new)
    rid, d, g = _submit(srv, dict(j, m=dev_m))
    out = []
    ths = [threading.Thread(target=lambda: out.append(srv.wait(rid))) for _ in range(2)]
    for t in ths:
        t.start()
    time.sleep(0.001)
    ths.append(threading.Thread(target=srv.drain))
    ths[-1].start()
    for t in ths:
        t.join()
    assert len(out) == 2 and all(x > 0.0 for x in out)
    assert torch.equal(d, ref[0]) and torch.equal(g, ref[1])
    srv.close()
    j["p"].close()
