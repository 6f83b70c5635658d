"""Many problems per call (msfv_batch_*): every instance of a mixed batch
matches the oracle and, bit for bit, its own eager forward + J^T v; graph
replays with the program's eager work and synchronisations in between give
the eager result every time, also after the inputs change in place; option
changes and autotuning do not change results."""
import numpy as np
import pytest

import workloads as W
from oracle import Geometry
from oracle import reduced as R

pytestmark = pytest.mark.gpu

# (n, r, sources, coarse solver); the multi-launch coarse solver polls from
# the host, so with several streams the batch drives those problems from
# worker threads
SHAPES = [((13, 11, 9), (4, 4, 4), 3, "twolevel"),
          ((36, 20, 19), (16, 8, 6), 2, "twolevel"),    # r = 16 along x: the generic local kernels
          ((32, 32), (4, 4), 2, "multi"),               # 2-D
          ((17, 9, 12), (8, 3, 4), 5, "multi"),
          ((24, 22, 20), (8, 8, 8), 1, "twolevel")]


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def batch_setup():
    import torch
    import paper_1707_07598_amd as msfv
    insts, probs, ms, vs = [], [], [], []
    for k, (n, r, ns, pc) in enumerate(SHAPES):
        inst = W.small_instance(n, r, seed=40 + k, ns=ns, nr=6)
        p = msfv.Problem(n, r, "reduced", coarse_precond=pc)
        p.set_sources(inst.sources)
        p.set_receivers(inst.receivers)
        insts.append(inst)
        probs.append(p)
        ms.append(torch.tensor(inst.m, dtype=torch.float64, device="cuda"))
        V = np.random.default_rng(100 + k).standard_normal((ns, 6))
        vs.append(torch.tensor(V, dtype=torch.float64, device="cuda"))
    # eager reference on each problem's own stream
    eager = []
    for p, m, v in zip(probs, ms, vs):
        D = p.forward(m).clone()
        g = p.jtv(v).clone()
        eager.append((D, g))
    b = msfv.Batch(probs)
    yield insts, probs, ms, vs, eager, b
    b.close()
    for p in probs:
        p.close()


def test_batch_matches_oracle_and_eager(batch_setup):
    import torch
    insts, probs, ms, vs, eager, b = batch_setup
    D, g = b.forward_jtv(ms, vs)
    for k, inst in enumerate(insts):
        geo = Geometry(inst.n, inst.r)
        st = R.forward(geo, inst.m, inst.sources, inst.receivers)
        g_ref = R.jtv(st, vs[k].cpu().numpy().T)
        assert _rel(D[k].cpu().numpy(), st.D.T) < 1e-10, k
        assert _rel(g[k].cpu().numpy(), g_ref) < 1e-8, k
        assert torch.equal(D[k], eager[k][0]) and torch.equal(g[k], eager[k][1]), k


def test_graph_replays_and_in_place_updates(batch_setup):
    import torch
    insts, probs, ms, vs, eager, b = batch_setup
    b.set_options(4, True)
    for rep in range(3):
        D, g = b.forward_jtv(ms, vs)
        for k in range(len(probs)):
            assert torch.equal(D[k], eager[k][0]) and torch.equal(g[k], eager[k][1]), (rep, k)
        # eager work and a synchronisation between replays
        probs[0].forward(ms[0])
        torch.cuda.synchronize()
    # change the inputs in place: the replayed graphs read the new values
    for m in ms:
        m.mul_(0.5)
    ref = []
    for p, m, v in zip(probs, ms, vs):
        ref.append((p.forward(m).clone(), p.jtv(v).clone()))
    for rep in range(2):
        D, g = b.forward_jtv(ms, vs)
        for k in range(len(probs)):
            assert torch.equal(D[k], ref[k][0]) and torch.equal(g[k], ref[k][1]), (rep, k)
    for m in ms:
        m.mul_(2.0)


def test_options_autotune_and_new_buffers(batch_setup):
    import torch
    insts, probs, ms, vs, eager, b = batch_setup
    for streams, graphs in [(1, False), (3, False), (16, True), (1, True)]:
        b.set_options(streams, graphs)
        assert b.options() == (streams, graphs)
        D, g = b.forward_jtv(ms, vs)
        for k in range(len(probs)):
            assert torch.equal(D[k], eager[k][0]) and torch.equal(g[k], eager[k][1]), (streams, graphs, k)
    s, gr = b.autotune(ms, vs)
    assert 1 <= s <= 16
    # new input buffers: graphs are captured again
    ms2 = [m.clone() for m in ms]
    D, g = b.forward_jtv(ms2, vs)
    for k in range(len(probs)):
        assert torch.equal(D[k], eager[k][0]) and torch.equal(g[k], eager[k][1]), k


def test_batch_errors():
    import paper_1707_07598_amd as msfv
    from paper_1707_07598_amd import _lib
    p = msfv.Problem((13, 11, 9), (4, 4, 4))
    with pytest.raises(msfv.MsfvError) as e:
        msfv.Batch([p, p])
    assert e.value.status == _lib.MSFV_EINVAL
    p.close()


def test_batch_error_from_a_polled_problem():
    """A failing problem on the multi-launch coarse solver (driven from a
    worker thread when there are several streams) surfaces at the batch sync;
    the other problems' results are still those of their eager calls."""
    import torch
    import paper_1707_07598_amd as msfv
    from paper_1707_07598_amd import _lib
    specs = [((13, 11, 9), (4, 4, 4), 2, "twolevel", 1000),
             ((32, 32), (4, 4), 2, "multi", 1),            # local solves capped: fails
             ((17, 9, 12), (8, 3, 4), 3, "multi", 1000)]
    probs, ms, vs = [], [], []
    for k, (n, r, ns, pc, maxit) in enumerate(specs):
        inst = W.small_instance(n, r, seed=60 + k, ns=ns, nr=4)
        p = msfv.Problem(n, r, "reduced", coarse_precond=pc, local_maxit=maxit)
        p.set_sources(inst.sources)
        p.set_receivers(inst.receivers)
        probs.append(p)
        ms.append(torch.tensor(inst.m, dtype=torch.float64, device="cuda"))
        vs.append(torch.tensor(np.random.default_rng(70 + k).standard_normal((ns, 4)), dtype=torch.float64,
                               device="cuda"))
    eager = {}
    for k in (0, 2):
        eager[k] = (probs[k].forward(ms[k]).clone(), probs[k].jtv(vs[k]).clone())
    b = msfv.Batch(probs)
    b.set_options(4, False)
    D, g = b.forward_jtv(ms, vs, sync=False)
    with pytest.raises(msfv.MsfvError) as e:
        b.sync()
    assert e.value.status == _lib.MSFV_ENOCONV
    for k in (0, 2):
        assert torch.equal(D[k], eager[k][0]) and torch.equal(g[k], eager[k][1]), k
    b.close()
    for p in probs:
        p.close()
