"""Recorded call sequences (mcd_graph_begin / mcd_graph_end): the parts of a
time step around the PPE solve run as one HIP graph each.  Every replay is
checked against the same step run call by call (bit for bit), with the
eager work of the solve between replays; calls that wait for the device are
refused while a graph is recorded and leave nothing half-run."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2404_17542_amd import configs
from gpu_helpers import bits_equal, np_

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_17542_amd import mcd
    mcd.load()
    return mcd


@pytest.mark.parametrize("which", ["cylinder", "taylor_green", "flapping"])
def test_graph_steps_equal_direct_calls(M, which):
    from paper_2404_17542_amd.sim import GpuSim
    case = {"cylinder": lambda: configs.c2_oscillating_cylinder(n=128, steps=6),
            "taylor_green": lambda: configs.c1_taylor_green(n=64, steps=6),
            "flapping": lambda: configs.c6_flapping_ellipse(n=256, steps=6)}[which]()
    eager = GpuSim(case, update_info=False)
    graph = GpuSim(case, update_info=False, graph=True)
    for k in range(6):
        re_ = eager.step()
        rg = graph.step()
        torch.cuda.synchronize()
        assert rg["iters"] == re_["iters"] and rg["converged"], k
        for name in ("pos", "role", "normal", "u", "P", "fP"):
            assert bits_equal(np_(getattr(graph, name)), np_(getattr(eager, name))), (k, name)
    st = [graph.ctx.graph_stats(q) for q in range(4)]
    print(which, st, "fallbacks", graph.graph_fallbacks)
    # preparations in slots 0 and 2 (six steps and the seventh recorded ahead),
    # projections in 1 and 3; each slot instantiated once, then updated in
    # place; no recording may fall back to direct calls
    assert graph.graph_fallbacks == 0
    assert all(q["instantiated"] == 1 for q in st)
    assert sum(st[q]["instantiated"] + st[q]["updated"] for q in (0, 2)) == 7
    assert sum(st[q]["instantiated"] + st[q]["updated"] for q in (1, 3)) == 6


def test_destroy_during_a_recording_is_deferred(M):
    """A context released while another context records is freed only after
    that recording ends (freeing memory or waiting for a stream in the middle
    of it could invalidate it); the recording then replays correctly."""
    from paper_2404_17542_amd.sim import GpuSim
    case = configs.c2_oscillating_cylinder(n=64, steps=3)
    victim = M.Context.from_case(case)
    sim = GpuSim(case, update_info=False, graph=True)
    ref = GpuSim(case, update_info=False)
    sim.step()
    ref.step()
    ctx = sim.ctx
    ctx.graph_begin(2)
    pre = sim._prepare()
    victim.close()                                 # released while slot 2 records
    assert M.load().mcd_pending_destroys() == 1
    ctx.graph_end(2, launch=True)
    assert M.load().mcd_pending_destroys() == 0
    pset, bodies_new, upd = pre
    info = sim.solve(pset, sim.initial_guess(pset, sim.guess))
    sim.finish(pset, bodies_new, info, upd)
    ref.step()
    torch.cuda.synchronize()
    for name in ("pos", "role", "u", "P"):
        assert bits_equal(np_(getattr(sim, name)), np_(getattr(ref, name))), name


def test_refused_calls_leave_nothing_half_run(M):
    from paper_2404_17542_amd.sim import GpuSim
    case = configs.c2_oscillating_cylinder(n=64, steps=2)
    sim = GpuSim(case, update_info=False)
    ctx = sim.ctx
    u0 = np_(sim.u).copy()
    ctx.graph_begin(2)
    with pytest.raises(M.McdError):
        ctx.graph_begin(2)                      # one capture at a time
    with pytest.raises(M.McdError):
        ctx.graph_launch(3)                     # refused while recording (and slot 3 holds nothing)
    ctx.project(0, sim.P, sim.fP, sim.ustar, case.dt, sim.role, sim.bodies, sim.u, pos=sim.pos)
    with pytest.raises(M.McdError) as ei:
        ctx.sync()                              # waits for the device: refused
    assert ei.value.status == 1
    with pytest.raises(M.McdError) as ei:
        ctx.graph_end(2)                        # the recorded sequence is incomplete: nothing runs
    assert ei.value.status == 1
    torch.cuda.synchronize()
    assert bits_equal(np_(sim.u), u0)
    with pytest.raises(M.McdError):
        ctx.graph_end(2)                        # no capture open
    with pytest.raises(M.McdError):
        ctx.graph_launch(2)                     # the failed recording left no graph
    with pytest.raises(M.McdError):
        ctx.graph_begin(M.MAX_GRAPHS if hasattr(M, "MAX_GRAPHS") else 4)
    r = sim.step()                              # the context works as before
    assert r["converged"]
    assert ctx.graph_stats(2) == {"instantiated": 0, "updated": 0}
