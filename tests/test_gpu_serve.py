"""Serving layer on the GPU: an open-loop stream of cluster and box
requests, checked against standalone evaluations; admission control."""
import numpy as np
import pytest
import torch

from synth import water_cluster, water_box
from synth.water import CONFIGS
from tests.gpu_util import say, gpu_params, engine_for, rms_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _small_pool():
    c = CONFIGS["box216"]
    systems = {f"cl{k}": water_cluster(nw, 300 + k) for k, nw in enumerate((3, 12, 30, 64))}
    for k in range(2):
        d = water_box(c["n_waters"], c["box"], 310 + k)
        d["params"] = dict(beta=c["beta"], cutoff=c["cutoff"], grid=c["grid"], order=5)
        systems[f"box216_{k}"] = d
    return systems


def _fresh(sysd, pos, tol, precision="fp64"):
    """Cold standalone evaluation of one request's system at its positions."""
    d = dict(sysd, pos=pos)
    if d.get("box") is None:
        kw = dict(tol=tol)
    else:
        p = d["params"]
        kw = dict(beta=p["beta"], cutoff=p["cutoff"], grid=p["grid"], tol=tol)
    eng = engine_for(d, gpu_params(d, max_iter=400, precision=precision, **kw))
    eng.solve()
    ep, ee, F = eng.energy_forces()
    eng.close()
    return ep, ee, F.cpu().numpy()


def test_stream_results_match_standalone():
    from paper_2201_00804_amd.serve import Server, request_stream, summarize
    systems = _small_pool()
    tol = 1e-10
    srv = Server(systems, precision="fp64", tol=tol)
    reqs = request_stream(systems, 160, rate=400.0, seed=3)
    wall = srv.run(reqs)
    summ = summarize(reqs, wall, srv)
    say(f"[serve] {summ}")
    assert summ["requests"] == 160 and summ["failed"] == 0 and not srv.errors
    assert summ["cluster"]["warm_share"] > 0.5 and summ["box"]["warm_share"] > 0.5
    rng = np.random.default_rng(0)
    for q in [reqs[k] for k in sorted(rng.choice(len(reqs), 12, replace=False))]:
        ep, ee, F = _fresh(systems[q.system], q.pos, tol)
        assert q.e_pol == pytest.approx(ep, rel=1e-8, abs=1e-10)
        assert q.e_elec == pytest.approx(ee, rel=1e-10, abs=1e-10)
        assert rms_rel(q.forces, F) < 1e-7
    srv.close()


@pytest.mark.parametrize("precond", ["diag", "molblock"])
def test_stream_results_match_standalone_mixed(precond):
    """The served precision (FP32-mixed), under a burst that keeps several
    box requests in flight at once: every sampled result equals a cold
    standalone mixed evaluation at the same positions within the mixed
    path's bounds (E_pol 1e-5 relative, E_elec 1e-5 relative, forces 1e-4
    relative RMS), whether it ran alone or beside other boxes and clusters,
    with either preconditioner in the box contexts (the standalone
    evaluations use the diagonal one: both converge to the tolerance)."""
    from paper_2201_00804_amd.serve import Server, request_stream, summarize
    systems = _small_pool()
    c = CONFIGS["box216"]
    for k in range(2, 4):
        d = water_box(c["n_waters"], c["box"], 310 + k)
        d["params"] = dict(beta=c["beta"], cutoff=c["cutoff"], grid=c["grid"], order=5)
        systems[f"box216_{k}"] = d
    tol = 1e-8
    srv = Server(systems, precision="mixed", tol=tol, box_slots=3, precond=precond)
    reqs = request_stream(systems, 200, rate=20000.0, seed=5)
    wall = srv.run(reqs)
    summ = summarize(reqs, wall, srv)
    say(f"[serve mixed] {summ}")
    assert summ["requests"] == 200 and summ["failed"] == 0 and not srv.errors
    assert summ["max_boxes_in_flight"] >= 2 and summ["box_overlap_share"] > 0.3
    rng = np.random.default_rng(1)
    boxes = [q for q in reqs if q.kind == "box"]
    clusters = [q for q in reqs if q.kind == "cluster"]
    picks = [boxes[k] for k in rng.choice(len(boxes), 6, replace=False)] + \
            [clusters[k] for k in rng.choice(len(clusters), 6, replace=False)]
    for q in picks:
        ep, ee, F = _fresh(systems[q.system], q.pos, tol, precision="mixed")
        say(f"  {q.kind} {q.system}: E_pol {q.e_pol:.8f} vs {ep:.8f}, E_elec {q.e_elec:.8f} vs "
            f"{ee:.8f}, F rms rel {rms_rel(q.forces, F):.2e}, warm {q.warm}")
        assert q.e_pol == pytest.approx(ep, rel=1e-5)
        assert q.e_elec == pytest.approx(ee, rel=1e-5)
        assert rms_rel(q.forces, F) < 1e-4
    srv.close()


def test_admission_evicts_and_rejects():
    from paper_2201_00804_amd import engine
    from paper_2201_00804_amd.serve import Server, Request
    systems = _small_pool()
    d = systems["box216_0"]
    fp = engine.footprint_bytes(len(d["pos"]), 648, d["box"],
                                engine.default_params(beta=0.45, cutoff=8.0, grid=20,
                                                      precision="mixed"))
    # one box slot: requests run in order, each evicting the other system
    srv = Server(systems, precision="mixed", hbm_budget=int(1.5 * fp), box_slots=1)
    reqs = [Request(k, f"box216_{k % 2}", "box", systems[f"box216_{k % 2}"]["pos"].copy(),
                    0.001 * k) for k in range(4)]
    srv.run(reqs)
    assert all(q.status == 0 for q in reqs)
    assert srv.evictions == 3 and len(srv.resident) == 1
    assert not any(q.warm for q in reqs)       # each came back cold after eviction
    srv.close()
    # three slots: a system that does not fit beside one in flight waits for
    # it (no eviction of a context in use); every request is still served
    srv = Server(systems, precision="mixed", hbm_budget=int(1.5 * fp), box_slots=3)
    reqs = [Request(k, f"box216_{k % 2}", "box", systems[f"box216_{k % 2}"]["pos"].copy(),
                    0.001 * k) for k in range(6)]
    srv.run(reqs)
    assert all(q.status == 0 for q in reqs) and not srv.errors
    assert srv.evictions >= 1 and len(srv.resident) == 1
    assert srv.resident_bytes <= srv.budget
    srv.close()
    tiny = Server(systems, precision="mixed", hbm_budget=fp // 2)
    q = Request(0, "box216_0", "box", d["pos"].copy(), 0.0)
    tiny.run([q])
    assert q.status == "rejected" and tiny.rejections == 1
    tiny.close()
