"""Host-side checks of the serving workload generator (no GPU)."""
import numpy as np

from synth import water_cluster, water_box


def _pool():
    systems = {f"cl{k}": water_cluster(2 + k, 700 + k) for k in range(4)}
    for k in range(2):
        d = water_box(27, 9.5, 710 + k)
        d["params"] = dict(beta=0.45, cutoff=4.5, grid=24, order=5)
        systems[f"bx{k}"] = d
    return systems


def test_stream_is_seeded_poisson_with_md_steps():
    from paper_2201_00804_amd.serve import request_stream
    systems = _pool()
    a = request_stream(systems, 3000, rate=500.0, seed=4)
    b = request_stream(systems, 3000, rate=500.0, seed=4)
    assert [q.system for q in a] == [q.system for q in b]
    assert all(np.array_equal(x.pos, y.pos) for x, y in zip(a, b))
    t = np.array([q.arrival for q in a])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 1 / 500.0) < 0.1 / 500.0          # mean inter-arrival
    assert abs(np.std(gaps) / gaps.mean() - 1.0) < 0.1          # exponential: CV = 1
    share = np.mean([q.kind == "cluster" for q in a])
    assert abs(share - 0.7) < 0.03
    # each repeat moves every site by at most 0.01 A from the previous request
    last = {}
    for q in a:
        if q.system in last:
            step = np.abs(q.pos - last[q.system])
            assert step.max() <= 0.01 and step.max() > 0
        else:
            assert np.array_equal(q.pos, systems[q.system]["pos"])
        last[q.system] = q.pos
