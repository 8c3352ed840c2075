"""Beeman dynamics through the C-ABI (sibfa_md_init / sibfa_md_run) against
the oracle's trajectory (oracle/md.py, pinned in tests/test_oracle_md.py):
positions, velocities and per-step energies after a few steps, with and
without local frames; and on the 216-water box the paper's MD system,
energy conservation and the predictor's saving of iterations.

Bars: positions 1e-9 A, velocities 1e-8 of the largest, energies 1e-8
relative (FP64 both sides; the GPU warm-starts each solve, the oracle solves
from the cold guess, both to 1e-11 D)."""
import numpy as np
import pytest
import torch

from oracle import md as omd
from oracle.model import System
from synth import water_cluster, water_box, water_md, water_frames, config_system
from tests.gpu_util import say, oracle_params, gpu_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _t(a, dt=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dt, device="cuda").contiguous()


def _md_engine(d, kw, m, precision="fp64", frames=None, predictor=0):
    from paper_2201_00804_amd import Engine
    eng = Engine(0)
    eng.load(d, gpu_params(d, precision=precision, **kw))
    if frames is not None:
        eng.set_local_frames(_t(frames, torch.int32), _t(d["dip"]), _t(d["quad"]), _t(d["alpha"]))
    if predictor:
        eng.set_predictor(predictor)
    eng.md_init(_t(m["masses"]), _t(m["vsites"], torch.int32), _t(m["bonds"], torch.int32),
                _t(m["bond_k"]), _t(m["bond_r0"]), _t(m["rep_radius"]), m["rep_eps"],
                _t(m["vel"]))
    return eng


@pytest.mark.parametrize("case", ["cluster", "box", "cluster-frames"])
def test_md_matches_oracle(case):
    if case.startswith("cluster"):
        d, kw = water_cluster(3, 2), dict(tol=1e-11)
    else:
        d, kw = water_box(8, 8.0, 12), dict(beta=0.5, cutoff=3.7, grid=12, tol=1e-11)
    frames = water_frames(d) if case.endswith("frames") else None
    m = water_md(d, 2)
    steps, dt = 5, 0.5
    ref = omd.run(d, oracle_params(d, **kw), m["masses"], m["vsites"], m["bonds"], m["bond_k"],
                  m["bond_r0"], m["vel"], dt, steps, frames=frames, rho=m["rep_radius"],
                  eps=m["rep_eps"])
    eng = _md_engine(d, kw, m, frames=frames)
    stats = eng.md_run(steps, dt)
    x, v = eng.md_state()
    eng.close()
    x, v = x.cpu().numpy(), v.cpu().numpy()
    xr, vr = ref[-1][0], ref[-1][1]
    dx = np.abs(x - xr).max()
    dv = np.abs(v - vr).max() / np.abs(vr).max()
    say(f"[md] {case}: after {steps} steps |dx| {dx:.1e} A, dv {dv:.1e}, "
        f"iterations {[s[5] for s in stats]}")
    assert dx < 1e-9 and dv < 1e-8
    for s, r in zip(stats, ref):
        for a, b in zip(s[:5], r[2:7]):
            assert abs(a - b) <= 1e-8 * max(abs(b), 1.0), (s, r[2:7])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_md_box216_energy_and_predictor(precision):
    """The paper's MD system (216 waters, 18.643 A box) over 10 fs: the
    spread of the total energy falls as dt^2 (0.5 fs against 0.25 fs
    steps), the Beeman property the oracle's trajectory is pinned by, here
    at a size the oracle cannot follow; and the 3rd-order predictor needs
    fewer solver iterations than the plain warm start over the same steps."""
    d, cfg = config_system("box216")
    kw = dict(beta=cfg["beta"], cutoff=cfg["cutoff"], grid=cfg["grid"], tol=cfg["tol"])
    m = water_md(d, 3)
    spread, its = {}, {}
    for dt, k in ((0.5, 1), (0.25, 1), (0.25, 3)):
        eng = _md_engine(d, kw, m, precision=precision, predictor=k)
        stats = np.array(eng.md_run(int(round(10 / dt)), dt))
        eng.close()
        et = stats[:, :5].sum(1)
        spread[(dt, k)] = et.max() - et.min()
        its[(dt, k)] = int(stats[5:, 5].sum())
        say(f"[md] box216 {precision} dt {dt} predictor {k}: E_tot spread {spread[(dt, k)]:.3e} "
            f"(E_kin {stats[:, 4].mean():.1f}), iterations {stats[:, 5].astype(int).tolist()}")
    ratio = spread[(0.5, 1)] / spread[(0.25, 1)]
    say(f"[md] spread ratio 0.5 fs / 0.25 fs: {ratio:.2f}")
    assert 3.0 < ratio < 5.5
    assert its[(0.25, 3)] < its[(0.25, 1)], its


def test_md_errors():
    from paper_2201_00804_amd import Engine, SibfaError
    d = water_cluster(3, 2)
    m = water_md(d, 0)
    eng = Engine(0)
    eng.load(d, gpu_params(d))
    with pytest.raises(SibfaError) as e:
        eng.md_run(2, 1.0)
    assert e.value.status == -2
    bad = m["masses"].copy()
    bad[3] = 1.0      # a barycentre with mass but listed as a virtual site
    with pytest.raises(SibfaError) as e:
        eng.md_init(_t(bad), _t(m["vsites"], torch.int32), _t(m["bonds"], torch.int32),
                    _t(m["bond_k"]), _t(m["bond_r0"]))
    assert e.value.status == -1
    with pytest.raises(SibfaError) as e:      # a positive strength needs radii
        eng.md_init(_t(m["masses"]), _t(m["vsites"], torch.int32), _t(m["bonds"], torch.int32),
                    _t(m["bond_k"]), _t(m["bond_r0"]), None, 0.5)
    assert e.value.status == -1
    bonds = m["bonds"].copy()
    bonds[0] = [0, 3]  # a bond to a virtual site
    with pytest.raises(SibfaError) as e:
        eng.md_init(_t(m["masses"]), _t(m["vsites"], torch.int32), _t(bonds, torch.int32),
                    _t(m["bond_k"]), _t(m["bond_r0"]))
    assert e.value.status == -1
    eng.md_init(_t(m["masses"]), _t(m["vsites"], torch.int32), _t(m["bonds"], torch.int32),
                _t(m["bond_k"]), _t(m["bond_r0"]))
    with pytest.raises(SibfaError) as e:
        eng.md_run(2, -1.0)
    assert e.value.status == -1
    assert len(eng.md_run(0, 1.0)) == 0
    eng.close()
