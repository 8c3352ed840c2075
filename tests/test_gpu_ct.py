"""Reduced charge transfer through the C-ABI (sibfa_set_charge_transfer /
sibfa_ct_energy_forces) against the FP64 oracle (oracle/ct.py, pinned in
tests/test_oracle_ct.py): E_ct and its forces on a cluster, the 27-water
box, the 120-water orthorhombic box and the 216-water box, each water with
two lone-pair sites.

With local frames (the dipoles and quadrupoles given in molecular frames,
sibfa_set_local_frames): E_ct and the forces including the rotation against
oracle/ct.py energy_forces_frames, itself pinned by central differences.

Bars: E_ct within 1e-10 relative, forces within 1e-8 of the largest (both
sides FP64, different summation order)."""
import numpy as np
import pytest
import torch

from oracle import ct as oct_
from oracle.model import System
from synth import (water_box, water_cluster, water_box_ortho, water_lone_pairs, water_ct,
                   config_system, water_frames, CT_SITES)
from tests.gpu_util import say, oracle_params, gpu_params, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _t(a, dt=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dt, device="cuda").contiguous()


def _case(name):
    if name == "cluster":
        return water_lone_pairs(water_cluster(12, 5)), {}
    if name == "box27":
        return water_lone_pairs(water_box(27, 9.5, 3)), dict(beta=0.45, cutoff=4.5, grid=24)
    if name == "ortho120":
        d = water_box_ortho((6, 5, 4), (3.1, 3.1, 3.1), 1)
        return water_lone_pairs(d), dict(beta=0.45, cutoff=4.5, grid=(36, 30, 24))
    d, cfg = config_system("box216")
    return water_lone_pairs(d), dict(beta=cfg["beta"], cutoff=cfg["cutoff"], grid=cfg["grid"])


def _ct_engine(d, kw, ct, precision="fp64"):
    from paper_2201_00804_amd import Engine
    eng = Engine(0)
    eng.load(d, gpu_params(d, precision=precision, **kw))
    eng.set_charge_transfer(_t(ct["lp"], torch.int32), _t(ct["lp_par"]),
                            _t(ct["acc"], torch.int32), _t(ct["ah"]), _t(ct["rvdw"]),
                            ct["eta"], ct["cs"], ct["cp"], ct["t"], ct["m"])
    return eng


@pytest.mark.parametrize("case", ["cluster", "box27", "ortho120", "box216"])
def test_ct_matches_oracle(case):
    d, kw = _case(case)
    ct = water_ct(d)
    E_o, F_o = oct_.energy_forces(System.from_dict(d), oracle_params(d, **kw), ct)
    eng = _ct_engine(d, kw, ct)
    E, F = eng.ct_energy_forces()
    E2, none = eng.ct_energy_forces(forces=False)
    eng.close()
    F = F.cpu().numpy()
    err = rel_err(F, F_o)
    say(f"[ct] {case}: E_ct {E:.10f} vs {E_o:.10f} (rel {abs(E - E_o) / abs(E_o):.1e}), "
        f"forces {err:.2e}, max |F| {np.abs(F_o).max():.3f}")
    assert abs(E - E_o) <= 1e-10 * abs(E_o)
    assert err <= 1e-8
    assert E2 == E and none is None


@pytest.mark.parametrize("case", ["cluster", "box27", "box216"])
def test_ct_local_frames_match_oracle(case):
    from paper_2201_00804_amd import SibfaError
    d, kw = _case(case)
    ct = water_ct(d)
    fr = water_frames(d, CT_SITES)
    E_o, F_o = oct_.energy_forces_frames(System.from_dict(d), fr, oracle_params(d, **kw), ct)
    eng = _ct_engine(d, kw, ct)
    eng.set_local_frames(_t(fr, torch.int32), _t(d["dip"]), _t(d["quad"]), _t(d["alpha"]))
    with pytest.raises(SibfaError) as e:   # frames switched the term off
        eng.ct_energy_forces()
    assert e.value.status == -2
    eng.set_charge_transfer(_t(ct["lp"], torch.int32), _t(ct["lp_par"]),
                            _t(ct["acc"], torch.int32), _t(ct["ah"]), _t(ct["rvdw"]),
                            ct["eta"], ct["cs"], ct["cp"], ct["t"], ct["m"])
    E, F = eng.ct_energy_forces()
    eng.close()
    F = F.cpu().numpy()
    err = rel_err(F, F_o)
    say(f"[ct frames] {case}: E_ct {E:.10f} vs {E_o:.10f} (rel {abs(E - E_o) / abs(E_o):.1e}), "
        f"forces {err:.2e}")
    assert abs(E - E_o) <= 1e-10 * abs(E_o)
    assert err <= 1e-8


def test_ct_leaves_the_polarization_path_alone_and_follows_positions():
    """Lone-pair sites are inert for E_pol and E_elec (equal to a context
    without them, up to the summation order); a CT call between two
    energy calls changes nothing; after update_positions the CT terms are
    those of the new geometry."""
    from paper_2201_00804_amd import Engine
    d5 = water_box(27, 9.5, 3)
    d, kw = water_lone_pairs(d5), dict(beta=0.45, cutoff=4.5, grid=24)
    ct = water_ct(d)
    eng = _ct_engine(d, kw, ct)
    ep, ee, _ = eng.energy_forces()
    eng.ct_energy_forces()
    ep2, ee2, _ = eng.energy_forces()
    assert (ep, ee) == (ep2, ee2)
    plain = Engine(0)
    plain.load(d5, gpu_params(d5, **kw))
    ep5, ee5, _ = plain.energy_forces()
    plain.close()
    assert ep == pytest.approx(ep5, rel=1e-10) and ee == pytest.approx(ee5, rel=1e-10)
    rng = np.random.default_rng(8)
    d2 = dict(d, pos=d["pos"] + 0.03 * rng.standard_normal(d["pos"].shape))
    eng.update_positions(_t(d2["pos"]))
    E, F = eng.ct_energy_forces()
    eng.close()
    E_o, F_o = oct_.energy_forces(System.from_dict(d2), oracle_params(d2, **kw), ct)
    assert abs(E - E_o) <= 1e-10 * abs(E_o) and rel_err(F.cpu().numpy(), F_o) <= 1e-8


def test_ct_errors():
    from paper_2201_00804_amd import Engine, SibfaError
    d, kw = _case("cluster")
    ct = water_ct(d)
    eng = Engine(0)
    eng.set_system(_t(d["pos"]), _t(d["mol"], torch.int32), None, gpu_params(d))
    with pytest.raises(SibfaError) as e:
        eng.set_charge_transfer(_t(ct["lp"], torch.int32), _t(ct["lp_par"]),
                                _t(ct["acc"], torch.int32), _t(ct["ah"]), _t(ct["rvdw"]),
                                1, 1, 1, 1, 1)
    assert e.value.status == -2
    eng.close()
    eng = _ct_engine(d, kw, ct)
    # a lone-pair site with a charge
    q = d["q"].copy()
    q[ct["lp"][0, 0]] = 0.1
    eng.set_multipoles(_t(q), _t(d["dip"]), _t(d["quad"]))
    with pytest.raises(SibfaError) as e:   # set_multipoles switched the term off
        eng.ct_energy_forces()
    assert e.value.status == -2
    with pytest.raises(SibfaError) as e:
        eng.set_charge_transfer(_t(ct["lp"], torch.int32), _t(ct["lp_par"]),
                                _t(ct["acc"], torch.int32), _t(ct["ah"]), _t(ct["rvdw"]),
                                ct["eta"], ct["cs"], ct["cp"], ct["t"], ct["m"])
    assert e.value.status == -1
    # a lone pair given a local dipole through the frames
    fr = water_frames(d, CT_SITES)
    fr[ct["lp"][0, 0]] = fr[ct["lp"][0, 1]]
    dl = d["dip"].copy()
    dl[ct["lp"][0, 0]] = 0.2
    eng.set_multipoles(_t(d["q"]), _t(d["dip"]), _t(d["quad"]))
    eng.set_local_frames(_t(fr, torch.int32), _t(dl), _t(d["quad"]))
    with pytest.raises(SibfaError) as e:
        eng.set_charge_transfer(_t(ct["lp"], torch.int32), _t(ct["lp_par"]),
                                _t(ct["acc"], torch.int32), _t(ct["ah"]), _t(ct["rvdw"]),
                                ct["eta"], ct["cs"], ct["cp"], ct["t"], ct["m"])
    assert e.value.status == -1
    eng.set_local_frames(None)
    # an acceptor spread over two molecules
    eng.set_multipoles(_t(d["q"]), _t(d["dip"]), _t(d["quad"]))
    acc = ct["acc"].copy()
    acc[0, 1] = 9
    with pytest.raises(SibfaError) as e:
        eng.set_charge_transfer(_t(ct["lp"], torch.int32), _t(ct["lp_par"]),
                                _t(acc, torch.int32), _t(ct["ah"]), _t(ct["rvdw"]),
                                ct["eta"], ct["cs"], ct["cp"], ct["t"], ct["m"])
    assert e.value.status == -1
    eng.close()
