"""Error paths through the C-ABI (every failure forced from the host; no
kernel is made to fault) and degenerate systems."""
import numpy as np
import pytest
import torch

import oracle
from oracle.model import System, Params
from synth import water_box, water_cluster
from tests.gpu_util import say, gpu_params, engine_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _status(exc):
    return exc.value.status


def _engine():
    from paper_2201_00804_amd import Engine
    return Engine(0)


def _t(a, dt=torch.float64):
    return torch.as_tensor(a, dtype=dt, device="cuda").contiguous()


def test_bad_arguments():
    from paper_2201_00804_amd import SibfaError
    d = water_box(27, 9.5, 3)
    eng = _engine()
    # cutoff at or above half the box
    with pytest.raises(SibfaError) as e:
        eng.set_system(_t(d["pos"]), _t(d["mol"], torch.int32), d["box"],
                       gpu_params(d, beta=0.45, cutoff=4.8, grid=24))
    assert _status(e) == -1
    # NaN positions
    bad = d["pos"].copy()
    bad[3, 1] = np.nan
    with pytest.raises(SibfaError) as e:
        eng.set_system(_t(bad), _t(d["mol"], torch.int32), d["box"],
                       gpu_params(d, beta=0.45, cutoff=4.5, grid=24))
    assert _status(e) == -1
    # odd grid / unsupported factor
    with pytest.raises(SibfaError) as e:
        eng.set_system(_t(d["pos"]), _t(d["mol"], torch.int32), d["box"],
                       gpu_params(d, beta=0.45, cutoff=4.5, grid=21))
    assert _status(e) == -1
    # the context stays usable after errors
    prm = gpu_params(d, beta=0.45, cutoff=4.5, grid=24)
    eng.set_system(_t(d["pos"]), _t(d["mol"], torch.int32), d["box"], prm)
    # call order: no multipoles yet
    with pytest.raises(SibfaError) as e:
        eng.solve()
    assert _status(e) == -2
    eng.set_multipoles(_t(d["q"]), _t(d["dip"]), _t(d["quad"]))
    # non positive definite polarizability
    al = d["alpha"].copy()
    al[0] = [1.0, 2.0, 0.0, 1.0, 0.0, 1.0]
    eng.set_polarizabilities(_t(al))
    with pytest.raises(SibfaError) as e:
        eng.solve()
    assert _status(e) == -1
    eng.set_polarizabilities(_t(d["alpha"]))
    eng.solve()
    # energies, forces and virial are each optional (the virial is a HOST
    # array of nine doubles)
    import ctypes
    w = (ctypes.c_double * 9)()
    assert eng.lib.sibfa_energy_forces(eng.h, None, None, None, w) == 0
    assert all(np.isfinite(list(w))) and any(x != 0.0 for x in w)
    assert eng.lib.sibfa_energy_forces(eng.h, None, None, None, None) == 0
    eng.close()


def test_nonfinite_positions_after_update():
    """update_positions only enqueues the copy; a NaN coordinate (or one
    beyond 1e6 box edges) is reported by the next call that computes, and
    the context stays usable."""
    from paper_2201_00804_amd import SibfaError
    d = water_box(27, 9.5, 3)
    eng = engine_for(d, gpu_params(d, beta=0.45, cutoff=4.5, grid=24))
    e0 = eng.energy_forces()[0]
    bad = d["pos"].copy()
    bad[7, 2] = np.inf
    eng.update_positions(_t(bad))
    with pytest.raises(SibfaError) as e:
        eng.solve()
    assert _status(e) == -1 and "NaN or Inf" in str(e.value)
    eng.update_positions(_t(d["pos"]))
    assert eng.energy_forces()[0] == e0
    # finite coordinates too far out for the periodic wrap (a run-away atom)
    # are rejected the same way; the kernels queued before the error is
    # read back see them wrapped to 0, inside the grid
    for far in (1e26, -7.1e19):
        bad = d["pos"].copy()
        bad[11, 0] = far
        eng.update_positions(_t(bad))
        with pytest.raises(SibfaError) as e:
            eng.energy_forces()
        assert _status(e) == -1 and "box edges" in str(e.value)
    eng.update_positions(_t(d["pos"]))
    assert eng.energy_forces()[0] == e0
    eng.close()


def test_molecule_ids_out_of_range_and_spread_molecule():
    from paper_2201_00804_amd import SibfaError
    d = water_box(27, 9.5, 3)
    prm = gpu_params(d, beta=0.45, cutoff=4.5, grid=24)
    eng = _engine()
    mol = d["mol"].copy()
    mol[5] = 10 ** 6
    eng.set_system(_t(d["pos"]), _t(mol, torch.int32), d["box"], prm)
    eng.set_multipoles(_t(d["q"]), _t(d["dip"]), _t(d["quad"]))
    eng.set_polarizabilities(_t(d["alpha"]))
    with pytest.raises(SibfaError) as e:
        eng.solve()
    assert _status(e) == -1
    eng.close()
    # a "molecule" whose sites lie farther apart than the neighbour search
    # reaches (1,024-water box: 6 cells per axis, so the 5x5x5 stencil does
    # not cover the whole box)
    from synth import config_system
    d, cfg = config_system("box1024")
    L = d["box"][0]
    dd = d["pos"] - d["pos"][0]
    dd -= L * np.round(dd / L)
    far = int(np.argmax(np.linalg.norm(dd, axis=1)))
    assert np.linalg.norm(dd[far]) > 2 * cfg["cutoff"] + 5
    mol = d["mol"].copy()
    mol[0] = mol[far]
    prm = gpu_params(d, beta=cfg["beta"], cutoff=cfg["cutoff"], grid=cfg["grid"])
    eng = _engine()
    eng.set_system(_t(d["pos"]), _t(mol, torch.int32), d["box"], prm)
    eng.set_multipoles(_t(d["q"]), _t(d["dip"]), _t(d["quad"]))
    eng.set_polarizabilities(_t(d["alpha"]))
    with pytest.raises(SibfaError) as e:
        eng.solve()
    assert _status(e) == -1
    eng.close()


def test_not_converged_returns_dipoles():
    from paper_2201_00804_amd import SibfaError
    d = water_cluster(12, 5)
    eng = engine_for(d, gpu_params(d, tol=1e-12, max_iter=3))
    with pytest.raises(SibfaError) as e:
        eng.solve()
    assert _status(e) == -5
    mu = eng.get_dipoles().cpu().numpy()
    assert np.isfinite(mu).all() and np.abs(mu).max() > 0
    eng.close()


def test_undamped_polarization_is_not_spd():
    """With the Thole factor pushed to 'no damping' the same-molecule
    couplings make T indefinite; the solver reports it (p.Tp <= 0)."""
    from paper_2201_00804_amd import SibfaError
    d = water_cluster(4, 6)
    T = oracle.dense_T_columns(System.from_dict(d), Params(method="direct", thole_a=1e9))
    assert np.linalg.eigvalsh(T).min() < 0
    eng = engine_for(d, gpu_params(d, thole_a=1e9, tol=1e-10, max_iter=200))
    with pytest.raises(SibfaError) as e:
        eng.solve()
    assert _status(e) in (-4, -5)
    say(f"  undamped: status {_status(e)}")
    eng.close()


def test_no_polarizable_sites():
    d = water_box(27, 9.5, 3)
    d["alpha"] = np.zeros_like(d["alpha"])
    kw = dict(beta=0.45, cutoff=4.5, grid=24)
    ref = oracle.evaluate(System.from_dict(d), Params(method="spme", beta=0.45, cutoff=4.5,
                                                      grid=(24, 24, 24)))
    eng = engine_for(d, gpu_params(d, **kw))
    mu, it, rms = eng.solve()
    assert it == 0 and float(mu.abs().max()) == 0.0
    e_pol, e_elec, F = eng.energy_forces()
    assert e_pol == 0.0
    assert e_elec == pytest.approx(ref["E_elec"], rel=1e-9)
    F = F.cpu().numpy()
    assert np.abs(F - ref["forces"]).max() <= 1e-8 * np.abs(ref["forces"]).max()
    eng.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_permanent_field(precision):
    """No permanent multipoles: E = 0, so the cold start is already the
    solution (mu = 0).  The solve must end converged (a zero residual also
    has p.Tp = 0, which must not read as an indefinite T) with zero
    energies and forces."""
    d = water_box(27, 9.5, 3)
    d = dict(d, q=np.zeros_like(d["q"]), dip=np.zeros_like(d["dip"]),
             quad=np.zeros_like(d["quad"]))
    eng = engine_for(d, gpu_params(d, beta=0.45, cutoff=4.5, grid=24, precision=precision))
    mu, it, rms = eng.solve()
    say(f"  {precision}: iterations {it}, rms {rms}")
    assert float(mu.abs().max()) == 0.0 and rms == 0.0
    e_pol, e_elec, F = eng.energy_forces()
    assert e_pol == 0.0 and e_elec == 0.0
    assert float(F.abs().max()) == 0.0
    eng.close()


def test_per_site_thole_factors():
    """Per-site Thole factors with a_ij = min(a_i, a_j) against the oracle."""
    d = water_cluster(7, 8)
    th = np.full(len(d["pos"]), 0.28)
    th[::7] = 0.39
    ref = oracle.evaluate(System.from_dict(d, thole=th), Params(method="direct", tol=1e-10))
    prm = gpu_params(d, tol=1e-10)
    eng = _engine()
    eng.set_system(_t(d["pos"]), _t(d["mol"], torch.int32), None, prm)
    eng.set_multipoles(_t(d["q"]), _t(d["dip"]), _t(d["quad"]))
    eng.set_polarizabilities(_t(d["alpha"]), _t(th))
    eng.solve()
    e_pol, e_elec, F = eng.energy_forces()
    assert e_pol == pytest.approx(ref["E_pol"], rel=1e-9)
    assert np.abs(F.cpu().numpy() - ref["forces"]).max() <= 1e-8 * np.abs(ref["forces"]).max()
    eng.close()


def test_device_memory_from_torch_allocator():
    """Contexts and batch executors take their device memory from torch's
    caching allocator (the alloc/free callbacks of the C-ABI): torch's
    allocated-bytes counter grows by at least the context's buffers while it
    lives and falls back when it is destroyed; results equal those of a
    context that allocates with hipMalloc itself."""
    from paper_2201_00804_amd import Engine
    d = water_box(27, 9.5, 3)
    prm = gpu_params(d, beta=0.45, cutoff=4.5, grid=24, tol=1e-10)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    eng = Engine(0)
    eng.load(d, prm)
    mu, it, _ = eng.solve()
    ep, ee, F = eng.energy_forces()
    held = torch.cuda.memory_allocated() - before
    own = Engine(0, torch_memory=False)
    own.load(d, prm)
    mu2, it2, _ = own.solve()
    ep2, ee2, F2 = own.energy_forces()
    own.close()
    say(f"  torch-held bytes while the context lives: {held}")
    assert held > 1_000_000
    assert torch.equal(mu, mu2) and torch.equal(F, F2) and (ep, ee, it) == (ep2, ee2, it2)
    del mu, F, mu2, F2
    eng.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before
