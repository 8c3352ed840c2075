"""The virial of sibfa_energy_forces (W_ab = -dE/d eps_ab at fixed
global-frame multipoles and dipoles) against the FP64 oracle's virial, which
is pinned by finite strains (tests/test_oracle_virial.py).

Bars: FP64 path, every component within 1e-8 of the largest (both sides
FP64); mixed path within 1e-5 of the largest."""
import numpy as np
import pytest
import torch

import oracle
from oracle.model import System
from synth import water_box, water_box_ortho, water_cluster, config_system
from tests.gpu_util import say, oracle_params, gpu_params, engine_for, rms_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


BARS = {"fp64": 1e-8, "mixed": 1e-5}


def _gpu_virial(d, kw, precision, forces=True):
    eng = engine_for(d, gpu_params(d, precision=precision, **kw))
    eng.solve()
    ep, ee, F, W = eng.energy_forces(forces=forces, virial=True)
    eng.close()
    return np.asarray(W), ep, ee, F


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["cluster33", "box27", "ortho120"])
def test_virial_matches_oracle(case, precision):
    if case == "cluster33":
        d, kw = water_cluster(33, 3), dict(tol=1e-10)
    elif case == "box27":
        d, kw = water_box(27, 9.5, 3), dict(beta=0.45, cutoff=4.5, grid=24, tol=1e-10)
    else:
        d = water_box_ortho((6, 5, 4), (3.1, 3.1, 3.1), 1)
        kw = dict(beta=0.45, cutoff=4.5, grid=(36, 30, 24), tol=1e-10)
    ref = oracle.evaluate(System.from_dict(d), oracle_params(d, **kw), forces=False,
                          with_virial=True)["virial"]
    W, ep, ee, F = _gpu_virial(d, kw, precision)
    err = np.abs(W - ref).max() / np.abs(ref).max()
    say(f"[virial] {case} {precision}: max |W - W_oracle| / max |W| = {err:.2e}; "
        f"trace {np.trace(W):.6f} vs {np.trace(ref):.6f}")
    assert err <= BARS[precision]


def test_virial_without_forces_and_energies_unchanged():
    """Asking for the virial only (no forces) gives the same virial, and
    asking for it leaves the energies bit for bit and the forces to rounding
    as without it (the force kernels' virial variant may contract its
    arithmetic differently)."""
    d, kw = water_box(27, 9.5, 5), dict(beta=0.45, cutoff=4.5, grid=24, tol=1e-10)
    eng = engine_for(d, gpu_params(d, **kw))
    eng.solve()
    ep0, ee0, F0 = eng.energy_forces()
    ep1, ee1, F1, W1 = eng.energy_forces(virial=True)
    ep2, ee2, _, W2 = eng.energy_forces(forces=False, virial=True)
    eng.close()
    assert (ep0, ee0) == (ep1, ee1) == (ep2, ee2)
    dF = rms_rel(F1.cpu().numpy(), F0.cpu().numpy())
    say(f"[virial] forces with / without the virial: rms rel {dF:.2e}")
    assert dF < 1e-12, dF
    assert np.array_equal(np.asarray(W1), np.asarray(W2))


def test_virial_box4096_mixed_vs_fp64():
    """At 4,096 waters: the mixed virial within 1e-5 of the FP64 one (every
    component, relative to the largest)."""
    d, prm = config_system("box4096")
    kw = dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"], tol=prm["tol"],
              max_iter=400)
    W64 = _gpu_virial(d, kw, "fp64", forces=False)[0]
    W32 = _gpu_virial(d, kw, "mixed", forces=False)[0]
    err = np.abs(W32 - W64).max() / np.abs(W64).max()
    say(f"[virial] box4096 mixed vs fp64: {err:.2e}, diag {np.diag(W64)}")
    assert err <= BARS["mixed"]
