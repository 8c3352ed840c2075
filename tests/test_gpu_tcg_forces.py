"""TCG-n forces through the C-ABI (sibfa_tcg_energy_forces) against central
differences of the oracle's TCG energy (model.tcg_energy, pinned in
tests/test_oracle_tcg_forces.py), cold and from a fixed guess, with and
without the peek step; and, where the oracle cannot follow, TCG at a high
order against the converged forces of sibfa_energy_forces.

Bars: forces within 1e-6 of the largest (the differences' own error is
about 1e-8), energies 1e-9 relative."""
import numpy as np
import pytest
import torch

from oracle.model import System, tcg_energy
from synth import water_box, water_cluster, config_system
from tests.gpu_util import say, oracle_params, gpu_params, engine_for, pol_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _fd(s, prm, order, omega, sites, x0=None, h=1e-5):
    out = []
    for i, a in sites:
        p = s.pos.copy()
        p[i, a] += h
        ep = tcg_energy(System(**{**s.__dict__, "pos": p}), prm, order, omega, x0)
        p[i, a] -= 2 * h
        em = tcg_energy(System(**{**s.__dict__, "pos": p}), prm, order, omega, x0)
        out.append(-(ep - em) / (2 * h))
    return np.array(out)


CASES = [("cluster", 1, 0.0, False), ("cluster", 2, 1.0, False), ("cluster", 3, 0.0, True),
         ("box", 1, 0.0, False), ("box", 2, 1.0, False), ("box", 2, 0.0, True)]


@pytest.mark.parametrize("case,order,omega,warm", CASES)
def test_tcg_forces_match_oracle_differences(case, order, omega, warm):
    if case == "cluster":
        d, kw = water_cluster(4, 6), {}
    else:
        d, kw = water_box(8, 8.0, 12), dict(beta=0.5, cutoff=3.7, grid=12)
    s = System.from_dict(d)
    prm = oracle_params(d, **kw)
    rows = pol_rows(d)
    eng = engine_for(d, gpu_params(d, **kw))
    x0 = None
    if warm:
        rng = np.random.default_rng(order)
        eng.solve()
        mu = eng.get_dipoles().cpu().numpy()
        x0 = mu[rows] * (1.0 + 0.05 * rng.standard_normal(mu[rows].shape))
        full = np.zeros_like(mu)
        full[rows] = x0
        eng.set_dipoles(torch.as_tensor(full, device="cuda"))
    ep, ee, F, _ = eng.tcg_energy_forces(order, omega, warm_start=warm)
    eng.close()
    F = F.cpu().numpy()
    e_ref = tcg_energy(s, prm, order, omega, x0)
    sites = [(0, 0), (1, 2), (2, 1), (3, 0), (4, 2), (7, 1), (10, 0), (13, 2)]
    fd = _fd(s, prm, order, omega, sites, x0)
    got = np.array([F[i, a] for i, a in sites])
    err = np.abs(got - fd).max() / np.abs(F).max()
    say(f"[tcg-forces] {case} order {order} omega {omega} warm {warm}: E {ep + ee:.10f} vs "
        f"{e_ref:.10f}, forces vs differences {err:.2e}")
    assert abs(ep + ee - e_ref) <= 1e-9 * abs(e_ref)
    assert err <= 1e-6


def test_high_order_tcg_forces_are_the_converged_forces():
    """At 216 waters: TCG-40 dipoles are converged far below 1e-8 D, so its
    forces (every step of the iteration differentiated) equal the
    fixed-dipole forces of the converged solve."""
    d, cfg = config_system("box216")
    kw = dict(beta=cfg["beta"], cutoff=cfg["cutoff"], grid=cfg["grid"], tol=1e-12, max_iter=400)
    eng = engine_for(d, gpu_params(d, **kw))
    eng.solve()
    ep0, ee0, F0 = eng.energy_forces()
    ep, ee, F, _ = eng.tcg_energy_forces(40)
    F0 = F0.cpu().numpy()
    F = F.cpu().numpy()
    ep1, ee1, F1, _ = eng.tcg_energy_forces(1)
    eng.close()
    err = np.abs(F - F0).max() / np.abs(F0).max()
    err1 = np.abs(F1.cpu().numpy() - F0).max() / np.abs(F0).max()
    say(f"[tcg-forces] box216: TCG-40 vs converged forces {err:.2e} (TCG-1 {err1:.2e}), "
        f"E_pol {ep:.8f} vs {ep0:.8f}")
    assert err <= 1e-7
    assert abs(ep - ep0) <= 1e-9 * abs(ep0) and ee == pytest.approx(ee0, rel=1e-12)
    assert err1 > 10 * err
