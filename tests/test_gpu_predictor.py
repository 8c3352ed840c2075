"""The warm-start predictor (sibfa_set_predictor) through the C-ABI: the
extrapolated guess, seen through TCG from it, against the oracle's TCG
from the oracle's extrapolation (solver.extrapolate, pinned in
tests/test_oracle_predictor.py) of the same dipole history; and fewer PCG
iterations along a smooth trajectory at unchanged converged results."""
import numpy as np
import pytest
import torch

import oracle
from oracle import solver
from oracle.model import System, Context, permanent_field
from synth import water_box, config_system
from tests.gpu_util import say, oracle_params, gpu_params, engine_for, rel_err, pol_rows

pytestmark = pytest.mark.gpu

MU_TOL = {"fp64": 1e-8, "mixed": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("k,pushed", [(2, 2), (3, 5), (4, 4), (6, 5), (3, 8), (1, 3)])
def test_predicted_guess_matches_oracle(k, pushed, precision):
    """`pushed` dipole sets handed over with set_dipoles (oldest first; more
    than six wrap the ring, fewer than k truncate the order), then TCG from
    the predicted guess."""
    d = water_box(27, 9.5, 3)
    kw = dict(beta=0.45, cutoff=4.5, grid=24)
    s = System.from_dict(d)
    op = oracle_params(d, **kw)
    ctx = Context(s, op)
    E0 = permanent_field(s, op, ctx=ctx)
    rows = pol_rows(d)
    mu_ref = oracle.model.solve(s, op, E0, ctx=ctx)[0]
    rng = np.random.default_rng(100 + 10 * k + pushed)
    hist = [mu_ref * (1.0 + 0.03 * rng.normal(size=mu_ref.shape)) for _ in range(pushed)]
    eng = engine_for(d, gpu_params(d, precision=precision, **kw))
    eng.set_predictor(k)
    for h in hist:
        full = np.zeros((len(d["pos"]), 3))
        full[rows] = h
        eng.set_dipoles(torch.as_tensor(full, device="cuda"))
    guess = solver.extrapolate(hist[::-1], k)
    for order, omega in ((1, 0.0), (3, 1.0)):
        mu_o, e_o = oracle.tcg(s, op, E0, order, omega, ctx=ctx, x0=guess)
        mu_g, e_g = eng.solve_tcg(order, omega, warm_start=True)
        err = rel_err(mu_g.cpu().numpy()[rows], mu_o)
        say(f"  predictor k={k} after {pushed} sets, TCG-{order}: mu err {err:.2e}, "
            f"E_pol {e_g:.10g} vs {e_o:.10g}")
        assert err < MU_TOL[precision]
        assert abs(e_g - e_o) <= 1e-6 * abs(e_o)
    eng.close()


def test_predictor_cuts_iterations_along_a_trajectory():
    """Positions moving on a smooth (quadratic) path, 0.01 A per step at
    most, warm-started solves each step: the 4th-order predictor needs fewer
    iterations in total than the plain warm start, and the converged
    energies at the last step equal a cold solve's to the tolerance."""
    d, cfg = config_system("box216")
    kw = dict(beta=cfg["beta"], cutoff=cfg["cutoff"], grid=cfg["grid"], tol=cfg["tol"])
    rng = np.random.default_rng(11)
    v = 0.004 * rng.standard_normal(d["pos"].shape)
    a = 0.0005 * rng.standard_normal(d["pos"].shape)
    steps = 10
    totals = {}
    last = {}
    for k in (1, 4):
        eng = engine_for(d, gpu_params(d, **kw))
        eng.set_predictor(k)
        its = []
        for t in range(steps):
            pos = d["pos"] + t * v + 0.5 * t * t * a
            eng.update_positions(torch.as_tensor(pos, device="cuda"))
            _, it, rms = eng.solve(warm_start=t > 0)
            its.append(it)
        last[k] = eng.energy_forces(forces=False)[:2]
        eng.close()
        totals[k] = sum(its[3:])
        say(f"  predictor order {k}: iterations per step {its}")
    cold = engine_for(dict(d, pos=d["pos"] + (steps - 1) * v + 0.5 * (steps - 1) ** 2 * a),
                      gpu_params(d, **kw))
    cold.solve()
    ec = cold.energy_forces(forces=False)[:2]
    cold.close()
    assert totals[4] < totals[1], totals
    for k in (1, 4):
        assert abs(last[k][0] - ec[0]) <= 1e-6 * abs(ec[0])
        assert abs(last[k][1] - ec[1]) <= 1e-9 * abs(ec[1])


def test_predictor_order_checked_and_history_cleared():
    from paper_2201_00804_amd import SibfaError
    d = water_box(27, 9.5, 3)
    eng = engine_for(d, gpu_params(d, beta=0.45, cutoff=4.5, grid=24))
    for bad in (-1, 7):
        with pytest.raises(SibfaError) as e:
            eng.set_predictor(bad)
        assert e.value.status == -1
    # new polarizabilities clear the kept dipoles and the history: a warm
    # TCG then has nothing to start from
    eng.set_predictor(3)
    eng.solve()
    eng.set_polarizabilities(torch.as_tensor(d["alpha"], device="cuda"))
    with pytest.raises(SibfaError) as e:
        eng.solve_tcg(1, warm_start=True)
    assert e.value.status == -2
    eng.close()
