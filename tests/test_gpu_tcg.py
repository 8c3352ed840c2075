"""Truncated conjugate gradient (TCG-n) through the C-ABI against the oracle's
TCG on the same seeded inputs.

Bars: FP64 dipoles elementwise within 1e-8 of their largest entry and E_pol
within 1e-6 relative (as for the converged path).  Mixed precision runs every
matvec in FP32 (FP64 accumulation) with no FP64 residual at the end: each
T p carries the FP32 rounding of its coefficients and operand (2^-24 times
the sum of |T_ij p_j|, tens of times |T p| here), so the dipoles are held to
the mixed path's bound of 1e-5 of their largest entry; E_pol still to 1e-6.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.model import System, Context, permanent_field
from oracle.units import COULOMB
from synth import water_box, water_box_ortho, water_cluster, config_system
from tests.gpu_util import say, oracle_params, gpu_params, engine_for, rel_err, pol_rows

pytestmark = pytest.mark.gpu

E_TOL = 1e-6
MU_TOL = {"fp64": 1e-8, "mixed": 1e-5}

CASES = {
    "cluster33": (lambda: water_cluster(33, 3), dict()),
    "box27": (lambda: water_box(27, 9.5, 3), dict(beta=0.45, cutoff=4.5, grid=24)),
    "ortho120": (lambda: water_box_ortho((6, 5, 4), (3.1, 3.1, 3.1), 1),
                 dict(beta=0.45, cutoff=4.5, grid=(36, 30, 24))),
}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_tcg_parity(name, precision):
    make, kw = CASES[name]
    d = make()
    say(f"[tcg] {name} {precision}: n_sites={len(d['pos'])}")
    s = System.from_dict(d)
    op = oracle_params(d, **kw)
    ctx = Context(s, op)
    E0 = permanent_field(s, op, ctx=ctx)
    rows = pol_rows(d)
    eng = engine_for(d, gpu_params(d, precision=precision, **kw))
    for order, omega in ((1, 0.0), (1, 1.0), (2, 0.0), (2, 0.9), (3, 1.0), (24, 0.0)):
        mu_o, e_o = oracle.tcg(s, op, E0, order, omega, ctx=ctx)
        mu_g, e_g = eng.solve_tcg(order, omega)
        mu_g = mu_g.cpu().numpy()
        err = rel_err(mu_g[rows], mu_o)
        say(f"  order {order} omega {omega}: E_pol gpu {e_g:.12g} oracle {e_o:.12g}; "
            f"mu err {err:.2e}")
        assert err < MU_TOL[precision], (order, omega, err)
        assert abs(e_g - e_o) <= E_TOL * abs(e_o), (order, omega, e_g, e_o)
        nonpol = np.setdiff1d(np.arange(len(d["pos"])), rows)
        assert np.all(mu_g[nonpol] == 0.0)
    eng.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tcg_warm_start(precision):
    """TCG from given dipoles (an extrapolated guess handed over with
    set_dipoles) against the oracle's TCG from the same guess; the kept
    dipoles are left as they were; no dipoles yet: E_STATE."""
    from paper_2201_00804_amd import SibfaError
    d = water_box(27, 9.5, 3)
    kw = dict(beta=0.45, cutoff=4.5, grid=24)
    s = System.from_dict(d)
    op = oracle_params(d, **kw)
    ctx = Context(s, op)
    E0 = permanent_field(s, op, ctx=ctx)
    rows = pol_rows(d)
    eng = engine_for(d, gpu_params(d, precision=precision, **kw))
    with pytest.raises(SibfaError) as ei:
        eng.solve_tcg(2, warm_start=True)
    assert ei.value.status == -2
    mu_ref = oracle.model.solve(s, op, E0, ctx=ctx)[0]
    rng = np.random.default_rng(5)
    guess = mu_ref * (1.0 + 0.05 * rng.normal(size=mu_ref.shape))
    full = np.zeros((len(d["pos"]), 3))
    full[rows] = guess
    full_t = torch.as_tensor(full, device="cuda")
    eng.set_dipoles(full_t)
    for order, omega in ((1, 0.0), (2, 1.0), (3, 0.0)):
        mu_o, e_o = oracle.tcg(s, op, E0, order, omega, ctx=ctx, x0=guess)
        mu_g, e_g = eng.solve_tcg(order, omega, warm_start=True)
        err = rel_err(mu_g.cpu().numpy()[rows], mu_o)
        say(f"  warm order {order} omega {omega}: E_pol gpu {e_g:.12g} oracle {e_o:.12g}; "
            f"mu err {err:.2e}")
        assert err < MU_TOL[precision], (order, omega, err)
        assert abs(e_g - e_o) <= E_TOL * abs(e_o), (order, omega, e_g, e_o)
    assert torch.equal(eng.get_dipoles(), full_t)
    eng.close()


def test_tcg_leaves_the_converged_state_alone():
    """A TCG call between a solve and the energies: the energies are those
    of the converged dipoles (the next energy call solves again, warm from
    them), bit for bit, and repeated TCG calls agree bit for bit."""
    d = water_box(27, 9.5, 3)
    eng = engine_for(d, gpu_params(d, beta=0.45, cutoff=4.5, grid=24, tol=1e-10))
    mu, it, _ = eng.solve()
    e_pol, e_elec, F = eng.energy_forces()
    mu1, e1 = eng.solve_tcg(2, 1.0)
    mu2, e2 = eng.solve_tcg(2, 1.0)
    assert e1 == e2 and torch.equal(mu1, mu2)
    assert e1 != e_pol
    e_pol2, e_elec2, F2 = eng.energy_forces()
    assert e_pol2 == e_pol and e_elec2 == e_elec and torch.equal(F, F2)
    assert torch.equal(eng.get_dipoles(), mu)
    _, e_none = eng.solve_tcg(1, 0.0, mu_out=False)
    assert e_none == eng.solve_tcg(1, 0.0)[1]
    eng.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tcg_zero_field(precision):
    """No permanent multipoles: the guess and every residual are zero; the
    steps must leave mu = 0 (no 0/0) and not report an indefinite T."""
    d = water_box(27, 9.5, 3)
    d = dict(d, q=np.zeros_like(d["q"]), dip=np.zeros_like(d["dip"]),
             quad=np.zeros_like(d["quad"]))
    eng = engine_for(d, gpu_params(d, beta=0.45, cutoff=4.5, grid=24, precision=precision))
    for order in (1, 3):
        mu, e = eng.solve_tcg(order, 1.0)
        assert float(mu.abs().max()) == 0.0 and e == 0.0
    eng.close()


def test_tcg_no_polarizable_sites():
    d = water_cluster(5, 4)
    d = dict(d, alpha=np.zeros_like(d["alpha"]))
    eng = engine_for(d, gpu_params(d))
    mu, e = eng.solve_tcg(2, 1.0)
    assert float(mu.abs().max()) == 0.0 and e == 0.0
    eng.close()


def test_tcg_bad_arguments():
    from paper_2201_00804_amd import Engine, SibfaError
    eng = Engine(0)
    with pytest.raises(SibfaError) as ei:
        eng.solve_tcg(1)
    assert ei.value.status == -2     # no system yet
    d = water_cluster(3, 5)
    eng.load(d, gpu_params(d))
    for order, omega in ((0, 0.0), (65, 0.0), (-3, 0.0), (1, float("nan")),
                         (1, float("inf"))):
        with pytest.raises(SibfaError) as ei:
            eng.solve_tcg(order, omega)
        assert ei.value.status == -1, (order, omega)
    mu, e = eng.solve_tcg(64, 0.0)   # the largest order is accepted
    assert np.isfinite(e)
    eng.close()


@pytest.mark.parametrize("name", ["box4096", "box32000"])
def test_tcg_is_the_truncated_pcg_at_full_size(name):
    """At the benchmark sizes, where the oracle cannot run the solve:
    TCG-n without the peek step is the PCG stopped after n iterations (the
    same kernels in the same order, FP64), bit for bit; the peek step adds
    omega alpha (E - T mu) computed from the library's own field and
    operator; E_pol is -1/2 f mu.E0 of the returned dipoles and field."""
    from paper_2201_00804_amd import SibfaError
    d, prm = config_system(name)
    kw = dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"])
    n_it = 3
    eng = engine_for(d, gpu_params(d, tol=1e-14, max_iter=n_it, **kw))
    say(f"[tcg] {name}: n_sites={len(d['pos'])}, {n_it} iterations")
    with pytest.raises(SibfaError) as ei:
        eng.solve()
    assert ei.value.status == -5          # not converged: mu is the 3rd iterate
    mu_pcg = eng.get_dipoles()
    mu, e = eng.solve_tcg(n_it, 0.0)
    assert torch.equal(mu, mu_pcg)
    E0 = eng.permanent_field()
    e_ref = -0.5 * COULOMB * float((mu * E0).sum())
    assert abs(e - e_ref) <= 1e-12 * abs(e_ref), (e, e_ref)
    omega = 0.85
    mu_pk, _ = eng.solve_tcg(n_it, omega)
    r = (E0 - eng.apply_T(mu)).cpu().numpy()
    a3 = np.asarray(d["alpha"])[:, [0, 1, 2, 1, 3, 4, 2, 4, 5]].reshape(-1, 3, 3)
    want = mu.cpu().numpy() + omega * np.einsum("nab,nb->na", a3, r)
    got = mu_pk.cpu().numpy()
    err = rel_err(got - mu.cpu().numpy(), want - mu.cpu().numpy())
    say(f"  peek step vs omega alpha (E - T mu): {err:.2e} of its largest entry")
    assert err < 1e-8
    eng.close()
