"""Parity at the full workload sizes, on sampled outputs the oracle computes
site by site, and properties that hold at any size.

At 4,096 and 32,000 waters the oracle evaluates, for a random sample of
sites, the permanent field, the rows of T applied to the GPU's induced
dipoles, and the forces at the GPU's dipoles (forces are taken at fixed mu,
so they can be checked site by site); the reciprocal and self energies are
checked in full.  The solve itself is checked through its residual
E - T mu at the sampled sites.  Energy/force consistency is checked by
central differences of the GPU's own energies (SPME forces are exact
gradients of the SPME energy).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.model import System, Context, permanent_field, apply_T, energy_forces
from oracle.units import COULOMB, DEBYE
from synth import config_system, water_box
from tests.gpu_util import say, oracle_params, gpu_params, engine_for, rel_err, rms_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


# Bars of the sampled parity.  FP64: both sides FP64, only summation order
# differs.  Mixed: the GPU's pair and PME arithmetic is FP32 (about 1e-7
# relative per term), so fields and T rows carry ~1e-6 of their largest
# entry; the residual against the oracle's field is then set by the FP32
# field (|alpha dE| ~ 1e-7 e A ~ 5e-7 D), not by the solver tolerance.
SAMPLED_BARS = {
    "fp64": dict(field=1e-8, rows=1e-8, resid=None, force=1e-5, erec=1e-9, eself=1e-12),
    "mixed": dict(field=1e-5, rows=1e-5, resid=1e-5, force=1e-4, erec=1e-6, eself=1e-12),
}


def _sampled_parity(name, n_sample, seed=3, precision="fp64"):
    bars = SAMPLED_BARS[precision]
    d, prm = config_system(name)
    kw = dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"], tol=prm["tol"])
    say(f"[large] {name} {precision}: {len(d['pos'])} sites, sample {n_sample}")
    eng = engine_for(d, gpu_params(d, precision=precision, max_iter=400, **kw))
    E0_g = eng.permanent_field().cpu().numpy()
    mu_g, it, rms = eng.solve()
    mu_g = mu_g.cpu().numpy()
    Tmu_g = eng.apply_T(torch.as_tensor(mu_g, device="cuda")).cpu().numpy()
    e_pol, e_elec, F_g = eng.energy_forces()
    F_g = F_g.cpu().numpy()
    st = eng.stats()
    eng.close()
    assert rms <= prm["tol"]

    s = System.from_dict(d)
    op = oracle_params(d, **kw)
    rng = np.random.default_rng(seed)
    pol = s.pol
    samp_pol = np.sort(rng.choice(pol, n_sample, replace=False))
    samp_all = np.sort(rng.choice(s.n, n_sample, replace=False))
    ctx = Context(s, op, subset=np.union1d(samp_pol, samp_all))
    # permanent field at sampled polarizable sites
    E0_o = permanent_field(s, op, ctx=ctx, sites=samp_pol)
    e_field = rel_err(E0_g[samp_pol], E0_o)
    # rows of T applied to the GPU dipoles, and the residual at those rows
    Tmu_o = apply_T(s, op, mu_g[pol], ctx=ctx, sites=samp_pol)
    e_rows = rel_err(Tmu_g[samp_pol], Tmu_o)
    a3 = s.alpha3[samp_pol]
    z = np.einsum("nab,nb->na", a3, E0_o - Tmu_o)
    resid = DEBYE * np.sqrt(np.mean(np.sum(z * z, 1)))
    # forces at fixed mu at sampled sites
    _, _, _, F_o = energy_forces(s, op, mu_g[pol], None, ctx=ctx, sites=samp_all)
    e_force = rms_rel(F_g[samp_all], F_o)
    say(f"  field {e_field:.2e}, T rows {e_rows:.2e}, residual vs oracle field {resid:.2e} D, "
        f"forces {e_force:.2e}")
    assert e_field < bars["field"]
    assert e_rows < bars["rows"]
    assert resid < (bars["resid"] or 20 * prm["tol"])
    assert e_force < bars["force"]
    # E_pol from the returned arrays (Eq. 19) and the variational form (Eq. 17)
    e19 = -0.5 * COULOMB * float(np.sum(mu_g[pol] * E0_g[pol]))
    assert e_pol == pytest.approx(e19, rel=1e-12)
    # Eq. 17 - Eq. 19 = -1/2 mu.(E - T mu): first order in the residual,
    # ~1e-9 relative at a 1e-8 D tolerance
    assert st["e_pol_variational"] == pytest.approx(e_pol, rel=1e-7)
    # reciprocal and self energies in full
    mult = (s.q, s.dip, s.th)
    erec, _ = ctx.recip_derivs(mult, s.pos[:1], 0)
    b = op.beta
    eself = -np.sum(b / np.sqrt(np.pi) * s.q ** 2
                    + 2 * b ** 3 / (3 * np.sqrt(np.pi)) * np.sum(s.dip ** 2, 1)
                    + 8 * b ** 5 / (45 * np.sqrt(np.pi)) * np.sum(s.th * s.th, (1, 2)))
    say(f"  E_rec rel {abs(st['e_elec_recip'] / (COULOMB * erec) - 1):.2e}, "
        f"E_self rel {abs(st['e_elec_self'] / (COULOMB * eself) - 1):.2e}")
    assert st["e_elec_recip"] == pytest.approx(COULOMB * erec, rel=bars["erec"])
    assert st["e_elec_self"] == pytest.approx(COULOMB * eself, rel=bars["eself"])
    say(f"  iters {it}, E_pol {e_pol:.6f}, E_elec {e_elec:.6f}")


@pytest.mark.slow
def test_box4096_sampled():
    _sampled_parity("box4096", 48)


@pytest.mark.slow
def test_box32000_sampled():
    _sampled_parity("box32000", 16)


@pytest.mark.slow
def test_box32000_sampled_mixed():
    """The benchmark workload in the benchmarked precision: sampled field,
    T rows and forces of the FP32-mixed path against the FP64 oracle."""
    _sampled_parity("box32000", 16, precision="mixed")


@pytest.mark.slow
def test_box96000_sampled():
    """The largest workload: 480,000 sites, a 144^3 grid (the five-pass FFT
    path: its planes do not fit a workgroup's LDS)."""
    _sampled_parity("box96000", 8)


def test_fd_forces_on_gpu_energy():
    """-(E(x+h) - E(x-h))/2h of the GPU's total energy against its forces,
    at a few sites of a 1,024-water box (cold solve to 1e-11 D each time)."""
    d, prm = config_system("box1024")
    kw = dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"], tol=1e-11)
    eng = engine_for(d, gpu_params(d, **kw, max_iter=400))
    pos = torch.as_tensor(d["pos"], device="cuda")
    eng.solve()
    _, _, F = eng.energy_forces()
    F = F.cpu().numpy()
    h = 1e-4
    scale = np.abs(F).max()
    L = d["box"][0]
    clear = []
    for i in range(0, len(d["pos"]), 97):
        dd = d["pos"] - d["pos"][i]
        dd -= L * np.round(dd / L)
        if np.all(np.abs(np.linalg.norm(dd, axis=1) - prm["cutoff"]) > 1e-3):
            clear.append(i)
    assert len(clear) >= 4
    for (i, a) in [(clear[0], 0), (clear[1], 1), (clear[len(clear) // 2], 2), (clear[-1], 0)]:
        e = []
        for sgn in (1, -1):
            p2 = pos.clone()
            p2[i, a] += sgn * h
            eng.update_positions(p2)
            eng.solve()
            ep, ee, _ = eng.energy_forces(forces=False)
            e.append(ep + ee)
        fd = -(e[0] - e[1]) / (2 * h)
        say(f"  FD site {i} axis {a}: {fd:.8f} vs {F[i, a]:.8f}")
        assert abs(fd - F[i, a]) <= 2e-4 * scale
    eng.close()


def test_warm_start_and_position_update_match_fresh():
    d, prm = config_system("box216")
    kw = dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"], tol=1e-10)
    eng = engine_for(d, gpu_params(d, **kw))
    mu0, it0, _ = eng.solve()
    mu1, it1, _ = eng.solve(warm_start=True)
    assert it1 <= 1
    assert rel_err(mu1.cpu().numpy(), mu0.cpu().numpy()) < 1e-8
    # move every site a little: warm start from the old dipoles
    rng = np.random.default_rng(11)
    d2 = dict(d, pos=d["pos"] + rng.uniform(-0.01, 0.01, size=d["pos"].shape))
    eng.update_positions(torch.as_tensor(d2["pos"], device="cuda"))
    mu2, it2, _ = eng.solve(warm_start=True)
    ep2, ee2, F2 = eng.energy_forces()
    fresh = engine_for(d2, gpu_params(d2, **kw))
    mu3, it3, _ = fresh.solve()
    ep3, ee3, F3 = fresh.energy_forces()
    say(f"  warm iterations {it2} vs cold {it3}")
    assert it2 < it3
    assert rel_err(mu2.cpu().numpy(), mu3.cpu().numpy()) < 1e-7
    assert ep2 == pytest.approx(ep3, rel=1e-9)
    assert ee2 == pytest.approx(ee3, rel=1e-12)
    assert rms_rel(F2.cpu().numpy(), F3.cpu().numpy()) < 1e-8
    eng.close()
    fresh.close()


# Bounds of the FP32-mixed path against the FP64 path, per result.  The
# FP32 parts are the pair arithmetic of the intermolecular real-space
# kernels (separations formed in FP64, then rounded) and the reciprocal
# part of T p; sums, reductions, the same-molecule terms, the self terms,
# the permanent multipoles' reciprocal pass and the true residual are FP64.
# A pair term then carries a few tens of FP32 unit roundoffs
# (u = 2^-24 = 6e-8; the FP32 erfcx and exp add at most 12 u), and the
# sums in FP64 average them:
#  E_pol          1e-6 relative (measured about 1 u)
#  forces         1e-5 relative RMS (measured about 10 u)
#  mu             1e-6 D RMS (measured below 1e-7 D: T's FP32 rounding
#                 scaled by the condition number, about 3.5)
#  E_elec real    5e-8 relative (pair terms of mixed signs average their
#                 rounding: measured 1e-8 at 216 waters, 2e-10 at 32,000)
#  E_elec recip   1e-12 relative (the same FP64 pass in both modes)
#  E_elec         5e-8 of |E_elec real| in absolute terms, and 3e-4 of
#                 E_elec itself, a small sum of large real-space, self and
#                 reciprocal terms (at 32,000 waters about 24 kcal/mol out of
#                 terms of about 2e6)
MIXED_BOUNDS = dict(e_pol=1e-6, e_elec=3e-4, e_elec_of_real=5e-8, real=5e-8, recip=1e-12,
                    force=1e-5, mu=1e-6)


@pytest.mark.parametrize("name", ["box216", "box4096",
                                  pytest.param("box32000", marks=pytest.mark.slow),
                                  pytest.param("box96000", marks=pytest.mark.slow)])
def test_mixed_precision_bounds(name):
    """FP32 pair/PME arithmetic with FP64 accumulation, reductions and true
    residual: the solve still meets the FP64 tolerance against the FP64
    operator, and each result stays within the bounds above of the FP64
    path."""
    d, prm = config_system(name)
    kw = dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"], tol=prm["tol"])
    res = {}
    for prec in ("fp64", "mixed"):
        eng = engine_for(d, gpu_params(d, precision=prec, max_iter=400, **kw))
        mu, it, rms = eng.solve()
        ep, ee, F = eng.energy_forces()
        res[prec] = (mu.cpu().numpy(), it, rms, ep, ee, F.cpu().numpy(), eng.stats())
        eng.close()
    mu64, it64, rms64, ep64, ee64, F64, st64 = res["fp64"]
    mu32, it32, rms32, ep32, ee32, F32, st32 = res["mixed"]
    b = MIXED_BOUNDS
    mu_rms = DEBYE * np.sqrt(np.mean(np.sum((mu32 - mu64) ** 2, 1)))
    parts = {k: abs(st32[k] - st64[k]) / abs(st64[k]) for k in ("e_elec_real", "e_elec_recip")}
    say(f"  {name} mixed: iters {it32} (fp64 {it64}), E_pol rel {abs(ep32 - ep64) / abs(ep64):.2e}, "
        f"E_elec rel {abs(ee32 - ee64) / abs(ee64):.2e} (real {parts['e_elec_real']:.2e}, "
        f"recip {parts['e_elec_recip']:.2e}), F rms rel {rms_rel(F32, F64):.2e}, "
        f"mu rms {mu_rms:.2e} D")
    assert rms32 <= prm["tol"]
    assert abs(ep32 - ep64) <= b["e_pol"] * abs(ep64)
    assert parts["e_elec_real"] <= b["real"] and parts["e_elec_recip"] <= b["recip"]
    assert abs(ee32 - ee64) <= b["e_elec_of_real"] * abs(st64["e_elec_real"])
    assert abs(ee32 - ee64) <= b["e_elec"] * abs(ee64)
    assert rms_rel(F32, F64) <= b["force"]
    assert mu_rms <= b["mu"]


def test_mixed_tight_tolerance():
    """A tolerance far below what FP32 iterations alone reach: the mixed
    solve gets there by replacing the recurrence residual with the FP64 true
    residual and continuing the same sequence.  Checked independently: the
    FP64 operator of a second context, applied to the mixed dipoles, leaves
    a residual against the mixed context's own field within the tolerance."""
    from tests.gpu_util import pol_rows
    d, prm = config_system("box1024")
    kw = dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"], tol=1e-11, max_iter=400)
    e32 = engine_for(d, gpu_params(d, precision="mixed", **kw))
    mu, it, rms = e32.solve()
    st = e32.stats()
    E0 = e32.permanent_field().cpu().numpy()
    e32.close()
    e64 = engine_for(d, gpu_params(d, precision="fp64", **kw))
    it64 = e64.solve()[1]
    Tmu = e64.apply_T(mu).cpu().numpy()
    e64.close()
    rows = pol_rows(d)
    r = (E0 - Tmu)[rows]
    a = d["alpha"][rows]
    A = np.stack([np.stack([a[:, 0], a[:, 1], a[:, 2]], 1), np.stack([a[:, 1], a[:, 3], a[:, 4]], 1),
                  np.stack([a[:, 2], a[:, 4], a[:, 5]], 1)], 1)
    z = np.einsum("nij,nj->ni", A, r)
    rho = DEBYE * np.sqrt(np.mean(np.sum(z * z, 1)))
    say(f"  tol 1e-11: mixed {it} iterations ({st['restarts']} replacements; fp64 {it64}), "
        f"reported rms {rms:.2e} D, recomputed {rho:.2e} D")
    assert rms <= 1e-11 and st["restarts"] >= 1
    assert rho <= 2e-11
    assert it <= it64 + 4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bitwise_reproducible(precision):
    """Cell sort, brick lists, spreading, FFT, solver reductions and forces
    take every sum in a fixed order, so two evaluations of the same input
    (fresh contexts, and a repeat on one context) agree bit for bit."""
    d, prm = config_system("box1024")
    kw = dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"], tol=prm["tol"],
              precision=precision)
    out = []
    for _ in range(2):
        eng = engine_for(d, gpu_params(d, **kw))
        mu, it, rms = eng.solve()
        ep, ee, F = eng.energy_forces()
        out.append((mu, it, rms, ep, ee, F))
        eng.update_positions(torch.as_tensor(d["pos"], device="cuda"))
        mu2, it2, rms2 = eng.solve()
        ep2, ee2, F2 = eng.energy_forces()
        out.append((mu2, it2, rms2, ep2, ee2, F2))
        eng.close()
    ref = out[0]
    for o in out[1:]:
        assert torch.equal(o[0], ref[0]) and torch.equal(o[5], ref[5])
        assert o[1:5] == ref[1:5]
