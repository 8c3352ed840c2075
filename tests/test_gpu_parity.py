"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Bars (FP64 path): energies within 1e-6 relative, forces within 1e-5
relative RMS; fields, T p and mu elementwise within 1e-8 of their largest
entry (both sides are FP64; only summation order and library erfc/exp
differ).  Integer work (neighbour counts) bit-exact.
"""
import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

import oracle
from oracle.model import System, Context, permanent_field, apply_T
from synth import water_box, water_box_ortho, water_cluster, config_system
from tests.gpu_util import (say, oracle_params, gpu_params, engine_for, rel_err, rms_rel,
                            pol_rows)

pytestmark = pytest.mark.gpu

E_TOL = 1e-6
F_TOL = 1e-5
V_TOL = 1e-8


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _compare_full(sysd, kw, label, iters_slack=1):
    say(f"[parity] {label}: n_sites={len(sysd['pos'])}")
    s = System.from_dict(sysd)
    op = oracle_params(sysd, **kw)
    ctx = Context(s, op)
    rows = pol_rows(sysd)
    E0_o = permanent_field(s, op, ctx=ctx)
    rng = np.random.default_rng(17)
    pvec = rng.normal(size=(len(rows), 3)) * 0.1
    Tp_o = apply_T(s, op, pvec, ctx=ctx)
    ref = oracle.evaluate(s, op)

    eng = engine_for(sysd, gpu_params(sysd, **kw))
    E0_g = eng.permanent_field().cpu().numpy()
    assert rel_err(E0_g[rows], E0_o) < V_TOL, rel_err(E0_g[rows], E0_o)
    nonpol = np.setdiff1d(np.arange(len(sysd["pos"])), rows)
    assert np.all(E0_g[nonpol] == 0.0)
    pfull = np.zeros((len(sysd["pos"]), 3))
    pfull[rows] = pvec
    Tp_g = eng.apply_T(torch.as_tensor(pfull, device="cuda")).cpu().numpy()
    assert rel_err(Tp_g[rows], Tp_o) < V_TOL, rel_err(Tp_g[rows], Tp_o)
    mu_g, it, rms = eng.solve()
    mu_g = mu_g.cpu().numpy()
    assert rms <= kw.get("tol", 1e-10)
    assert rel_err(mu_g[rows], ref["mu"]) < 1e-7, rel_err(mu_g[rows], ref["mu"])
    assert abs(it - ref["iters"]) <= iters_slack, (it, ref["iters"])
    e_pol, e_elec, F = eng.energy_forces()
    F = F.cpu().numpy()
    st = eng.stats()
    say(f"  E_pol gpu {e_pol:.12g} oracle {ref['E_pol']:.12g}; E_elec gpu {e_elec:.12g} "
        f"oracle {ref['E_elec']:.12g}; F rms rel {rms_rel(F, ref['forces']):.3e}; "
        f"iters {it}/{ref['iters']}")
    assert abs(e_pol - ref["E_pol"]) <= E_TOL * abs(ref["E_pol"]) + 1e-12
    assert abs(e_elec - ref["E_elec"]) <= E_TOL * abs(ref["E_elec"]) + 1e-12
    assert abs(st["e_pol_variational"] - ref["E_pol_var"]) <= E_TOL * abs(ref["E_pol"]) + 1e-12
    assert rms_rel(F, ref["forces"]) <= F_TOL
    eng.close()


@pytest.mark.parametrize("nw,seed", [(1, 0), (2, 1), (9, 2), (33, 3), (64, 4)])
def test_cluster_parity(nw, seed):
    _compare_full(water_cluster(nw, seed), dict(tol=1e-10), f"cluster{nw}")


def test_small_box_parity():
    # 27 waters, 9.5 A box: every site sees most of the box; ragged PME grid 24
    _compare_full(water_box(27, 9.5, 3), dict(beta=0.45, cutoff=4.5, grid=24, tol=1e-10),
                  "box27")


def test_orthorhombic_box_parity():
    # 120 waters in an 18.6 x 15.5 x 12.4 A box: unequal sides, a different
    # grid size per axis (non-square FFT planes), and cell counts 8 x 6 x 5
    # (the shifted-stencil list builder)
    d = water_box_ortho((6, 5, 4), (3.1, 3.1, 3.1), 1)
    _compare_full(d, dict(beta=0.45, cutoff=4.5, grid=(36, 30, 24), tol=1e-10), "ortho120")


def test_small_box_other_orders():
    for order, grid in ((4, 20), (6, 30)):
        _compare_full(water_box(27, 9.5, 5), dict(beta=0.45, cutoff=4.5, grid=grid, order=order,
                                                  tol=1e-10), f"box27-order{order}")


def test_multipass_fft_matches_plane_fft(monkeypatch):
    """The convolution runs as whole z-planes in LDS when a plane fits and as
    five line passes otherwise; both give the same field, T p, dipoles and
    forces (and the five-pass path alone meets the oracle)."""
    d = water_box(27, 9.5, 7)
    kw = dict(beta=0.45, cutoff=4.5, grid=24, tol=1e-10)
    res = {}
    for planes in ("1", "0"):
        monkeypatch.setenv("SIBFA_FFT_PLANES", planes)
        eng = engine_for(d, gpu_params(d, **kw))
        E0 = eng.permanent_field().cpu().numpy()
        mu, it, _ = eng.solve()
        ep, ee, F = eng.energy_forces()
        res[planes] = (E0, mu.cpu().numpy(), ep, ee, F.cpu().numpy())
        eng.close()
    a, b = res["1"], res["0"]
    assert rel_err(a[0], b[0]) < 1e-12 and rel_err(a[1], b[1]) < 1e-10
    assert a[2] == pytest.approx(b[2], rel=1e-11) and a[3] == pytest.approx(b[3], rel=1e-12)
    assert rms_rel(a[4], b[4]) < 1e-11
    monkeypatch.setenv("SIBFA_FFT_PLANES", "0")
    _compare_full(d, kw, "box27-multipass")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_one_stream_matches_two(monkeypatch, precision):
    """With the second stream switched off (SIBFA_PME_OVERLAP=0) every step
    runs in order on one stream: the PME brick lists and the permanent
    reciprocal potential after the neighbour lists instead of beside them,
    the real-space matvec after the reciprocal chain.  The kernels and their
    summation orders are the same, so the results are bit-identical."""
    say(f"[streams] box1024 {precision}")
    d, prm = config_system("box1024")
    kw = dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"], tol=prm["tol"],
              precision=precision, precond="molblock")
    res = {}
    for overlap in ("1", "0"):
        monkeypatch.setenv("SIBFA_PME_OVERLAP", overlap)
        eng = engine_for(d, gpu_params(d, **kw))
        mu, it, rms = eng.solve()
        ep, ee, F = eng.energy_forces()
        res[overlap] = (mu.cpu().numpy(), it, rms, ep, ee, F.cpu().numpy())
        eng.close()
    a, b = res["1"], res["0"]
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and a[2] == b[2]
    assert a[3] == b[3] and a[4] == b[4] and np.array_equal(a[5], b[5])


@pytest.mark.parametrize("scale", [0.05, 3.0])
def test_damping_split_extremes(scale):
    """The all-pairs rows are split at the radius beyond which no
    polarizable pair is Thole-damped (x >= 50), set from the largest mean
    polarizability.  Small polarizabilities put that radius below most pair
    distances (nearly every pair far), large ones beyond the cutoff (every
    pair near); both must still meet the oracle."""
    d = water_box(27, 9.5, 11)
    d = dict(d, alpha=d["alpha"] * scale)
    _compare_full(d, dict(beta=0.45, cutoff=4.5, grid=24, tol=1e-10), f"box27-alpha*{scale}")


@pytest.mark.slow
def test_box216_parity():
    d, prm = config_system("box216")
    _compare_full(d, dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"], tol=1e-10),
                  "box216")


def _kdtree_counts(sysd, cutoff):
    """Intermolecular sites within the cutoff of each site (minimum image),
    from a periodic k-d tree: every site within the cutoff (the site itself
    included) less the sites of its own molecule, all of which lie within
    the cutoff (checked)."""
    box = np.asarray(sysd["box"], float)
    pos = np.mod(sysd["pos"], box)
    mol = np.asarray(sysd["mol"])
    order = np.argsort(mol, kind="stable")
    ms = mol[order]
    starts = np.flatnonzero(np.r_[True, ms[1:] != ms[:-1]])
    sizes = np.diff(np.r_[starts, len(ms)])
    for size in np.unique(sizes):
        grp = order[starts[sizes == size][:, None] + np.arange(size)[None, :]]
        d = pos[grp][:, :, None, :] - pos[grp][:, None, :, :]
        d -= box * np.round(d / box)
        assert np.linalg.norm(d, axis=-1).max() < cutoff
    tree = cKDTree(pos, boxsize=box)
    within = tree.query_ball_point(pos, cutoff, return_length=True)
    own = np.bincount(mol, minlength=mol.max() + 1)[mol]
    return within.astype(np.int64) - own


def test_kdtree_counts_match_pair_enumeration():
    """The count helper against an explicit pair enumeration (small box)."""
    d = water_box(27, 9.5, 3)
    pos = np.mod(d["pos"], d["box"])
    tree = cKDTree(pos, boxsize=d["box"])
    pairs = tree.query_pairs(4.5, output_type="ndarray")
    mol = d["mol"]
    inter = pairs[mol[pairs[:, 0]] != mol[pairs[:, 1]]]
    cnt = np.zeros(len(pos), np.int64)
    np.add.at(cnt, inter[:, 0], 1)
    np.add.at(cnt, inter[:, 1], 1)
    assert np.array_equal(_kdtree_counts(d, 4.5), cnt)


@pytest.mark.parametrize("name", ["box216", "box4096",
                                  pytest.param("box32000", marks=pytest.mark.slow)])
def test_neighbor_counts_exact(name):
    say(f"[nlist] {name}")
    d, prm = config_system(name)
    eng = engine_for(d, gpu_params(d, beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"]))
    got = eng.neighbor_counts().cpu().numpy()
    ref = _kdtree_counts(d, prm["cutoff"])
    assert np.array_equal(got, ref)
    eng.close()


def test_neighbor_lists_grow_on_overflow():
    """A dense pocket (the waters within 12 A of the box centre pulled in by
    half) gives its sites about twice the neighbours the density estimate
    sizes the lists for, and more sites per cell than one pass of the
    builder holds: the builder must see the overflow in its count maxima,
    grow the lists and rebuild.  Counts stay exact, max_neighbors is their
    maximum, and the lists' contents give the oracle's permanent-field and
    T rows at sites of the pocket."""
    say("[nlist] dense pocket, box4096")
    d, prm = config_system("box4096")
    d = dict(d)
    pos = np.array(d["pos"], float)
    box = np.asarray(d["box"], float)
    mol = np.asarray(d["mol"])
    c = 0.5 * box
    first = np.flatnonzero(np.r_[True, mol[1:] != mol[:-1]])
    near = np.zeros(len(pos), bool)
    for m0, m1 in zip(first, np.r_[first[1:], len(pos)]):
        if np.linalg.norm(pos[m0] - c) < 12.0:
            near[m0:m1] = True
    pos[near] = c + 0.5 * (pos[near] - c)
    d["pos"] = pos
    eng = engine_for(d, gpu_params(d, beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"]))
    got = eng.neighbor_counts().cpu().numpy()
    ref = _kdtree_counts(d, prm["cutoff"])
    estimate = 1.3 * len(pos) / np.prod(box) * 4.0 / 3.0 * np.pi * prm["cutoff"] ** 3 + 64
    assert ref.max() > estimate            # the pocket overflows the first lists
    assert np.array_equal(got, ref)
    assert eng.stats()["max_neighbors"] == ref.max()
    # list contents: permanent-field rows and rows of T at polarizable sites
    # of the pocket against the oracle's sampled rows (FP64 both sides)
    E0_g = eng.permanent_field().cpu().numpy()
    rng = np.random.default_rng(5)
    mu = np.zeros_like(pos)
    s = System.from_dict(d)
    mu[s.pol] = rng.normal(scale=0.05, size=(len(s.pol), 3))
    Tmu_g = eng.apply_T(torch.as_tensor(mu, device="cuda")).cpu().numpy()
    eng.close()
    kw = dict(beta=prm["beta"], cutoff=prm["cutoff"], grid=prm["grid"])
    op = oracle_params(d, **kw)
    samp = np.sort(rng.choice(s.pol[near[s.pol]], 16, replace=False))
    ctx = Context(s, op, subset=samp)
    assert rel_err(E0_g[samp], permanent_field(s, op, ctx=ctx, sites=samp)) < 1e-8
    assert rel_err(Tmu_g[samp], apply_T(s, op, mu[s.pol], ctx=ctx, sites=samp)) < 1e-8


def test_polarizable_count_changes_on_a_live_context():
    """set_polarizabilities may change which sites are polarizable: the
    polarizable-pair lists (whose row counts follow that number) are
    re-sized, and the results equal those of a fresh context."""
    d = water_box(27, 9.5, 13)
    kw = dict(beta=0.45, cutoff=4.5, grid=24, tol=1e-10)
    few = d["alpha"].copy()
    few[np.arange(len(few)) % 5 != 0] = 0.0      # only the O sites
    iso = np.zeros_like(d["alpha"])
    iso[:, [0, 3, 5]] = 0.6                        # every site, isotropic
    eng = engine_for(dict(d, alpha=few), gpu_params(d, **kw))
    eng.solve()
    for alpha in (iso, few, iso):
        eng.set_polarizabilities(torch.as_tensor(alpha, device="cuda"))
        mu, it, _ = eng.solve()
        ep, ee, F = eng.energy_forces()
        ref = engine_for(dict(d, alpha=alpha), gpu_params(d, **kw))
        mu_r, it_r, _ = ref.solve()
        ep_r, ee_r, F_r = ref.energy_forces()
        say(f"  npol {int(np.count_nonzero(alpha.any(1)))}: iters {it}/{it_r}")
        assert it == it_r
        assert torch.equal(mu, mu_r)
        assert ep == ep_r and ee == ee_r
        assert torch.equal(F, F_r)
        ref.close()
    eng.close()
