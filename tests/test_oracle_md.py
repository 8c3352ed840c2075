"""Pins of the oracle's Beeman dynamics (oracle/md.py).

M1  The generic integrator is exact for a constant acceleration (a
    parabola) and follows a harmonic oscillator's cosine with an error that
    falls as dt^2.
M2  Bond and repulsion forces equal differences of their energies (one
    repulsive pair also by hand); atom forces with the
    virtual-site forces handed to the parents equal differences of the total
    energy when moving an atom also moves its midpoints; a free cluster has
    zero net force, and with local frames zero net torque.
M3  Along a full-model trajectory the total energy (kinetic + E_pol +
    E_elec + bond + repulsion) fluctuates by an amount that falls as dt^2.
"""
import numpy as np
import pytest

from oracle import md
from oracle.model import Params
from synth import water_cluster, water_box, water_md, water_frames


def test_m1_constant_acceleration_is_exact():
    rng = np.random.default_rng(1)
    x0, v0, a = rng.normal(size=(3, 4, 3))
    out = md.beeman(lambda x: (a.copy(), None), x0, v0, 0.7, 5, np.arange(4))
    for s, (x, v, _) in enumerate(out, 1):
        t = 0.7 * s
        assert np.allclose(x, x0 + v0 * t + 0.5 * a * t * t, atol=1e-12)
        assert np.allclose(v, v0 + a * t, atol=1e-12)


def test_m1_harmonic_oscillator_second_order():
    errs = []
    for dt in (0.1, 0.05):
        n = int(round(3.0 / dt))
        out = md.beeman(lambda x: (-x, None), np.array([[1.0, 0, 0]]), np.zeros((1, 3)), dt, n,
                        np.arange(1))
        errs.append(abs(out[-1][0][0, 0] - np.cos(3.0)))
    assert errs[0] < 1e-2 and 3.5 < errs[0] / errs[1] < 4.5, errs


def test_m2_bond_forces():
    rng = np.random.default_rng(2)
    pos = rng.normal(size=(4, 3)) * 1.5
    bonds = np.array([[0, 1], [1, 2], [0, 3]])
    k = np.array([300.0, 120.0, 80.0])
    r0 = np.array([1.0, 1.2, 0.9])
    _, F = md.bond_energy_forces(pos, bonds, k, r0, None)
    h = 1e-6
    for i in range(4):
        for a in range(3):
            p = pos.copy()
            p[i, a] += h
            ep = md.bond_energy_forces(p, bonds, k, r0, None)[0]
            p[i, a] -= 2 * h
            em = md.bond_energy_forces(p, bonds, k, r0, None)[0]
            assert abs(-(ep - em) / (2 * h) - F[i, a]) < 1e-6


def test_m2_repulsion_forces():
    """Stand-in repulsion: forces are differences of its energy; pairs in one
    molecule, pairs with a zero radius and pairs beyond the cutoff (minimum
    image) add nothing."""
    rng = np.random.default_rng(4)
    pos = rng.uniform(0, 6.0, size=(9, 3))
    mol = np.array([0, 0, 0, 1, 1, 1, 2, 2, 2])
    rho = np.array([1.6, 0.3, 0.0] * 3)
    box = np.array([6.0, 6.0, 6.0])
    e, F = md.repulsion_energy_forces(pos, mol, rho, 0.5, box, 2.9)
    assert np.all(F[2::3] == 0.0)
    h = 1e-6
    for i in range(9):
        for a in range(3):
            p = pos.copy()
            p[i, a] += h
            ep = md.repulsion_energy_forces(p, mol, rho, 0.5, box, 2.9)[0]
            p[i, a] -= 2 * h
            em = md.repulsion_energy_forces(p, mol, rho, 0.5, box, 2.9)[0]
            assert abs(-(ep - em) / (2 * h) - F[i, a]) < 1e-6 * max(1.0, np.abs(F).max())
    # one pair by hand
    two = np.array([[0.0, 0, 0], [2.5, 0, 0]])
    e2, F2 = md.repulsion_energy_forces(two, np.array([0, 1]), np.array([1.6, 1.6]), 0.5, None,
                                        np.inf)
    assert e2 == pytest.approx(0.5 * (3.2 / 2.5) ** 12)
    assert F2[1, 0] == pytest.approx(12 * e2 / 2.5)


def test_m2_atom_forces_with_virtual_sites():
    d = water_cluster(2, 3)
    m = water_md(d, 0)
    prm = Params(method="direct", tol=1e-12)
    args = (m["masses"], m["vsites"], m["bonds"], m["bond_k"], m["bond_r0"] * 1.02)
    pos = md.place_vsites(d["pos"], m["vsites"], None)
    F, ep, ee, eb, er = md.atom_forces(d, prm, pos, *args, rho=m["rep_radius"], eps=0.5)
    assert np.all(F[m["masses"] == 0] == 0.0)
    scale = np.abs(F).max()
    assert np.abs(F.sum(0)).max() < 1e-9 * scale
    # global-frame multipoles do not turn with the molecules, so only with
    # local frames do the torques vanish too
    Ff = md.atom_forces(d, prm, pos, *args, frames=water_frames(d), rho=m["rep_radius"],
                        eps=0.5)[0]
    assert np.abs(np.cross(pos, Ff).sum(0)).max() < 1e-8 * scale * np.abs(pos).max()
    assert np.abs(np.cross(pos, F).sum(0)).max() > 1e-3 * scale

    def etot(p):
        q = md.place_vsites(p, m["vsites"], None)
        _, a, b, c, r = md.atom_forces(d, prm, q, *args, rho=m["rep_radius"], eps=0.5)
        return a + b + c + r

    h = 1e-5
    for i, a in ((0, 0), (1, 2), (2, 1), (5, 1), (6, 0)):
        p = pos.copy()
        p[i, a] += h
        e1 = etot(p)
        p[i, a] -= 2 * h
        e2 = etot(p)
        assert abs(-(e1 - e2) / (2 * h) - F[i, a]) < 1e-6 * scale, (i, a)


def test_m3_energy_conservation_is_second_order():
    d = water_cluster(3, 2)
    m = water_md(d, 0)
    prm = Params(method="direct", tol=1e-11)
    spread = []
    for dt in (0.5, 0.25):
        out = md.run(d, prm, m["masses"], m["vsites"], m["bonds"], m["bond_k"], m["bond_r0"],
                     m["vel"], dt, int(round(10 / dt)))
        et = np.array([sum(o[2:7]) for o in out])
        spread.append(et.max() - et.min())
    assert spread[0] < 0.05 and 3.0 < spread[0] / spread[1] < 5.5, spread


def test_m3_periodic_box_runs():
    d = water_box(8, 8.0, 12)
    m = water_md(d, 1)
    prm = Params(method="spme", beta=0.5, cutoff=3.7, grid=(12, 12, 12), order=5, tol=1e-10)
    out = md.run(d, prm, m["masses"], m["vsites"], m["bonds"], m["bond_k"], m["bond_r0"],
                 m["vel"], 0.5, 6, rho=m["rep_radius"], eps=m["rep_eps"])
    et = np.array([sum(o[2:7]) for o in out])
    assert np.isfinite(et).all() and et.max() - et.min() < 0.05 * abs(out[0][6])
