"""Pins of the oracle's virial W_ab = -dE_tot/d eps_ab (strain r -> (1 + eps) r
of every site and of the cell; multipoles, polarizabilities and the induced
dipoles fixed in the global frame).

V1  Cluster, direct sums: every component against central differences of the
    energy at fixed mu under strained positions.
V2  Brute-force Ewald (image sums and the k-sum), every component: the
    off-diagonal strains make the cell triclinic, which the brute-force
    sums take as lattice vectors.  Against central differences at fixed mu,
    and, for two components, of the re-solved total energy (mu is stationary,
    so the two derivatives agree).
V3  SPME: the diagonal components against central differences of the SPME
    energy (a diagonal strain keeps the cell orthorhombic); every component
    against the brute-force Ewald virial at order 8 on a fine grid.
V4  Pure dilation of a cluster of charges only: the virial is then the
    Coulomb energy itself (tr W = E for a homogeneous function of degree -1
    in the separations), a closed form independent of the code above.
"""
import numpy as np
import pytest

import oracle
from oracle.model import (System, Params, Context, permanent_field, apply_T,
                          electrostatic_energy, virial)
from oracle.units import COULOMB
from synth import water_cluster, water_box


def _strained(d, eps):
    F = np.eye(3) + eps
    out = dict(d, pos=d["pos"] @ F.T)
    if d.get("box") is not None:
        box = np.asarray(d["box"], float)
        H = np.diag(box) if box.ndim == 1 else box
        H2 = H @ F.T
        off = H2 - np.diag(np.diag(H2))
        out["box"] = np.diag(H2).copy() if np.all(off == 0.0) else H2
    return out


def _e_fixed(d, prm, mu):
    """E_elec + f (1/2 mu.T mu - mu.E), the functional of Eq. 17 at fixed mu."""
    s = System.from_dict(d)
    c = Context(s, prm)
    E0 = permanent_field(s, prm, ctx=c)
    Tmu = apply_T(s, prm, mu, ctx=c)
    return electrostatic_energy(s, prm, ctx=c) + COULOMB * (0.5 * np.sum(mu * Tmu)
                                                            - np.sum(mu * E0))


def _e_solved(d, prm):
    o = oracle.evaluate(System.from_dict(d), prm, forces=False)
    return o["E_pol"] + o["E_elec"]


def _fd(d, prm, a, b, fn, h=1e-5):
    e = np.zeros((3, 3))
    e[a, b] = h
    ep = fn(_strained(d, e))
    em = fn(_strained(d, -e))
    return -(ep - em) / (2 * h)


def _check_all(d, prm, comps, rtol, solved=()):
    s = System.from_dict(d)
    o = oracle.evaluate(s, prm, forces=False, with_virial=True)
    W, mu = o["virial"], o["mu"]
    scale = np.abs(W).max()
    for (a, b) in comps:
        fd = _fd(d, prm, a, b, lambda dd: _e_fixed(dd, prm, mu))
        assert abs(fd - W[a, b]) <= rtol * scale, (a, b, fd, W[a, b])
    for (a, b) in solved:
        fd = _fd(d, prm, a, b, lambda dd: _e_solved(dd, prm))
        assert abs(fd - W[a, b]) <= 10 * rtol * scale, (a, b, fd, W[a, b])
    return W


ALL = [(a, b) for a in range(3) for b in range(3)]


def test_v1_cluster_fd():
    d = water_cluster(4, 3)
    W = _check_all(d, Params(method="direct", tol=1e-12), ALL, 1e-7)
    # multipoles fixed in the global frame: W is not symmetric in general
    assert np.abs(W - W.T).max() > 1e-6 * np.abs(W).max()


def test_v2_ewald_triclinic_fd():
    d = water_box(4, 6.5, 11)
    prm = Params(method="ewald", beta=0.55, realspace="images", rmax=11.0, tol=1e-12)
    _check_all(d, prm, ALL, 1e-7, solved=[(0, 0), (1, 2)])


def test_v2_triclinic_lattice_sums_are_invariant():
    """The brute-force sums on a general lattice: a cubic cell described by
    rotated lattice vectors, with every site and multipole rotated the same
    way, gives the same energy (pins the lattice handling the strain
    derivatives above rely on)."""
    d = water_box(4, 6.5, 11)
    prm = Params(method="ewald", beta=0.55, realspace="images", rmax=11.0, tol=1e-12)
    rng = np.random.default_rng(4)
    q4 = rng.normal(size=4)
    q4 /= np.linalg.norm(q4)
    w, x, y, z = q4
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                  [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                  [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])

    def rot6(t6):
        xx, xy, xz, yy, yz, zz = t6.T
        T = np.stack([np.stack([xx, xy, xz], -1), np.stack([xy, yy, yz], -1),
                      np.stack([xz, yz, zz], -1)], -2)
        T = np.einsum("ab,nbc,dc->nad", R, T, R)
        return np.stack([T[:, 0, 0], T[:, 0, 1], T[:, 0, 2], T[:, 1, 1], T[:, 1, 2],
                         T[:, 2, 2]], 1)

    d2 = dict(d, pos=d["pos"] @ R.T, dip=d["dip"] @ R.T, quad=rot6(d["quad"]),
              alpha=rot6(d["alpha"]), box=np.diag(d["box"]) @ R.T)
    e1 = _e_solved(d, prm)
    e2 = _e_solved(d2, prm)
    assert abs(e1 - e2) <= 1e-9 * abs(e1)


def _cutoff_clear(d, cutoff, margin):
    L = np.asarray(d["box"], float)
    for i in range(len(d["pos"])):
        dd = d["pos"] - d["pos"][i]
        dd -= L * np.round(dd / L)
        if np.any(np.abs(np.linalg.norm(dd, axis=1) - cutoff) < margin):
            return False
    return True


def test_v3_spme_diagonal_fd():
    # no pair within 2e-3 A of the cutoff: a 1e-5 strain moves none across it
    d = water_box(8, 8.0, 12)
    assert _cutoff_clear(d, 3.7, 2e-3)
    prm = Params(method="spme", beta=0.5, cutoff=3.7, grid=(12, 12, 12), order=5, tol=1e-12)
    _check_all(d, prm, [(0, 0), (1, 1), (2, 2)], 1e-7, solved=[(2, 2)])


def test_v3_spme_matches_ewald_virial_at_fine_grid():
    d = water_box(27, 9.5, 3)
    base = dict(beta=0.45, cutoff=4.5, tol=1e-12)
    s = System.from_dict(d)
    we = oracle.evaluate(s, Params(method="ewald", realspace="minimage", **base),
                         forces=False, with_virial=True)["virial"]
    ws = oracle.evaluate(s, Params(method="spme", grid=(48, 48, 48), order=8, **base),
                         forces=False, with_virial=True)["virial"]
    assert np.abs(ws - we).max() <= 1e-7 * np.abs(we).max(), np.abs(ws - we).max()


def test_v4_charge_cluster_dilation():
    rng = np.random.default_rng(5)
    n = 7
    pos = rng.uniform(-3, 3, size=(n, 3))
    q = rng.uniform(-1, 1, size=n)
    s = System(pos=pos, mol=np.arange(n), q=q, dip=np.zeros((n, 3)), quad=np.zeros((n, 6)),
               alpha=np.zeros((n, 6)))
    prm = Params(method="direct")
    W = virial(s, prm, np.zeros((0, 3)))
    e = 0.0
    for i in range(n):
        for j in range(i + 1, n):
            e += q[i] * q[j] / np.linalg.norm(pos[i] - pos[j])
    assert np.trace(W) == pytest.approx(COULOMB * e, rel=1e-12)
    # a central pair sum: W is symmetric
    assert np.abs(W - W.T).max() <= 1e-12 * np.abs(W).max()


@pytest.mark.parametrize("plant", ["no_site_terms", "no_inverse_m2", "transposed"])
def test_virial_pins_see_planted_mistakes(plant, monkeypatch):
    """Mistakes planted in the oracle's reciprocal virial -- the amplitude
    (site) terms dropped, the 1/m^2 part of the kernel derivative dropped,
    or the tensor transposed -- each fail the brute-force Ewald FD check."""
    from oracle import recip
    if plant == "no_site_terms":
        monkeypatch.setattr(recip, "_site_virial", lambda mult, derivs: np.zeros((3, 3)))
    elif plant == "no_inverse_m2":
        def planted(pos, box, beta, mult, chunk=2000):
            V = recip.cell_volume(box)
            m, m2 = recip.kvectors(box, beta)
            q, d, th = mult
            energy, derivs = recip.ewald_recip(pos, box, beta, mult, pos, 2, chunk)
            W = energy * np.eye(3) + recip._site_virial(mult, derivs)
            C = np.exp(-np.pi ** 2 * m2 / beta ** 2) / m2 / (np.pi * V)
            S = recip.structure_factor(m, pos, q, d, th)
            W -= np.einsum("m,ma,mb->ab", C * (np.pi ** 2 / beta ** 2) * np.abs(S) ** 2, m, m)
            return energy, W
        monkeypatch.setattr(recip, "ewald_recip_virial", planted)
    else:
        orig = recip.ewald_recip_virial
        monkeypatch.setattr(recip, "ewald_recip_virial",
                            lambda *a, **k: (orig(*a, **k)[0], orig(*a, **k)[1].T))
    d = water_box(4, 6.5, 11)
    prm = Params(method="ewald", beta=0.55, realspace="images", rmax=11.0, tol=1e-12)
    with pytest.raises(AssertionError):
        _check_all(d, prm, ALL, 1e-7)
