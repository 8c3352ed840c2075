"""Pins of the oracle's local-frame multipoles and their forces.

L1  The frame is orthonormal and right-handed, its z axis bisects the two
    bonds and its x axis lies in their plane; its analytic derivative equals
    central differences of the frame.
L2  The multipole gradients G^d, G^Theta, G^alpha equal central differences
    of the converged energy with respect to one global dipole, quadrupole
    and polarizability component (stationarity makes the fixed-mu
    derivative the full one).
L3  The total forces with frames equal central differences of the energy
    as a function of site positions (multipoles re-rotated at every
    displacement): cluster, brute-force Ewald box, SPME box.
L4  With frames a free cluster is isotropic: the forces sum to zero and so
    do the torques sum r x F; a rigid rotation leaves the energy unchanged.
L5  The virial with frames equals central differences of the re-solved
    energy under a homogeneous strain of sites and cell, the local
    multipoles following their strained frames (cluster: all components;
    brute-force Ewald: diagonal and off-diagonal; SPME: diagonal).
"""
import numpy as np
import pytest

import oracle
from oracle import frames as fr
from oracle.model import System, Params
from synth import water_cluster, water_box, water_frames


def _local(d):
    return System.from_dict(d), water_frames(d)


def test_l1_frame_and_its_derivative():
    rng = np.random.default_rng(1)
    ro, ra, rb = rng.normal(size=(3, 6, 3))
    R = fr.frame(ro, ra, rb)
    assert np.allclose(np.einsum("nab,nac->nbc", R, R), np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(R), 1.0)
    u = (ra - ro) / np.linalg.norm(ra - ro, axis=1, keepdims=True)
    v = (rb - ro) / np.linalg.norm(rb - ro, axis=1, keepdims=True)
    ez = R[:, :, 2]
    assert np.allclose(np.sum(ez * u, 1), np.sum(ez * v, 1))          # bisector
    assert np.allclose(np.sum(np.cross(u, v) * R[:, :, 0], 1), 0.0, atol=1e-14)  # in plane
    assert np.all(np.sum(R[:, :, 0] * u, 1) > 0)                       # towards a
    dR = fr.frame_derivatives(ro, ra, rb)
    h = 1e-6
    for k in range(3):
        for c in range(3):
            pts = [ro.copy(), ra.copy(), rb.copy()]
            pts[k][:, c] += h
            Rp = fr.frame(*pts)
            pts[k][:, c] -= 2 * h
            Rm = fr.frame(*pts)
            assert np.abs((Rp - Rm) / (2 * h) - dR[:, k, c]).max() < 1e-8


def _energy_global(s, prm):
    o = oracle.evaluate(s, prm, forces=False)
    return o["E_pol"] + o["E_elec"]


@pytest.mark.parametrize("method", ["direct", "ewald"])
def test_l2_multipole_gradients(method):
    if method == "direct":
        d, prm = water_cluster(3, 4), Params(method="direct", tol=1e-12)
    else:
        d = water_box(4, 6.5, 11)
        prm = Params(method="ewald", beta=0.55, realspace="images", rmax=11.0, tol=1e-12)
    s = System.from_dict(d)
    o = oracle.evaluate(s, prm, forces=False)
    Gd, GT, Ga = fr.multipole_gradients(s, prm, o["mu"])
    h = 1e-5
    for i, a in ((0, 2), (3, 0), (7, 1)):
        for key, grad, comp in (("dip", Gd, (i, a)), ("quad", GT, None), ("alpha", Ga, None)):
            arr = getattr(s, key)
            # alpha along off-diagonal (trace-free) directions only: a change
            # of tr(alpha) also changes the Thole widths, which a rotation
            # never does and G^alpha leaves out
            k6 = a if key == "dip" else ((0, 3, 5, 1, 2, 4)[a + 3 * (i % 2)] if key == "quad"
                                         else (1, 2, 4)[a])
            if key == "alpha" and not np.any(arr[i] != 0):
                continue
            vals = []
            for sign in (1, -1):
                arr2 = arr.copy()
                arr2[i, k6] += sign * h
                if key == "quad" and k6 in (0, 3):      # keep it traceless
                    arr2[i, 5] -= sign * h
                vals.append(_energy_global(System(**{**s.__dict__, key: arr2}), prm))
            fd = (vals[0] - vals[1]) / (2 * h)
            if key == "dip":
                an = grad[i, a]
            else:
                M = np.zeros((3, 3))
                pairs6 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
                p, q = pairs6[k6]
                M[p, q] = M[q, p] = 1.0
                if key == "quad" and k6 in (0, 3):
                    M[2, 2] -= 1.0
                an = float(np.sum(grad[i] * M))
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (key, i, k6, fd, an)


def _fd_frames(d, prm, sites, h=1e-4, rtol=1e-6):
    s, f = _local(d)
    o = fr.evaluate(s, f, prm)
    F = o["forces"]

    def etot(pos):
        g = fr.to_global(System(**{**s.__dict__, "pos": pos}), f)
        return _energy_global(g, prm)

    scale = np.abs(F).max()
    for (i, a) in sites:
        p = s.pos.copy()
        p[i, a] += h
        ep = etot(p)
        p[i, a] -= 2 * h
        em = etot(p)
        fd = -(ep - em) / (2 * h)
        assert abs(fd - F[i, a]) <= rtol * scale, (i, a, fd, F[i, a])
    return o


def test_l3_fd_cluster():
    # frame sites (O 0, H1 1, H2 2) and a bond barycentre (3) of water 0,
    # and the O of water 2
    _fd_frames(water_cluster(3, 2), Params(method="direct", tol=1e-12),
               [(0, 0), (1, 1), (2, 2), (3, 0), (10, 1)])


def test_l3_fd_ewald():
    _fd_frames(water_box(4, 6.5, 11), Params(method="ewald", beta=0.55, realspace="images",
                                              rmax=11.0, tol=1e-12),
               [(0, 2), (1, 0), (7, 1), (13, 2)])


def test_l3_fd_spme():
    d = water_box(8, 8.0, 12)
    prm = Params(method="spme", beta=0.5, cutoff=3.7, grid=(12, 12, 12), order=5, tol=1e-12)
    _fd_frames(d, prm, [(0, 0), (1, 2), (6, 1), (12, 0)])


def test_l4_free_cluster_is_isotropic():
    d = water_cluster(4, 6)
    s, f = _local(d)
    prm = Params(method="direct", tol=1e-12)
    o = fr.evaluate(s, f, prm)
    F = o["forces"]
    scale = np.abs(F).max()
    assert np.abs(F.sum(0)).max() < 1e-10 * scale
    torque = np.cross(s.pos, F).sum(0)
    assert np.abs(torque).max() < 1e-9 * scale * np.abs(s.pos).max()
    # without the rotation terms the torques do not vanish
    F0 = F - fr.frame_forces(s, f, prm, o["mu"])
    assert np.abs(np.cross(s.pos, F0).sum(0)).max() > 1e-4 * scale
    th = 0.7
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    s2 = System(**{**s.__dict__, "pos": s.pos @ Rz.T})
    o2 = fr.evaluate(s2, f, prm)
    assert o2["E_pol"] + o2["E_elec"] == pytest.approx(o["E_pol"] + o["E_elec"], rel=1e-12)


@pytest.mark.parametrize("drop", [0, 1, 2])
def test_frame_pins_see_a_dropped_term(drop, monkeypatch):
    """Dropping the dipole, quadrupole or polarizability term of the
    rotation derivative (planted in the oracle) fails the FD check."""
    orig = fr.multipole_gradients

    def planted(*a, **k):
        g = list(orig(*a, **k))
        g[drop] = np.zeros_like(g[drop])
        return tuple(g)

    monkeypatch.setattr(fr, "multipole_gradients", planted)
    with pytest.raises(AssertionError):
        _fd_frames(water_cluster(3, 2), Params(method="direct", tol=1e-12),
                   [(0, 0), (1, 1), (2, 2), (0, 2), (1, 0)])


def _strain(d, eps):
    F = np.eye(3) + eps
    out = dict(d, pos=d["pos"] @ F.T)
    if d.get("box") is not None:
        H2 = np.diag(np.asarray(d["box"], float)) @ F.T
        off = H2 - np.diag(np.diag(H2))
        out["box"] = np.diag(H2).copy() if np.all(off == 0.0) else H2
    return out


def _fd_virial(d, prm, comps, h=1e-5, rtol=1e-6):
    """W_ab = -dE/d eps_ab of the re-solved energy with the local multipoles
    re-rotated in the strained frames, against frames.virial."""
    s, f = _local(d)
    o = fr.evaluate(s, f, prm)
    W = fr.virial(s, f, prm, o["mu"])
    scale = np.abs(W).max()

    def etot(dd):
        r = fr.evaluate(System.from_dict(dd), f, prm)
        return r["E_pol"] + r["E_elec"]

    for a, b in comps:
        e = np.zeros((3, 3))
        e[a, b] = h
        fd = -(etot(_strain(d, e)) - etot(_strain(d, -e))) / (2 * h)
        assert abs(fd - W[a, b]) <= rtol * scale, (a, b, fd, W[a, b])
    return W


def test_l5_virial_cluster():
    """Every component for a cluster; without the frame term the check
    fails (the frame term is not small)."""
    d = water_cluster(3, 2)
    prm = Params(method="direct", tol=1e-12)
    W = _fd_virial(d, prm, [(a, b) for a in range(3) for b in range(3)])
    s, f = _local(d)
    o = fr.evaluate(s, f, prm)
    W0 = oracle.model.virial(fr.to_global(s, f), prm, o["mu"])
    assert np.abs(W - W0).max() > 1e-3 * np.abs(W).max()


def test_l5_virial_ewald():
    d = water_box(4, 6.5, 11)
    prm = Params(method="ewald", beta=0.55, realspace="images", rmax=11.0, tol=1e-12)
    _fd_virial(d, prm, [(0, 0), (2, 2), (0, 1), (2, 1)])


def test_l5_virial_spme():
    d = water_box(8, 8.0, 12)
    prm = Params(method="spme", beta=0.5, cutoff=3.7, grid=(12, 12, 12), order=5, tol=1e-12)
    _fd_virial(d, prm, [(0, 0), (1, 1)])


def test_l5_virial_sees_a_wrong_frame_term(monkeypatch):
    """The frame term with its sign flipped (planted in the oracle) fails
    the strain-difference check."""
    orig = fr._frame_terms
    monkeypatch.setattr(fr, "_frame_terms", lambda *a, **k: -orig(*a, **k))
    d = water_cluster(3, 2)
    prm = Params(method="direct", tol=1e-12)
    with pytest.raises(AssertionError):
        _fd_virial(d, prm, [(0, 0), (1, 2), (2, 1)])


def test_sites_without_frame_keep_global_values():
    """Rows of -1 (no frame): those sites' values are used as given and add
    no rotation forces; the forces still match differences of the energy."""
    d = water_cluster(3, 2)
    s, f = _local(d)
    f = f.copy()
    f[5:10] = -1                      # water 1 without a frame
    prm = Params(method="direct", tol=1e-12)
    g = fr.to_global(s, f)
    assert np.array_equal(g.dip[5:10], s.dip[5:10]) and np.array_equal(g.alpha[5:10],
                                                                       s.alpha[5:10])
    o = fr.evaluate(s, f, prm)

    def etot(pos):
        return _energy_global(fr.to_global(System(**{**s.__dict__, "pos": pos}), f), prm)

    F = o["forces"]
    h = 1e-4
    for (i, a) in ((0, 0), (6, 1), (11, 2)):
        p = s.pos.copy()
        p[i, a] += h
        ep = etot(p)
        p[i, a] -= 2 * h
        fd = -(ep - etot(p)) / (2 * h)
        assert abs(fd - F[i, a]) <= 1e-6 * np.abs(F).max()
