"""Pins of the oracle's reduced charge transfer (oracle/ct.py).

C1  Potentials.  With charges and dipoles only, V at a lone pair and V_int
    at an acceptor atom equal the textbook sums q/r + d.R/r^3 over the
    other molecules (own molecule for V_int); with quadrupoles, minus the
    gradient of V (differences) equals the oracle's field, which is pinned
    separately.  Periodic: V at the lone pairs is independent of the Ewald
    beta (brute-force Ewald) and SPME on a fine grid reproduces it.
C2  Energy structure.  E_ct is invariant under rigid motions of a cluster,
    linear in the occupation, E_ct * dE is independent of ae (only dE
    contains it), vanishes when a1 and a2 are made equivalent (e1 = e2) and
    when eta grows large.
C3  Forces equal central differences of E_ct (cluster, brute-force Ewald,
    SPME), with the net force of a cluster zero; dropping the potential
    (w) forces or their reciprocal part (planted) fails.  The paper prints
    no charge-transfer value for a system these inputs can reproduce: the
    values themselves are parity unpinned.
C4  Local frames: with the dipoles and quadrupoles given in molecular
    frames, the forces (fixed-multipole part plus the rotation through the
    derivatives of E_ct with respect to the global multipoles) equal central
    differences of E_ct at the rotated multipoles (cluster, SPME); dropping
    the rotation part (planted) fails.
"""
import numpy as np
import pytest

from oracle import ct as oct_
from oracle.model import System, Params, Context
from oracle import realspace as rs
from oracle import frames as ofr
from synth import water_cluster, water_box, water_lone_pairs, water_ct, water_frames, CT_SITES


def _cluster(nw=3, seed=2):
    d = water_lone_pairs(water_cluster(nw, seed))
    return System.from_dict(d), water_ct(d), d


def test_c1_potentials_charges_and_dipoles():
    s, c, d = _cluster()
    s = System(**{**s.__dict__, "quad": np.zeros_like(s.quad)})
    V, Vint = oct_.potentials(s, Params(method="direct"))
    pos, q, dip, mol = s.pos, s.q, s.dip, s.mol
    for L in c["lp"][:, 0]:
        R = pos[L] - pos
        r = np.linalg.norm(R, axis=1)
        other = mol != mol[L]
        ref = np.sum(q[other] / r[other]) + np.sum(np.sum(dip[other] * R[other], 1) / r[other] ** 3)
        assert V[L] == pytest.approx(ref, rel=1e-12, abs=1e-14)
    for a in np.unique(c["acc"]):
        R = pos[a] - pos
        r = np.linalg.norm(R, axis=1)
        own = (mol == mol[a]) & (np.arange(len(pos)) != a)
        ref = np.sum(q[own] / r[own]) + np.sum(np.sum(dip[own] * R[own], 1) / r[own] ** 3)
        assert Vint[a] == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_c1_potential_gradient_is_the_field():
    s, c, d = _cluster()
    prm = Params(method="direct")
    ctx = Context(s, prm)
    E = rs.pair_sum(ctx.pairs, "MM", "bare", prm.beta, ctx.thole, (None, None, None),
                    (s.q, s.dip, s.th), "field", s.n)
    h = 1e-6
    for L in c["lp"][:3, 0]:
        for a in range(3):
            p = s.pos.copy()
            p[L, a] += h
            vp = oct_.potentials(System(**{**s.__dict__, "pos": p}), prm)[0][L]
            p[L, a] -= 2 * h
            vm = oct_.potentials(System(**{**s.__dict__, "pos": p}), prm)[0][L]
            assert -(vp - vm) / (2 * h) == pytest.approx(E[L, a], rel=1e-6, abs=1e-9)


def test_c1_periodic_potential_beta_invariant_and_spme():
    d = water_lone_pairs(water_box(4, 6.5, 11))
    s = System.from_dict(d)
    lps = water_ct(d)["lp"][:, 0]
    Vs = [oct_.potentials(s, Params(method="ewald", beta=b, realspace="images", rmax=12.0))[0][lps]
          for b in (0.5, 0.6)]
    assert np.abs(Vs[0] - Vs[1]).max() < 1e-7 * np.abs(Vs[0]).max()
    # SPME with the real-space sum converged inside the 3.2 A cutoff
    # (erfc(1.3 * 3.2) ~ 1e-8) and a fine grid
    Vp = oct_.potentials(s, Params(method="spme", beta=1.3, cutoff=3.2, grid=(64, 64, 64),
                                   order=8))[0][lps]
    Ve = oct_.potentials(s, Params(method="ewald", beta=0.55, realspace="images", rmax=12.0))[0][lps]
    assert np.abs(Vp - Ve).max() < 1e-6 * np.abs(Ve).max()


def test_c2_energy_structure():
    s, c, d = _cluster()
    prm = Params(method="direct")
    E0, _ = oct_.energy_forces(s, prm, c)
    assert E0 < 0
    th = 0.9
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    # a rigid motion of a cluster: rotate the positions and the multipoles
    from oracle.frames import _sym6_to_mat, _mat_to_sym6
    rot = System(**{**s.__dict__, "pos": s.pos @ Rz.T + 3.0, "dip": s.dip @ Rz.T,
                    "quad": _mat_to_sym6(np.einsum("ab,nbc,dc->nad", Rz, _sym6_to_mat(s.quad), Rz)),
                    "alpha": _mat_to_sym6(np.einsum("ab,nbc,dc->nad", Rz, _sym6_to_mat(s.alpha),
                                                    Rz))})
    assert oct_.energy_forces(rot, prm, c)[0] == pytest.approx(E0, rel=1e-11)
    c2 = dict(c, lp_par=c["lp_par"] * np.array([3.0, 1.0]))
    assert oct_.energy_forces(s, prm, c2)[0] == pytest.approx(3.0 * E0, rel=1e-12)
    # E * dE does not depend on ae: one lone pair, one acceptor
    one = dict(c, lp=c["lp"][:1], lp_par=c["lp_par"][:1].copy())
    V, _ = oct_.potentials(s, prm)
    prods = []
    for ae in (200.0, 400.0):
        one["lp_par"][0, 1] = ae
        e = oct_.energy_forces(s, prm, one)[0]
        prods.append(e)
    # all pairs share the lone pair, so dE differs only through ah (equal here)
    dE = [ae + 332.0637133 * V[one["lp"][0, 0]] - c["ah"][0] for ae in (200.0, 400.0)]
    assert prods[0] * dE[0] == pytest.approx(prods[1] * dE[1], rel=1e-12)
    # a1 and a2 equivalent (a2 := a1): e1 = e2
    same = dict(c, acc=np.stack([c["acc"][:, 0], c["acc"][:, 0]], 1))
    assert abs(oct_.energy_forces(s, prm, same)[0]) < 1e-25
    big = dict(c, eta=200.0)
    assert abs(oct_.energy_forces(s, prm, big)[0]) < 1e-30


def _fd_forces(s, prm, c, sites, h=1e-5, rtol=1e-6):
    E, F = oct_.energy_forces(s, prm, c)
    scale = np.abs(F).max()
    for i, a in sites:
        p = s.pos.copy()
        p[i, a] += h
        ep = oct_.energy_forces(System(**{**s.__dict__, "pos": p}), prm, c)[0]
        p[i, a] -= 2 * h
        em = oct_.energy_forces(System(**{**s.__dict__, "pos": p}), prm, c)[0]
        assert abs(-(ep - em) / (2 * h) - F[i, a]) <= rtol * scale, (i, a, -(ep - em) / (2 * h),
                                                                     F[i, a])
    return F


# sites: O, H, B, L1 of water 0; O and L2 of water 1
SITES = [(0, 0), (1, 1), (3, 2), (5, 0), (7, 2), (13, 1)]


def test_c3_forces_cluster():
    s, c, d = _cluster()
    F = _fd_forces(s, Params(method="direct"), c, SITES)
    assert np.abs(F.sum(0)).max() < 1e-10 * np.abs(F).max()


def test_c3_forces_ewald():
    d = water_lone_pairs(water_box(4, 6.5, 11))
    _fd_forces(System.from_dict(d), Params(method="ewald", beta=0.55, realspace="images",
                                           rmax=11.0), water_ct(d), SITES)


def test_c3_forces_spme():
    d = water_lone_pairs(water_box(8, 8.0, 12))
    _fd_forces(System.from_dict(d), Params(method="spme", beta=0.5, cutoff=3.7,
                                           grid=(12, 12, 12), order=5), water_ct(d), SITES)


@pytest.mark.parametrize("plant", ["no_w_forces", "no_recip_w"])
def test_c3_planted_mistakes_fail(plant, monkeypatch):
    orig = rs.pair_sum

    def charges_only(M):
        return M[0] is not None and M[1] is None and M[2] is None

    def planted_pair_sum(pairs, cls, kernel, beta, thole, Mi, Mj, what, n, pair_mask=None):
        if what == "force" and cls == "MM" and (charges_only(Mi) or charges_only(Mj)):
            return np.zeros((n, 3))
        return orig(pairs, cls, kernel, beta, thole, Mi, Mj, what, n, pair_mask)

    if plant == "no_w_forces":
        monkeypatch.setattr(rs, "pair_sum", planted_pair_sum)
        s, c, d = _cluster()
        prm = Params(method="direct")
    else:
        orig_rd = Context.recip_derivs

        def no_w(self, mult, at, nderiv):
            e, der = orig_rd(self, mult, at, nderiv)
            if mult[1] is None:      # the w charges only
                der = [np.zeros_like(x) for x in der]
            return e, der

        monkeypatch.setattr(Context, "recip_derivs", no_w)
        d = water_lone_pairs(water_box(8, 8.0, 12))
        s, c = System.from_dict(d), water_ct(d)
        prm = Params(method="spme", beta=0.5, cutoff=3.7, grid=(12, 12, 12), order=5)
    with pytest.raises(AssertionError):
        _fd_forces(s, prm, c, SITES)


def _fd_forces_frames(s, frames, prm, c, sites, h=1e-5, rtol=1e-6):
    E, F = oct_.energy_forces_frames(s, frames, prm, c)
    scale = np.abs(F).max()
    for i, a in sites:
        p = s.pos.copy()
        p[i, a] += h
        ep = oct_.energy_forces_frames(System(**{**s.__dict__, "pos": p}), frames, prm, c)[0]
        p[i, a] -= 2 * h
        em = oct_.energy_forces_frames(System(**{**s.__dict__, "pos": p}), frames, prm, c)[0]
        assert abs(-(ep - em) / (2 * h) - F[i, a]) <= rtol * scale, (i, a, -(ep - em) / (2 * h),
                                                                     F[i, a])
    return F


def test_c4_forces_frames_cluster():
    s, c, d = _cluster()
    fr = water_frames(d, CT_SITES)
    F = _fd_forces_frames(s, fr, Params(method="direct"), c, SITES)
    assert np.abs(F.sum(0)).max() < 1e-10 * np.abs(F).max()
    # the rotation part is not small here
    F0 = oct_.energy_forces(ofr.to_global(s, fr), Params(method="direct"), c)[1]
    assert np.abs(F - F0).max() > 1e-2 * np.abs(F).max()


def test_c4_forces_frames_spme():
    d = water_lone_pairs(water_box(8, 8.0, 12))
    _fd_forces_frames(System.from_dict(d), water_frames(d, CT_SITES),
                      Params(method="spme", beta=0.5, cutoff=3.7, grid=(12, 12, 12), order=5),
                      water_ct(d), SITES)


def test_c4_planted_no_rotation_fails(monkeypatch):
    monkeypatch.setattr(ofr, "gradient_forces", lambda s, f, Gd, GT, Ga=None: np.zeros((s.n, 3)))
    s, c, d = _cluster()
    with pytest.raises(AssertionError):
        _fd_forces_frames(s, water_frames(d, CT_SITES), Params(method="direct"), c, SITES)
