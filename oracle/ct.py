"""Reduced many-body charge transfer (charge delocalization) energy and its
forces.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Many-Body Charge Transfer/Charge Delocalization, the reduced
expression (Eq. 13-16): for every lone pair l (carried by atom c) and every
acceptor bond k (atoms a1, a2) of another molecule,
  E_ct = sum_l sum_k -n(l) (e1 - e2)^2 / dE
  e1   = exp(-eta rho1) (V_int(a1) - V_l) (C_s t + C_p m cos(alpha))
  e2   = exp(-eta rho2) (V_int(a2) - V_l) (C_s t + C_p m cos(beta))
  dE   = ae(l) + V_l - ah(k)
  rho1 = |r_c - r_a1| / (2 sqrt(rvdw_c rvdw_a1)), rho2 likewise with a2,
  alpha, beta the angles at c between (r_l - r_c) and (r_a1 - r_c),
  (r_a2 - r_c).

Readings where the paper is terse:
  * V_l is the electrostatic potential of the permanent multipoles of all
    other molecules at the lone pair (the total potential, Ewald-summed in a
    periodic cell, own molecule excluded as for the permanent field);
    V_int(a) the potential at acceptor atom a of the other sites of its own
    molecule (bare Coulomb).  Potentials enter the energies in kcal/mol per
    unit charge (times the Coulomb constant).
  * a1 is the hydrogen of the X-H acceptor bond, a2 the heavy atom; dE uses
    the affinity ah of the acceptor bond.
  * Pairs are taken when |r_c - r_a1| is below the real-space cutoff
    (periodic, minimum image); a cluster takes all pairs.
  * t and m (tabulated in the cited works) and C_s, C_p, eta are single
    constants for the water lone pair - O-H acceptor combination.
Lone-pair sites carry no multipoles and no polarizability.

Forces: the direct derivatives of each pair term (distances, angles), plus
those of the potentials through w_l = dE/dV_l and u_a = dE/dV_int(a):
-grad(sum_l w_l V_l) is the force of point charges w_l at the lone pairs
interacting with the other molecules' multipoles (Ewald-summed when
periodic), -grad(sum_a u_a V_int(a)) the bare intramolecular analogue.
"""
import numpy as np

from . import realspace as rs
from .model import Context
from .units import COULOMB


def _wrap(d, box):
    if box is None:
        return d
    b = np.asarray(box, float)
    return d - b * np.round(d / b)


def potentials(sysm, prm, ctx=None):
    """(V at every site from the other molecules' multipoles, Ewald-summed
    when periodic, V_int at every site from its own molecule's other
    sites), e/A.  Only meaningful at sites without multipoles of their own
    (V) -- lone pairs -- and at any site (V_int)."""
    c = ctx if ctx is not None else Context(sysm, prm)
    s = c.s
    mult = (s.q, s.dip, s.th)
    none3 = (None, None, None)
    V = rs.pair_sum(c.pairs, "MM", c.kernel, prm.beta, c.thole, none3, mult, "potential", s.n)
    if prm.periodic:
        _, der = c.recip_derivs(mult, s.pos, 0)
        V = V + der[0]
    Vint = rs.pair_sum(c.pairs, "intra", "bare", prm.beta, c.thole, none3, mult, "potential",
                       s.n)
    return V, Vint


def _pairs(sysm, prm, ct):
    """(l, k) index pairs: carrier and a1 in different molecules, within the
    cutoff when periodic."""
    pos, mol, box = sysm.pos, sysm.mol, sysm.box
    lp = np.asarray(ct["lp"], int)
    acc = np.asarray(ct["acc"], int)
    out = []
    for l in range(len(lp)):
        c = lp[l, 1]
        for k in range(len(acc)):
            a1 = acc[k, 0]
            if mol[a1] == mol[c]:
                continue
            if box is not None:
                if np.linalg.norm(_wrap(pos[a1] - pos[c], box)) >= prm.cutoff:
                    continue
            out.append((l, k))
    return out


def _pair_terms(sysm, ct, V, Vint, l, k):
    """Energy of one pair and its partial derivatives: (E, dE/dV_l,
    dE/dVint_a1, dE/dVint_a2, gradients w.r.t. r_l, r_c, r_a1, r_a2)."""
    pos, box = sysm.pos, sysm.box
    L, c = ct["lp"][l]
    a1, a2 = ct["acc"][k]
    n_occ, ae = ct["lp_par"][l]
    ah = ct["ah"][k]
    rv = ct["rvdw"]
    eta, cs, cp, t, m = ct["eta"], ct["cs"], ct["cp"], ct["t"], ct["m"]
    u = _wrap(pos[L] - pos[c], box)
    d1 = _wrap(pos[a1] - pos[c], box)
    d2 = _wrap(pos[a2] - pos[c], box)
    nu, r1, r2 = np.linalg.norm(u), np.linalg.norm(d1), np.linalg.norm(d2)
    s1 = 2.0 * np.sqrt(rv[c] * rv[a1])
    s2 = 2.0 * np.sqrt(rv[c] * rv[a2])
    ca = u @ d1 / (nu * r1)
    cb = u @ d2 / (nu * r2)
    x1 = np.exp(-eta * r1 / s1)
    x2 = np.exp(-eta * r2 / s2)
    X1 = COULOMB * (Vint[a1] - V[L])
    X2 = COULOMB * (Vint[a2] - V[L])
    g1 = cs * t + cp * m * ca
    g2 = cs * t + cp * m * cb
    e1 = x1 * X1 * g1
    e2 = x2 * X2 * g2
    dE = ae + COULOMB * V[L] - ah
    E = -n_occ * (e1 - e2) ** 2 / dE
    G = -2.0 * n_occ * (e1 - e2) / dE          # dE/de1 = G, dE/de2 = -G
    GD = n_occ * (e1 - e2) ** 2 / dE ** 2      # dE/d(dE)
    dV = COULOMB * (-G * x1 * g1 + G * x2 * g2 + GD)
    dVi1 = COULOMB * G * x1 * g1
    dVi2 = -COULOMB * G * x2 * g2
    # geometry
    de1_dr1 = -eta / s1 * e1
    de2_dr2 = -eta / s2 * e2
    de1_dca = x1 * X1 * cp * m
    de2_dcb = x2 * X2 * cp * m
    dca_du = d1 / (nu * r1) - ca * u / nu ** 2
    dca_dd1 = u / (nu * r1) - ca * d1 / r1 ** 2
    dcb_du = d2 / (nu * r2) - cb * u / nu ** 2
    dcb_dd2 = u / (nu * r2) - cb * d2 / r2 ** 2
    g_u = G * de1_dca * dca_du - G * de2_dcb * dcb_du
    g_d1 = G * (de1_dr1 * d1 / r1 + de1_dca * dca_dd1)
    g_d2 = -G * (de2_dr2 * d2 / r2 + de2_dcb * dcb_dd2)
    g_c = -(g_u + g_d1 + g_d2)
    return E, dV, dVi1, dVi2, g_u, g_c, g_d1, g_d2


def _charges(sysm, prm, ct, c):
    """(E_ct, direct forces, W = dE/dV at the lone pairs, U = dE/dV_int at
    the acceptor atoms), per site."""
    s = c.s
    V, Vint = potentials(s, prm, c)
    lp = np.asarray(ct["lp"], int)
    acc = np.asarray(ct["acc"], int)
    E = 0.0
    F = np.zeros((s.n, 3))
    W = np.zeros(s.n)     # dE/dV at lone-pair sites
    U = np.zeros(s.n)     # dE/dV_int at acceptor atoms
    for l, k in _pairs(s, prm, ct):
        e, dV, dVi1, dVi2, g_u, g_c, g_d1, g_d2 = _pair_terms(s, ct, V, Vint, l, k)
        E += e
        L, cr = lp[l]
        a1, a2 = acc[k]
        W[L] += dV
        U[a1] += dVi1
        U[a2] += dVi2
        F[L] -= g_u
        F[cr] -= g_c
        F[a1] -= g_d1
        F[a2] -= g_d2
    return E, F, W, U


def energy_forces(sysm, prm, ct, ctx=None):
    """(E_ct kcal/mol, forces (n, 3) kcal/mol/A), the multipoles fixed in
    the global frame."""
    c = ctx if ctx is not None else Context(sysm, prm)
    s = c.s
    E, F, W, U = _charges(s, prm, ct, c)
    mult = (s.q, s.dip, s.th)
    wq = (W, None, None)
    uq = (U, None, None)
    F += rs.pair_sum(c.pairs, "MM", c.kernel, prm.beta, c.thole, wq, mult, "force", s.n)
    F += rs.pair_sum(c.pairs, "MM", c.kernel, prm.beta, c.thole, mult, wq, "force", s.n)
    F += rs.pair_sum(c.pairs, "intra", "bare", prm.beta, c.thole, uq, mult, "force", s.n)
    F += rs.pair_sum(c.pairs, "intra", "bare", prm.beta, c.thole, mult, uq, "force", s.n)
    if prm.periodic:
        _, dm = c.recip_derivs(mult, s.pos, 1)
        _, dw = c.recip_derivs(wq, s.pos, 3)
        F -= W[:, None] * dm[1]
        F -= (s.q[:, None] * dw[1] + np.einsum("nb,nab->na", s.dip, dw[2])
              + np.einsum("nbc,nabc->na", s.th, dw[3]) / 3.0)
    return E, F


def multipole_gradients(sysm, prm, ct, ctx=None):
    """(G^d (n,3), G^Theta (n,3,3)): derivatives of E_ct with respect to the
    global dipoles and quadrupoles.  E_ct depends on the multipoles through
    V_l and V_int only, so G^d = -(field of the charges W at the lone pairs
    and U at the acceptor atoms), with the same sums as their potentials
    (other molecules, Ewald-summed when periodic, for W; own molecule, bare,
    for U), and G^Theta = -1/3 of the field gradient."""
    c = ctx if ctx is not None else Context(sysm, prm)
    s = c.s
    _, _, W, U = _charges(s, prm, ct, c)
    none3 = (None, None, None)
    wq = (W, None, None)
    uq = (U, None, None)
    E = rs.pair_sum(c.pairs, "MM", c.kernel, prm.beta, c.thole, none3, wq, "field", s.n)
    E += rs.pair_sum(c.pairs, "intra", "bare", prm.beta, c.thole, none3, uq, "field", s.n)
    dE = rs.pair_sum(c.pairs, "MM", c.kernel, prm.beta, c.thole, none3, wq, "fieldgrad", s.n)
    dE += rs.pair_sum(c.pairs, "intra", "bare", prm.beta, c.thole, none3, uq, "fieldgrad", s.n)
    Gd = -E
    GT = -dE / 3.0
    if prm.periodic:
        _, der = c.recip_derivs(wq, s.pos, 2)
        Gd = Gd + der[1]
        GT = GT + der[2] / 3.0
    return Gd, GT


def energy_forces_frames(sys_local, frames, prm, ct):
    """(E_ct, forces) with multipoles given in local frames: the energy at
    the rotated multipoles, the forces with them fixed plus the forces of
    the rotation."""
    from .frames import to_global, gradient_forces
    glob = to_global(sys_local, frames)
    c = Context(glob, prm)
    E, F = energy_forces(glob, prm, ct, c)
    Gd, GT = multipole_gradients(glob, prm, ct, c)
    return E, F + gradient_forces(sys_local, frames, Gd, GT)
