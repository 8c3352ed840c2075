"""Molecular local frames: permanent multipoles and polarizabilities given
in a frame attached to each molecule and rotated to the global frame at the
current geometry, with the forces that follow from that rotation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Multipolar Electrostatics: the distributed multipoles (and, in
SIBFA, the anisotropic polarizabilities) are stored in a local frame of the
molecule and rotated to the global frame at every step, so that the forces
carry the derivative of that rotation (the torques).

Reading for the frame (the paper does not print one): a molecule's frame is
built from three of its sites (o, a, b) -- for water O, H1, H2 -- as
  u = (r_a - r_o)/|r_a - r_o|,  v = (r_b - r_o)/|r_b - r_o|,
  e_z = (u + v)/|u + v|                 (the bisector),
  e_x = (u - (u.e_z) e_z)/|...|         (in the plane, towards a),
  e_y = e_z x e_x,
R = [e_x e_y e_z] (columns), and a site's global quantities are
  d = R d_loc,  Theta = R Theta_loc R^T,  alpha = R alpha_loc R^T.
The Thole widths tr(alpha)/3 are unchanged by the rotation.

Forces.  With the induced dipoles stationary, the total derivative of
E = E_elec + E_pol with respect to a site position r_k is the fixed-multipole
derivative plus the chain rule through R:
  dE/dr_k = dE/dr_k|_fixed + sum_pq (dE/dR)_pq dR_pq/dr_k,
  dE/dR   = sum over the molecule's sites of
            G^d d_loc^T + 2 G^Theta R Theta_loc + 2 G^alpha R alpha_loc,
where G^d = dE/dd, G^Theta = dE/dTheta and G^alpha = dE/dalpha at fixed mu:
  G^d_i     = grad phi(r_i) summed over the interactions d_i takes part in
              (MM class with the permanent multipoles, Mmu class with the
              induced dipoles, the reciprocal potential of the combined
              density) plus the Ewald self term -4 beta^3/(3 sqrt pi)
              (d_i + mu_i) (the self energy of d and the self field that
              removes d_i's reciprocal interaction with mu_i),
  G^Theta_i = 1/3 of the same second derivatives, plus
              -16 beta^5/(45 sqrt pi) Theta_i,
  G^alpha_i = -1/2 (alpha_i^-1 mu_i)(alpha_i^-1 mu_i)^T
              (T's diagonal block is alpha_i^-1).
"""
import math

import numpy as np

from . import realspace as rs
from .model import System, Context, permanent_field, solve, energy_forces
from .units import COULOMB


def _unit(x):
    n = np.linalg.norm(x, axis=-1, keepdims=True)
    return x / n, n


def frame(ro, ra, rb):
    """Rotation matrices (..., 3, 3), columns e_x, e_y, e_z."""
    u, _ = _unit(ra - ro)
    v, _ = _unit(rb - ro)
    ez, _ = _unit(u + v)
    w = u - np.sum(u * ez, -1, keepdims=True) * ez
    ex, _ = _unit(w)
    ey = np.cross(ez, ex)
    return np.stack([ex, ey, ez], axis=-1)


def frame_derivatives(ro, ra, rb):
    """dR/dr for each frame site and coordinate: (..., 3 sites (o, a, b),
    3 coordinates, 3, 3), by differentiating each step above
    (d(x/|x|) = (I - n n^T) dx / |x|)."""
    A, B = ra - ro, rb - ro
    u, nA = _unit(A)
    v, nB = _unit(B)
    s = u + v
    ez, ns = _unit(s)
    uz = np.sum(u * ez, -1, keepdims=True)
    w = u - uz * ez
    ex, nw = _unit(w)
    ey = np.cross(ez, ex)
    shape = ro.shape[:-1]
    out = np.zeros(shape + (3, 3, 3, 3))

    def dunit(n, norm, dx):
        return (dx - np.sum(n * dx, -1, keepdims=True) * n) / norm

    for k, (sa, sb) in enumerate(((-1.0, -1.0), (1.0, 0.0), (0.0, 1.0))):
        for c in range(3):
            e = np.zeros(shape + (3,))
            e[..., c] = 1.0
            du = dunit(u, nA, sa * e)
            dv = dunit(v, nB, sb * e)
            dez = dunit(ez, ns, du + dv)
            dw = du - np.sum(du * ez, -1, keepdims=True) * ez \
                - np.sum(u * dez, -1, keepdims=True) * ez - uz * dez
            dex = dunit(ex, nw, dw)
            dey = np.cross(dez, ex) + np.cross(ez, dex)
            out[..., k, c, :, :] = np.stack([dex, dey, dez], axis=-1)
    return out


def _sym6_to_mat(t6):
    xx, xy, xz, yy, yz, zz = np.moveaxis(t6, -1, 0)
    return np.stack([np.stack([xx, xy, xz], -1), np.stack([xy, yy, yz], -1),
                     np.stack([xz, yz, zz], -1)], -2)


def _mat_to_sym6(m):
    return np.stack([m[..., 0, 0], m[..., 0, 1], m[..., 0, 2], m[..., 1, 1], m[..., 1, 2],
                     m[..., 2, 2]], -1)


def site_rotations(pos, frames):
    """R of every site's molecule (n, 3, 3); frames (n, 3) site indices, a
    row of -1 for a site without a frame (R = identity: its local values
    are global)."""
    f = np.asarray(frames, int)
    R = np.broadcast_to(np.eye(3), (len(f), 3, 3)).copy()
    on = f[:, 0] >= 0
    R[on] = frame(pos[f[on, 0]], pos[f[on, 1]], pos[f[on, 2]])
    return R


def to_global(sys_local, frames):
    """The System with d, Theta, alpha rotated from the local frames at the
    current positions."""
    s = sys_local
    R = site_rotations(s.pos, frames)
    dip = np.einsum("nab,nb->na", R, s.dip)
    quad = _mat_to_sym6(np.einsum("nab,nbc,ndc->nad", R, _sym6_to_mat(s.quad), R))
    alpha = _mat_to_sym6(np.einsum("nab,nbc,ndc->nad", R, _sym6_to_mat(s.alpha), R))
    alpha[np.all(s.alpha == 0.0, axis=1)] = 0.0
    return System(pos=s.pos, mol=s.mol, q=s.q, dip=dip, quad=quad, alpha=alpha, box=s.box,
                  thole=s.thole)


def multipole_gradients(sysm, prm, mu_pol, ctx=None):
    """(G^d (n,3), G^Theta (n,3,3), G^alpha (n,3,3)): derivatives of
    E_elec + E_pol with respect to the global dipoles, quadrupoles (as full
    symmetric matrices) and polarizabilities at fixed mu, kcal/mol units."""
    c = ctx if ctx is not None else Context(sysm, prm)
    s = c.s
    mult = (s.q, s.dip, s.th)
    mud = (None, c.full(mu_pol), None)
    none3 = (None, None, None)
    E = rs.pair_sum(c.pairs, "MM", c.kernel, prm.beta, c.thole, none3, mult, "field", s.n)
    E += rs.pair_sum(c.pairs, "Mmu", c.kernel, prm.beta, c.thole, none3, mud, "field", s.n)
    dE = rs.pair_sum(c.pairs, "MM", c.kernel, prm.beta, c.thole, none3, mult, "fieldgrad", s.n)
    dE += rs.pair_sum(c.pairs, "Mmu", c.kernel, prm.beta, c.thole, none3, mud, "fieldgrad",
                      s.n)
    Gd = -E
    GT = -dE / 3.0
    if prm.periodic:
        comb = (s.q, s.dip + mud[1], s.th)
        _, der = c.recip_derivs(comb, s.pos, 2)
        b = prm.beta
        # the Ewald self terms remove a site's interaction with itself in
        # the reciprocal sum; for the dipole they act on d + mu (the
        # permanent self energy and the self field of E and of T p)
        Gd = Gd + der[1] - 4.0 * b ** 3 / (3.0 * math.sqrt(math.pi)) * comb[1]
        GT = GT + der[2] / 3.0 - 16.0 * b ** 5 / (45.0 * math.sqrt(math.pi)) * s.th
    Ga = np.zeros((s.n, 3, 3))
    a3 = s.alpha3[c.pol]
    am = np.linalg.solve(a3, mu_pol[:, :, None])[:, :, 0]
    Ga[c.pol] = -0.5 * np.einsum("na,nb->nab", am, am)
    return COULOMB * Gd, COULOMB * GT, COULOMB * Ga


def _terms_from_gradients(sys_local, frames, Gd, GT, Ga=None):
    """Per site n and frame site k = o, a, b of n's frame: the force
    -sum_pq C_n,pq dR_pq/dr_k (n, 3, 3), C_n the site's term of dE/dR built
    from the derivatives of an energy with respect to the global dipoles
    (Gd), quadrupoles (GT, full symmetric) and polarizabilities (Ga)."""
    s_loc = sys_local
    f = np.asarray(frames, int)
    R = site_rotations(s_loc.pos, f)
    C = np.einsum("na,nb->nab", Gd, s_loc.dip)
    C += 2.0 * np.einsum("nab,nbc,ncd->nad", GT, R, _sym6_to_mat(s_loc.quad))
    if Ga is not None:
        C += 2.0 * np.einsum("nab,nbc,ncd->nad", Ga, R, _sym6_to_mat(s_loc.alpha))
    on = f[:, 0] >= 0
    per = np.zeros((s_loc.n, 3, 3))
    dR = frame_derivatives(s_loc.pos[f[on, 0]], s_loc.pos[f[on, 1]], s_loc.pos[f[on, 2]])
    per[on] = -np.einsum("npq,nkcpq->nkc", C[on], dR)
    return per


def _frame_terms(sys_local, frames, prm, mu_pol, ctx=None):
    f = np.asarray(frames, int)
    glob = to_global(sys_local, f)
    Gd, GT, Ga = multipole_gradients(glob, prm, mu_pol, ctx)
    return _terms_from_gradients(sys_local, f, Gd, GT, Ga)


def _gather(per, frames, n):
    f = np.asarray(frames, int)
    F = np.zeros((n, 3))
    # each site's contribution, through its own frame sites
    on = f[:, 0] >= 0
    for k in range(3):
        np.add.at(F, f[on, k], per[on, k, :])
    return F


def gradient_forces(sys_local, frames, Gd, GT, Ga=None):
    """The forces (n,3) of the rotation for any energy of the global
    multipoles, given its derivatives Gd (n,3), GT (n,3,3) and, optionally,
    Ga (n,3,3): -sum_pq (dE/dR)_pq dR_pq/dr_k on each frame site k."""
    return _gather(_terms_from_gradients(sys_local, frames, Gd, GT, Ga), frames, sys_local.n)


def frame_forces(sys_local, frames, prm, mu_pol, ctx=None):
    """The forces (n,3) from the rotation of the local multipoles and
    polarizabilities: -sum_pq (dE/dR)_pq dR_pq/dr_k on each frame site k."""
    return _gather(_frame_terms(sys_local, frames, prm, mu_pol, ctx), frames, sys_local.n)


def _min_image(d, box):
    if box is None:
        return d
    b = np.asarray(box, float)
    H = np.diag(b) if b.ndim == 1 else b      # rows: lattice vectors
    frac = d @ np.linalg.inv(H)
    return d - np.round(frac) @ H


def virial(sys_local, frames, prm, mu_pol, ctx=None):
    """Virial (3,3, kcal/mol) with local frames: W_ab = -dE/d eps_ab when the
    strain r -> (1 + eps) r moves the sites and the cell and the local
    multipoles follow their strained frames.  It is the virial at fixed
    global multipoles (model.virial) plus the frame term: for every site's
    frame, sum over its sites k of F_k (r_k - r_o)^T, F_k the forces of
    the rotation (they sum to zero over the frame, so the origin o is
    free; minimum-image separations in a periodic cell)."""
    from .model import virial as fixed_virial
    f = np.asarray(frames, int)
    glob = to_global(sys_local, f)
    c = ctx if ctx is not None else Context(glob, prm)
    W = fixed_virial(glob, prm, mu_pol, ctx=c)
    per = _frame_terms(sys_local, f, prm, mu_pol, ctx=c)
    pos = sys_local.pos
    on = f[:, 0] >= 0
    rel = np.stack([_min_image(pos[f[on, k]] - pos[f[on, 0]], sys_local.box) for k in range(3)],
                   1)
    return W + np.einsum("nkc,nkd->cd", per[on], rel)


def evaluate(sys_local, frames, prm):
    """Full evaluation with local frames: rotate, field, solve, energies,
    and forces including the rotation terms."""
    glob = to_global(sys_local, frames)
    c = Context(glob, prm)
    E0 = permanent_field(glob, prm, ctx=c)
    mu, iters, rho = solve(glob, prm, E0, ctx=c)
    e_pol, e_var, e_elec, F = energy_forces(glob, prm, mu, E0, ctx=c)
    F = F + frame_forces(sys_local, frames, prm, mu, ctx=c)
    return dict(E_pol=e_pol, E_elec=e_elec, forces=F, mu=mu, iters=iters, system=glob)
