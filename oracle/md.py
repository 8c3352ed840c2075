"""Beeman molecular dynamics over the oracle's energies and forces.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Computational Details: the simulations use the Beeman integrator
with 1 fs steps and solve the polarization at every step.  The paper's
bonded and short-range terms are not available, so a trajectory here adds
stand-ins: harmonic bonds that hold the molecules together, a soft
repulsion eps ((rho_i + rho_j)/r)^12 between sites of different molecules
(both radii positive) within the cutoff, and massless midpoint virtual
sites (the bond barycentres of the water model) that hand their forces to
their parents.

Beeman's scheme (Beeman 1976), for positions x, velocities v and
accelerations a:
  x(t + dt) = x(t) + v(t) dt + (4 a(t) - a(t - dt)) dt^2 / 6
  v(t + dt) = v(t) + (2 a(t + dt) + 5 a(t) - a(t - dt)) dt / 6
started with a(-dt) = a(0).  Units: A, fs, g/mol, kcal/mol, so
a = F / m * ACCEL with ACCEL = 4.184e-4 (1 kcal/mol/A per g/mol in A/fs^2).
"""
import numpy as np

from .model import System, evaluate
from .frames import to_global, frame_forces

ACCEL = 4.184e-4


def _wrap(d, box):
    if box is None:
        return d
    b = np.asarray(box, float)
    return d - b * np.round(d / b)


def place_vsites(pos, vsites, box):
    """Virtual sites at the midpoint (minimum image) of their two parents."""
    out = pos.copy()
    v = np.flatnonzero(vsites[:, 0] >= 0)
    p, q = vsites[v, 0], vsites[v, 1]
    out[v] = pos[p] + 0.5 * _wrap(pos[q] - pos[p], box)
    return out


def bond_energy_forces(pos, bonds, k, r0, box):
    """E = sum 1/2 k (|r_i - r_j| - r0)^2 and its forces (n, 3)."""
    F = np.zeros_like(pos)
    if len(bonds) == 0:
        return 0.0, F
    i, j = bonds[:, 0], bonds[:, 1]
    d = _wrap(pos[i] - pos[j], box)
    r = np.linalg.norm(d, axis=1)
    ext = r - r0
    f = (-k * ext / r)[:, None] * d
    np.add.at(F, i, f)
    np.add.at(F, j, -f)
    return float(np.sum(0.5 * k * ext ** 2)), F


def repulsion_energy_forces(pos, mol, rho, eps, box, cutoff):
    """Stand-in repulsion E = sum over pairs of sites of different molecules,
    both with a positive radius, within the cutoff of
    eps ((rho_i + rho_j) / r)^12, and its forces (brute force over all
    pairs, minimum image)."""
    F = np.zeros_like(pos)
    if eps == 0.0:
        return 0.0, F
    n = len(pos)
    i, j = np.triu_indices(n, 1)
    keep = (mol[i] != mol[j]) & (rho[i] > 0) & (rho[j] > 0)
    i, j = i[keep], j[keep]
    d = _wrap(pos[i] - pos[j], box)
    r2 = np.sum(d * d, axis=1)
    inside = r2 < cutoff * cutoff
    i, j, d, r2 = i[inside], j[inside], d[inside], r2[inside]
    e = eps * ((rho[i] + rho[j]) ** 2 / r2) ** 6
    f = (12.0 * e / r2)[:, None] * d
    np.add.at(F, i, f)
    np.add.at(F, j, -f)
    return float(e.sum()), F


def atom_forces(sysd, prm, pos, masses, vsites, bonds, k, r0, frames=None, rho=None, eps=0.0):
    """(F on every site with the virtual-site forces handed to their parents
    (zero rows at virtual sites), E_pol, E_elec, E_bond, E_rep) at `pos`, the
    polarization solved from the cold guess to prm.tol."""
    box = sysd.get("box")
    s = System.from_dict(dict(sysd, pos=pos))
    if frames is None:
        o = evaluate(s, prm)
        F = o["forces"].copy()
    else:
        g = to_global(s, frames)
        o = evaluate(g, prm)
        F = o["forces"] + frame_forces(s, frames, prm, o["mu"])
    er = 0.0
    if eps > 0.0:
        cut = prm.cutoff if box is not None else np.inf
        er, Fr = repulsion_energy_forces(pos, np.asarray(sysd["mol"]), rho, eps, box, cut)
        F = F + Fr
    v = np.flatnonzero(vsites[:, 0] >= 0)
    for col in (0, 1):
        np.add.at(F, vsites[v, col], 0.5 * F[v])
    F[v] = 0.0
    eb, Fb = bond_energy_forces(pos, bonds, k, r0, box)
    return F + Fb, o["E_pol"], o["E_elec"], eb, er


def kinetic(vel, masses):
    return float(0.5 * np.sum(masses[:, None] * vel ** 2) / ACCEL)


def beeman(accel, x0, v0, dt, n_steps, atoms):
    """Generic Beeman integrator: accel(x) -> (a, info); only the rows
    `atoms` move.  Returns the list of (x, v, info) after each step."""
    x = x0.copy()
    v = v0.copy()
    a, _ = accel(x)
    ap = a.copy()
    out = []
    for _ in range(n_steps):
        x = x.copy()
        x[atoms] += v[atoms] * dt + (4.0 * a[atoms] - ap[atoms]) * dt * dt / 6.0
        an, info = accel(x)
        v = v.copy()
        v[atoms] += (2.0 * an[atoms] + 5.0 * a[atoms] - ap[atoms]) * dt / 6.0
        ap, a = a, an
        out.append((x, v, info))
    return out


def run(sysd, prm, masses, vsites, bonds, k, r0, vel, dt, n_steps, frames=None, rho=None,
        eps=0.0):
    """A trajectory of the full model: returns per step (x, v, E_pol, E_elec,
    E_bond, E_rep, E_kin)."""
    box = sysd.get("box")
    atoms = np.flatnonzero(masses > 0)
    inv_m = np.zeros_like(masses)
    inv_m[atoms] = 1.0 / masses[atoms]

    def accel(x):
        xs = place_vsites(x, vsites, box)
        F, ep, ee, eb, er = atom_forces(sysd, prm, xs, masses, vsites, bonds, k, r0, frames,
                                        rho, eps)
        return F * inv_m[:, None] * ACCEL, (ep, ee, eb, er)

    x0 = place_vsites(np.asarray(sysd["pos"], float), vsites, box)
    v0 = np.where((masses > 0)[:, None], vel, 0.0)
    steps = beeman(accel, x0, v0, dt, n_steps, atoms)
    return [(place_vsites(x, vsites, box), v, *info, kinetic(v, masses))
            for x, v, info in steps]
