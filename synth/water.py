"""Synthetic rigid-water systems with random multipoles and polarizabilities.

Each water has five sites in the order O, H1, H2, B1, B2, where B1 and B2 are
the O-H bond barycentres.  Charges are O -0.8, H +0.4, B 0.  Every site gets a
random dipole (uniform in the ball |d| <= 0.1 e*A) and a random traceless
quadrupole (xx, yy, xy, xz, yz uniform in [-0.1, 0.1] e*A^2, zz = -(xx+yy)).
O, B1 and B2 get a random SPD polarizability R diag(l1,l2,l3) R^T with
eigenvalues uniform in [0.3, 1.0] A^3 and a Haar-random rotation R; the H
sites are not polarizable (zero tensor).

Layouts (all float64, caller order):
  pos   [n, 3]  A
  mol   [n]     int32 molecule id
  q     [n]     e
  dip   [n, 3]  e*A
  quad  [n, 6]  e*A^2, (xx, xy, xz, yy, yz, zz), traceless
  alpha [n, 6]  A^3,   (xx, xy, xz, yy, yz, zz), zero row = not polarizable
  box   [3] or None (cluster)

Periodic boxes: waters sit on a jittered simple-cubic lattice
(n_side = ceil(N^(1/3)), a random subset of lattice points, spacing L/n_side,
jitter U[-0.1, 0.1] A per axis) with Haar-random orientations; an
orientation is redrawn while any site of the water lies within 1.0 A of a
site of another water.  Clusters: oxygens placed one after the other,
uniformly in a sphere of radius 1.15 (3n / (4 pi 0.0334))^(1/3) A, keeping
O-O >= 2.5 A, then oriented the same way.

The random stream is numpy's PCG64 seeded with 22010804 + seed index; the
draw order is fixed (lattice subset, jitter, orientations, orientation
redraws, dipoles, quadrupoles, polarizabilities).
"""
import math

import numpy as np
from scipy.spatial import cKDTree

SITE_NAMES = ("O", "H1", "H2", "B1", "B2")
WATER_SITES = 5
_OH = 0.9572
_HOH = math.radians(104.52)
_SEED_BASE = 22010804

# Named workloads: sizes and discretisation parameters of the water boxes.
CONFIGS = {
    "box216": dict(index=1, n_waters=216, box=18.643, cutoff=8.0, beta=0.45,
                   grid=20, order=5, tol=1e-8),
    "box4096": dict(index=2, n_waters=4096, box=49.66, cutoff=9.0, beta=0.40,
                    grid=48, order=5, tol=1e-8),
    "box32000": dict(index=3, n_waters=32000, box=98.55, cutoff=9.0,
                     beta=0.40, grid=96, order=5, tol=1e-8),
    "box96000": dict(index=5, n_waters=96000, box=142.2, cutoff=9.0,
                     beta=0.40, grid=144, order=5, tol=1e-8),
    "box1024": dict(index=4, n_waters=1024, box=31.318, cutoff=9.0,
                    beta=0.40, grid=32, order=5, tol=1e-8),
}


def _water_frame():
    """Body-frame coordinates of O, H1, H2, B1, B2 (O at origin)."""
    h = 0.5 * _HOH
    h1 = np.array([_OH * math.sin(h), 0.0, _OH * math.cos(h)])
    h2 = np.array([-_OH * math.sin(h), 0.0, _OH * math.cos(h)])
    o = np.zeros(3)
    return np.stack([o, h1, h2, 0.5 * (o + h1), 0.5 * (o + h2)])


def _haar_rotations(rng, n):
    """n Haar-random rotation matrices from normalised Gaussian quaternions."""
    qv = rng.standard_normal((n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    rot = np.empty((n, 3, 3))
    rot[:, 0, 0] = 1 - 2 * (y * y + z * z)
    rot[:, 0, 1] = 2 * (x * y - z * w)
    rot[:, 0, 2] = 2 * (x * z + y * w)
    rot[:, 1, 0] = 2 * (x * y + z * w)
    rot[:, 1, 1] = 1 - 2 * (x * x + z * z)
    rot[:, 1, 2] = 2 * (y * z - x * w)
    rot[:, 2, 0] = 2 * (x * z - y * w)
    rot[:, 2, 1] = 2 * (y * z + x * w)
    rot[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return rot


def _place_sites(centres, rot):
    frame = _water_frame()
    return centres[:, None, :] + np.einsum("nab,sb->nsa", rot, frame)


def _clash_molecules(sites, box, min_sep=1.0):
    """Molecule indices (later of each clashing pair) with an intermolecular
    site pair closer than min_sep."""
    n = sites.shape[0]
    flat = sites.reshape(-1, 3)
    if box is not None:
        flat = np.mod(flat, box)
        tree = cKDTree(flat, boxsize=box)
    else:
        tree = cKDTree(flat)
    pairs = tree.query_pairs(min_sep, output_type="ndarray")
    if len(pairs) == 0:
        return np.zeros(0, dtype=np.int64)
    mi = pairs[:, 0] // WATER_SITES
    mj = pairs[:, 1] // WATER_SITES
    inter = mi != mj
    later = np.maximum(mi[inter], mj[inter])
    del n
    return np.unique(later)


def _orient(rng, centres, box):
    rot = _haar_rotations(rng, len(centres))
    for _ in range(1000):
        sites = _place_sites(centres, rot)
        bad = _clash_molecules(sites, box)
        if len(bad) == 0:
            return sites
        rot[bad] = _haar_rotations(rng, len(bad))
    raise RuntimeError("could not orient waters without clashes")


def _multipoles(rng, n_waters):
    n = n_waters * WATER_SITES
    q = np.tile(np.array([-0.8, 0.4, 0.4, 0.0, 0.0]), n_waters)
    # dipoles uniform in the ball of radius 0.1
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    rad = 0.1 * rng.random(n) ** (1.0 / 3.0)
    dip = v * rad[:, None]
    u = rng.uniform(-0.1, 0.1, size=(n, 5))  # xx, yy, xy, xz, yz
    quad = np.empty((n, 6))
    quad[:, 0] = u[:, 0]
    quad[:, 3] = u[:, 1]
    quad[:, 1] = u[:, 2]
    quad[:, 2] = u[:, 3]
    quad[:, 4] = u[:, 4]
    quad[:, 5] = -(u[:, 0] + u[:, 1])
    # polarizabilities at O, B1, B2
    pol_mask = np.tile(np.array([True, False, False, True, True]), n_waters)
    npol = int(pol_mask.sum())
    eig = rng.uniform(0.3, 1.0, size=(npol, 3))
    rot = _haar_rotations(rng, npol)
    a3 = np.einsum("nab,nb,ncb->nac", rot, eig, rot)
    alpha = np.zeros((n, 6))
    alpha[pol_mask] = np.stack([a3[:, 0, 0], a3[:, 0, 1], a3[:, 0, 2],
                                a3[:, 1, 1], a3[:, 1, 2], a3[:, 2, 2]], axis=1)
    return q, dip, quad, alpha


def _pack(sites, n_waters, box, rng):
    q, dip, quad, alpha = _multipoles(rng, n_waters)
    pos = sites.reshape(-1, 3).copy()
    mol = np.repeat(np.arange(n_waters, dtype=np.int32), WATER_SITES)
    return dict(pos=pos, mol=mol, q=q, dip=dip, quad=quad, alpha=alpha,
                box=None if box is None else np.array([box, box, box], float))


def water_box(n_waters, box_len, seed_index=0):
    """Jittered-lattice periodic water box (positions wrapped into [0, L))."""
    rng = np.random.Generator(np.random.PCG64(_SEED_BASE + seed_index))
    n_side = int(math.ceil(n_waters ** (1.0 / 3.0) - 1e-9))
    if n_side ** 3 < n_waters:
        n_side += 1
    spacing = box_len / n_side
    chosen = np.sort(rng.choice(n_side ** 3, size=n_waters, replace=False))
    ix = chosen % n_side
    iy = (chosen // n_side) % n_side
    iz = chosen // (n_side * n_side)
    centres = (np.stack([ix, iy, iz], axis=1) + 0.5) * spacing
    centres = centres + rng.uniform(-0.1, 0.1, size=centres.shape)
    sites = _orient(rng, centres, np.array([box_len] * 3))
    sites = np.mod(sites, box_len)
    return _pack(sites, n_waters, box_len, rng)


def water_box_ortho(counts, spacing, seed_index=0):
    """Orthorhombic periodic box: a full jittered lattice of counts[a]
    waters along axis a with lattice spacing[a] (box sides counts * spacing,
    positions wrapped into the box)."""
    rng = np.random.Generator(np.random.PCG64(_SEED_BASE + 2000 + seed_index))
    counts = np.asarray(counts, dtype=int)
    spacing = np.asarray(spacing, dtype=float)
    box = counts * spacing
    grid = np.stack(np.meshgrid(*[np.arange(c) for c in counts], indexing="ij"), axis=-1)
    centres = (grid.reshape(-1, 3) + 0.5) * spacing
    centres = centres + rng.uniform(-0.1, 0.1, size=centres.shape)
    n_waters = len(centres)
    sites = _orient(rng, centres, box)
    sites = np.mod(sites, box)
    d = _pack(sites, n_waters, None, rng)
    d["box"] = box.copy()
    return d


def water_cluster(n_waters, seed_index=0):
    """Random compact gas-phase water cluster (O-O >= 2.5 A)."""
    rng = np.random.Generator(np.random.PCG64(_SEED_BASE + 1000 + seed_index))
    radius = 1.15 * (3.0 * n_waters / (4.0 * math.pi * 0.0334)) ** (1.0 / 3.0)
    centres = []
    tries = 0
    while len(centres) < n_waters:
        tries += 1
        if tries > 200000:
            raise RuntimeError("cluster placement failed")
        p = rng.uniform(-radius, radius, size=3)
        if p @ p > radius * radius:
            continue
        if centres:
            d = np.linalg.norm(np.asarray(centres) - p, axis=1)
            if d.min() < 2.5:
                continue
        centres.append(p)
    sites = _orient(rng, np.asarray(centres), None)
    return _pack(sites, n_waters, None, rng)


def config_system(name):
    """System dict plus its discretisation parameters for a named workload."""
    c = CONFIGS[name]
    sysd = water_box(c["n_waters"], c["box"], seed_index=c["index"])
    params = dict(beta=c["beta"], cutoff=c["cutoff"], grid=c["grid"],
                  order=c["order"], tol=c["tol"])
    return sysd, params


def water_frames(sysd, sites_per_water=WATER_SITES):
    """Frame sites of every site for local-frame multipoles: each water's
    five sites (O, H1, H2, B1, B2, consecutive) use the frame of its O, H1
    and H2.  Returns int32 [n, 3] site indices (caller order).  The random
    dipoles, quadrupoles and polarizabilities of the system dicts serve as
    the local-frame values (their distributions do not depend on the
    frame).  With sites_per_water = CT_SITES (the lone pairs appended by
    water_lone_pairs) the two lone-pair rows are -1: no frame."""
    n = len(sysd["pos"])
    first = (np.arange(n) // sites_per_water) * sites_per_water
    f = np.stack([first, first + 1, first + 2], axis=1).astype(np.int32)
    if sites_per_water == CT_SITES:
        f[np.arange(n) % CT_SITES >= WATER_SITES] = -1
    return f


MASSES = {"O": 15.999, "H": 1.008}   # g/mol; the bond barycentres are massless


def water_md(sysd, seed_index=0, temperature=300.0, k_oh=500.0, k_hh=150.0, rho_o=1.6,
             rho_h=0.8, rho_b=0.8, rep_eps=0.5):
    """Dynamics inputs for a water system: masses (O, H; B1 and B2 massless),
    the barycentres as midpoint virtual sites of (O, H1) and (O, H2),
    three harmonic bonds per water (O-H1, O-H2, H1-H2; kcal/mol/A^2) with
    rest lengths from the current geometry, repulsion radii (O rho_o, H
    rho_h, B rho_b, A; every site carries random multipoles, so every site
    needs a wall) with the strength rep_eps (kcal/mol), and Maxwell-Boltzmann
    velocities (A/fs) at `temperature` from numpy's PCG64 seeded with
    22010804 + 1000 + seed_index (zero rows at the virtual sites)."""
    pos = np.asarray(sysd["pos"], float)
    n = len(pos)
    nw = n // WATER_SITES
    base = np.arange(nw) * WATER_SITES
    masses = np.zeros(n)
    masses[base] = MASSES["O"]
    masses[base + 1] = MASSES["H"]
    masses[base + 2] = MASSES["H"]
    vsites = -np.ones((n, 2), dtype=np.int32)
    vsites[base + 3] = np.stack([base, base + 1], 1)
    vsites[base + 4] = np.stack([base, base + 2], 1)
    bonds = np.concatenate([np.stack([base, base + 1], 1), np.stack([base, base + 2], 1),
                            np.stack([base + 1, base + 2], 1)]).astype(np.int32)
    k = np.concatenate([np.full(nw, k_oh), np.full(nw, k_oh), np.full(nw, k_hh)])
    r0 = np.linalg.norm(pos[bonds[:, 0]] - pos[bonds[:, 1]], axis=1)
    rng = np.random.default_rng(_SEED_BASE + 1000 + seed_index)
    kt = 0.0019872041 * temperature                   # kcal/mol
    sigma = np.zeros(n)
    atoms = masses > 0
    sigma[atoms] = np.sqrt(kt * 4.184e-4 / masses[atoms])
    vel = rng.standard_normal((n, 3)) * sigma[:, None]
    rho = np.zeros(n)
    rho[base] = rho_o
    rho[base + 1] = rho_h
    rho[base + 2] = rho_h
    rho[base + 3] = rho_b
    rho[base + 4] = rho_b
    return dict(masses=masses, vsites=vsites, bonds=bonds, bond_k=k, bond_r0=r0, vel=vel,
                rep_radius=rho, rep_eps=float(rep_eps))


CT_SITES = 7   # O, H1, H2, B1, B2, L1, L2


def water_lone_pairs(sysd, length=0.5, half_angle_deg=54.74):
    """The system with two lone-pair sites appended to every water (order O,
    H1, H2, B1, B2, L1, L2): at the oxygen plus `length` A along
    -cos(h) e_z +- sin(h) e_y, e_z the H-O-H bisector (towards the H), e_y
    the normal of the molecular plane.  Lone pairs carry no multipoles and
    no polarizability."""
    pos = np.asarray(sysd["pos"], float)
    nw = len(pos) // WATER_SITES
    w = pos.reshape(nw, WATER_SITES, 3)
    o, h1, h2 = w[:, 0], w[:, 1], w[:, 2]
    u = (h1 - o) / np.linalg.norm(h1 - o, axis=1, keepdims=True)
    v = (h2 - o) / np.linalg.norm(h2 - o, axis=1, keepdims=True)
    ez = (u + v) / np.linalg.norm(u + v, axis=1, keepdims=True)
    ey = np.cross(u, v)
    ey /= np.linalg.norm(ey, axis=1, keepdims=True)
    h = math.radians(half_angle_deg)
    l1 = o + length * (-math.cos(h) * ez + math.sin(h) * ey)
    l2 = o + length * (-math.cos(h) * ez - math.sin(h) * ey)
    out = {}
    new_pos = np.concatenate([w, l1[:, None], l2[:, None]], axis=1).reshape(-1, 3)
    out["pos"] = new_pos
    out["mol"] = np.repeat(np.arange(nw, dtype=np.int32), CT_SITES)

    def widen(a, width):
        a = np.asarray(a, float).reshape(nw, WATER_SITES, *((width,) if width else ()))
        z = np.zeros((nw, 2) + ((width,) if width else ()))
        return np.concatenate([a, z], axis=1).reshape((nw * CT_SITES,) +
                                                      ((width,) if width else ()))

    out["q"] = widen(sysd["q"], 0)
    out["dip"] = widen(sysd["dip"], 3)
    out["quad"] = widen(sysd["quad"], 6)
    out["alpha"] = widen(sysd["alpha"], 6)
    out["box"] = sysd.get("box")
    return out


def water_ct(sysd7, n_occ=2.0, ae=250.0, ah=20.0, rvdw_o=1.7, rvdw_h=1.2, eta=3.0, cs=0.5,
             cp=0.87, t=0.4, m=0.3):
    """Charge-transfer inputs for a system from water_lone_pairs: each lone
    pair (L1, L2) carried by its oxygen with occupation n_occ and ionization
    energy ae (kcal/mol); each O-H bond an acceptor (a1 = H, a2 = O) with
    affinity ah (kcal/mol); van der Waals radii (O, H; 1 A elsewhere); the
    constants eta, C_s, C_p, t, m.  All values are synthetic: the paper's
    parameters are not available."""
    n = len(sysd7["pos"])
    nw = n // CT_SITES
    base = np.arange(nw) * CT_SITES
    lp = np.concatenate([np.stack([base + 5, base], 1), np.stack([base + 6, base], 1)])
    lp = lp[np.argsort(lp[:, 0], kind="stable")].astype(np.int32)
    acc = np.concatenate([np.stack([base + 1, base], 1), np.stack([base + 2, base], 1)])
    acc = acc[np.argsort(acc[:, 0], kind="stable")].astype(np.int32)
    rvdw = np.ones(n)
    rvdw[base] = rvdw_o
    rvdw[base + 1] = rvdw_h
    rvdw[base + 2] = rvdw_h
    lp_par = np.tile([n_occ, ae], (len(lp), 1))
    return dict(lp=lp, lp_par=lp_par, acc=acc, ah=np.full(len(acc), float(ah)), rvdw=rvdw,
                eta=eta, cs=cs, cp=cp, t=t, m=m)
