"""Top level of the oracle: permanent field, T, solve, energies, forces.

Paper, technical appendix (Polarization): with E the 3N field of the
permanent multipoles (up to quadrupole) at the polarizable sites and T the
polarization matrix (alpha_i^-1 on the diagonal blocks, -T_ij off the
diagonal, symmetric positive definite thanks to Thole damping),
  E_pol = 1/2 mu^T T mu - mu^T E      (Eq. 17)
  T mu  = E                           (Eq. 18)
  E_pol = -1/2 mu^T E  at the solution (Eq. 19).
Energies are reported in kcal/mol (COULOMB * e^2/A).

Electrostatics (Eq. 2) is taken as the plain multipole-multipole energy;
the short-range penetration correction is not part of this path.

Methods:
  'direct'  gas-phase cluster, bare Coulomb over all pairs, no cutoff;
  'ewald'   periodic, Ewald real space (minimum image within a cutoff, or all
            images within rmax) plus the brute-force k-sum;
  'spme'    periodic, Ewald real space under minimum image within the
            cutoff plus Smooth PME.
Ewald self terms (Taylor expansion of erf(beta r)/r at r = 0):
  E_self = -sum_i [beta/sqrt(pi) q_i^2 + 2 beta^3/(3 sqrt(pi)) |d_i|^2
                   + 8 beta^5/(45 sqrt(pi)) Theta_i:Theta_i],
  self field of a site's own dipole: +4 beta^3/(3 sqrt(pi)) d_i.
Tin-foil boundary; molecules are neutral, so no background term.

Forces are -dE_tot/dr at fixed mu, E_tot = E_elec + E_pol.  Because mu
makes E_pol stationary, this is the full gradient.  The reciprocal part is
taken as the reciprocal energy of the combined density (q, d + mu, Theta).
"""
import dataclasses
import math
from typing import Optional

import numpy as np

from . import realspace as rs
from . import recip
from . import solver as sv
from .solver import pcg
from .units import COULOMB


def _quad_tensor(quad6):
    xx, xy, xz, yy, yz, zz = quad6.T
    return np.stack([np.stack([xx, xy, xz], -1),
                     np.stack([xy, yy, yz], -1),
                     np.stack([xz, yz, zz], -1)], -2)


@dataclasses.dataclass
class System:
    pos: np.ndarray
    mol: np.ndarray
    q: np.ndarray
    dip: np.ndarray
    quad: np.ndarray            # (n,6) xx,xy,xz,yy,yz,zz
    alpha: np.ndarray           # (n,6) xx,xy,xz,yy,yz,zz
    box: Optional[np.ndarray] = None
    thole: Optional[np.ndarray] = None   # per-site a; None -> Params.thole_a

    @classmethod
    def from_dict(cls, d, thole=None):
        return cls(pos=np.asarray(d["pos"], float), mol=np.asarray(d["mol"]),
                   q=np.asarray(d["q"], float), dip=np.asarray(d["dip"], float),
                   quad=np.asarray(d["quad"], float),
                   alpha=np.asarray(d["alpha"], float),
                   box=None if d.get("box") is None else np.asarray(d["box"], float),
                   thole=thole)

    @property
    def n(self):
        return len(self.pos)

    @property
    def th(self):
        return _quad_tensor(self.quad)

    @property
    def alpha3(self):
        return _quad_tensor(self.alpha)

    @property
    def pol(self):
        """Indices of polarizable sites (nonzero polarizability)."""
        return np.flatnonzero(np.any(self.alpha != 0.0, axis=1))

    @property
    def abar(self):
        return (self.alpha[:, 0] + self.alpha[:, 3] + self.alpha[:, 5]) / 3.0


@dataclasses.dataclass
class Params:
    method: str = "direct"          # 'direct' | 'ewald' | 'spme'
    beta: float = 0.4
    cutoff: float = 9.0
    grid: tuple = (32, 32, 32)
    order: int = 5
    realspace: str = "minimage"     # ewald: 'minimage' | 'images'
    rmax: float = 14.0              # ewald 'images' real-space radius
    thole_a: float = 0.28
    tol: float = 1e-8               # Debye, RMS of alpha r
    max_iter: int = 200
    mumu_intramolecular: bool = True  # False: the variant excluding them
    precond: str = "diag"           # 'diag' (alpha per site) | 'molblock'

    @property
    def periodic(self):
        return self.method != "direct"


class Context:
    """Pairs and per-site arrays prepared once per (system, params)."""

    def __init__(self, sysm: System, prm: Params, subset=None):
        self.s = sysm
        self.p = prm
        a = sysm.thole if sysm.thole is not None else np.full(sysm.n, prm.thole_a)
        self.thole = (sysm.abar, np.asarray(a, float))
        self.kernel = "bare" if prm.method == "direct" else "ewald"
        if prm.method == "direct":
            self.pairs = rs.pairs_cluster(sysm.pos, sysm.mol)
        elif prm.method == "ewald" and prm.realspace == "images":
            self.pairs = rs.pairs_images(sysm.pos, sysm.mol, sysm.box, prm.rmax)
        else:
            self.pairs = rs.pairs_min_image(sysm.pos, sysm.mol, sysm.box,
                                            prm.cutoff, subset=subset)
        self.pol = sysm.pol
        self.is_pol = np.zeros(sysm.n, bool)
        self.is_pol[self.pol] = True
        self.mumu_cls = "mumu" if prm.mumu_intramolecular else "mumu_excl"

    # -- reciprocal-space helpers ---------------------------------------
    def recip_derivs(self, mult, at, nderiv):
        s, p = self.s, self.p
        if p.method == "ewald":
            return recip.ewald_recip(s.pos, s.box, p.beta, mult, at, nderiv)
        K = np.broadcast_to(np.asarray(p.grid, int), (3,))
        grid = recip.spme_spread(s.pos, s.box, K, p.order, mult)
        G = recip.spme_influence(s.box, K, p.order, p.beta)
        energy, phi = recip.spme_potential(grid, G)
        return energy, recip.spme_gather(at, s.box, K, p.order, phi, nderiv)

    def self_field_coef(self):
        b = self.p.beta
        return 4.0 * b ** 3 / (3.0 * math.sqrt(math.pi))

    def full(self, v_pol):
        out = np.zeros((self.s.n, 3))
        out[self.pol] = v_pol
        return out


def _ctx(sysm, prm, ctx=None, subset=None):
    return ctx if ctx is not None else Context(sysm, prm, subset=subset)


def permanent_field(sysm, prm, ctx=None, sites=None):
    """E at the polarizable sites (N_pol,3) in e/A^2, or at `sites` (a subset
    of polarizable site indices) when given."""
    c = _ctx(sysm, prm, ctx, subset=sites)
    s = c.s
    targets = c.pol if sites is None else np.asarray(sites, int)
    tmask = np.zeros(s.n, bool)
    tmask[targets] = True
    mult = (s.q, s.dip, s.th)
    E = rs.pair_sum(c.pairs, "Mmu", c.kernel, prm.beta, c.thole,
                    (None, None, None), mult, "field", s.n,
                    pair_mask=tmask[c.pairs.i])[targets]
    if prm.periodic:
        _, der = c.recip_derivs(mult, s.pos[targets], 1)
        E = E - der[1]
        E = E + c.self_field_coef() * s.dip[targets]
    return E


def apply_T(sysm, prm, p_pol, ctx=None, sites=None):
    """T p for p on all polarizable sites; rows for `sites` if given."""
    c = _ctx(sysm, prm, ctx, subset=sites)
    s = c.s
    targets = c.pol if sites is None else np.asarray(sites, int)
    tmask = np.zeros(s.n, bool)
    tmask[targets] = True
    pf = c.full(p_pol)
    mask = tmask[c.pairs.i] & c.is_pol[c.pairs.j]
    field = rs.pair_sum(c.pairs, c.mumu_cls, c.kernel, prm.beta, c.thole,
                        (None, None, None), (None, pf, None), "field", s.n,
                        pair_mask=mask)[targets]
    if prm.periodic:
        _, der = c.recip_derivs((None, pf, None), s.pos[targets], 1)
        field = field - der[1]
        field = field + c.self_field_coef() * pf[targets]
    a3 = s.alpha3[targets]
    ainv_p = np.linalg.solve(a3, pf[targets][:, :, None])[:, :, 0]
    return ainv_p - field


def precond(sysm, r_pol):
    a3 = sysm.alpha3[sysm.pol]
    return np.einsum("nab,nb->na", a3, r_pol)


MAX_BLOCK_SITES = 4   # molecules with more polarizable sites keep alpha per site


def molblock_inverses(sysm, prm, ctx=None):
    """The molecular block preconditioner: for every molecule with at most
    MAX_BLOCK_SITES polarizable sites, the inverse of its block of T in the
    bare (unscreened) form -- alpha_i^-1 on the diagonal, minus the
    Thole-damped field tensor of a unit dipole between two sites of the
    molecule off it (the mumu class, bare kernel).  For a cluster that is
    exactly the molecule's block of T; in a box the molecule's periodic
    images and the Ewald self terms are left out, which only changes how
    well it preconditions.  A block that is not positive definite, and every
    larger molecule, falls back to alpha per site.  Returns a list of
    (polarizable indices, inverse (3k, 3k))."""
    from .tensors import deriv_tensor
    c = _ctx(sysm, prm, ctx)
    s = c.s
    pol = c.pol
    mol = s.mol[pol]
    a3 = s.alpha3[pol]
    abar, at = c.thole
    out = []
    for m in np.unique(mol):
        idx = np.flatnonzero(mol == m)
        k = len(idx)
        if k > MAX_BLOCK_SITES:
            out += [(np.array([t]), a3[t]) for t in idx]
            continue
        M = np.zeros((k, 3, k, 3))
        for u in range(k):
            M[u, :, u, :] = np.linalg.inv(a3[idx[u]])
        if k > 1:
            uu, vv = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
            off = uu != vv
            uu, vv = uu[off], vv[off]
            i, j = pol[idx[uu]], pol[idx[vv]]
            R = s.pos[i] - s.pos[j]
            r = np.linalg.norm(R, axis=1)
            coef = rs.class_coefficients(c.mumu_cls, r, np.ones(len(r), bool), "bare", prm.beta,
                                         abar[i], abar[j], np.minimum(at[i], at[j]), 2)
            D2 = deriv_tensor(2, R, coef)     # field of a unit dipole at j seen at i
            for n_, (u, v) in enumerate(zip(uu, vv)):
                M[u, :, v, :] = -D2[n_]
        M = M.reshape(3 * k, 3 * k)
        try:
            np.linalg.cholesky(M)
        except np.linalg.LinAlgError:
            out += [(np.array([t]), a3[t]) for t in idx]
            continue
        out.append((idx, np.linalg.inv(M)))
    return out


def precond_blocks(blocks, r_pol):
    z = np.zeros_like(r_pol)
    for idx, Minv in blocks:
        z[idx] = (Minv @ r_pol[idx].ravel()).reshape(-1, 3)
    return z


def dense_T_columns(sysm, prm, ctx=None):
    """Dense 3N_pol x 3N_pol T assembled column by column from apply_T."""
    c = _ctx(sysm, prm, ctx)
    n3 = 3 * len(c.pol)
    T = np.zeros((n3, n3))
    for k in range(n3):
        e = np.zeros(n3)
        e[k] = 1.0
        T[:, k] = apply_T(sysm, prm, e.reshape(-1, 3), ctx=c).ravel()
    return T


def dense_T_blocks(sysm, prm, ctx=None):
    """Dense T assembled block by block: alpha_i^-1 on the diagonal and
    minus the field tensor of a unit dipole at j seen at i off it (real
    space: the second derivative tensor of the class kernel; reciprocal:
    -(4 pi/V) sum_m exp(-pi^2 m^2/beta^2)/m^2 m m cos(2 pi m.(r_i - r_j));
    plus the Ewald self field on the diagonal).  Direct and brute-force
    Ewald only."""
    from .tensors import deriv_tensor
    c = _ctx(sysm, prm, ctx)
    s = c.s
    pol = c.pol
    loc = -np.ones(s.n, int)
    loc[pol] = np.arange(len(pol))
    npol = len(pol)
    T = np.zeros((npol, 3, npol, 3))
    a3 = s.alpha3
    for k, i in enumerate(pol):
        T[k, :, k, :] = np.linalg.inv(a3[i])
    pr = c.pairs
    mask = c.is_pol[pr.i] & c.is_pol[pr.j]
    idx = np.flatnonzero(mask)
    R = pr.R[idx]
    r = np.linalg.norm(R, axis=1)
    ii, jj = pr.i[idx], pr.j[idx]
    abar, at = c.thole
    coef = rs.class_coefficients(c.mumu_cls, r, pr.same[idx], c.kernel,
                                 prm.beta, abar[ii], abar[jj],
                                 np.minimum(at[ii], at[jj]), 2)
    D2 = deriv_tensor(2, R, coef)          # field of unit dipole: E = D2 p
    for n_, (i, j) in enumerate(zip(ii, jj)):
        T[loc[i], :, loc[j], :] -= D2[n_]
    if prm.periodic:
        if prm.method != "ewald":
            raise ValueError("block assembly needs brute-force Ewald")
        box = s.box
        V = recip.cell_volume(box)
        m, m2 = recip.kvectors(box, prm.beta)
        w = np.exp(-np.pi ** 2 * m2 / prm.beta ** 2) / m2
        P = s.pos[pol]
        for a in range(npol):
            dr = P[a] - P
            cosv = np.cos(2 * np.pi * (dr @ m.T))          # (npol, M)
            blk = -(4 * np.pi / V) * np.einsum("km,m,ma,mb->kab", cosv, w, m, m)
            T[a, :, :, :] -= np.transpose(blk, (1, 0, 2))
            T[a, :, a, :] -= c.self_field_coef() * np.eye(3)
    return T.reshape(3 * npol, 3 * npol)


def electrostatic_energy(sysm, prm, ctx=None):
    """Plain multipolar E_elec (kcal/mol): MM real-space pairs, plus the
    reciprocal and self terms when periodic."""
    c = _ctx(sysm, prm, ctx)
    s = c.s
    mult = (s.q, s.dip, s.th)
    e = rs.pair_sum(c.pairs, "MM", c.kernel, prm.beta, c.thole, mult, mult,
                    "energy", s.n)
    if prm.periodic:
        erec, _ = c.recip_derivs(mult, s.pos[:1], 0)
        b = prm.beta
        th = s.th
        eself = -np.sum(b / math.sqrt(math.pi) * s.q ** 2
                        + 2 * b ** 3 / (3 * math.sqrt(math.pi)) * np.sum(s.dip ** 2, 1)
                        + 8 * b ** 5 / (45 * math.sqrt(math.pi)) * np.sum(th * th, (1, 2)))
        e = e + erec + eself
    return COULOMB * e


def energy_forces(sysm, prm, mu_pol, E0, ctx=None, sites=None):
    """(E_pol, E_pol_var, E_elec, forces (n,3) or rows of `sites`)."""
    c = _ctx(sysm, prm, ctx, subset=sites)
    s = c.s
    targets = np.arange(s.n) if sites is None else np.asarray(sites, int)
    tmask = np.zeros(s.n, bool)
    tmask[targets] = True
    pm = tmask[c.pairs.i]
    mult = (s.q, s.dip, s.th)
    muf = c.full(mu_pol)
    mud = (None, muf, None)
    F = rs.pair_sum(c.pairs, "MM", c.kernel, prm.beta, c.thole, mult, mult,
                    "force", s.n, pair_mask=pm)
    F += rs.pair_sum(c.pairs, "Mmu", c.kernel, prm.beta, c.thole, mud, mult,
                     "force", s.n, pair_mask=pm)
    F += rs.pair_sum(c.pairs, "Mmu", c.kernel, prm.beta, c.thole, mult, mud,
                     "force", s.n, pair_mask=pm)
    F += rs.pair_sum(c.pairs, c.mumu_cls, c.kernel, prm.beta, c.thole, mud,
                     mud, "force", s.n, pair_mask=pm)
    F = F[targets]
    if prm.periodic:
        comb = (s.q, s.dip + muf, s.th)
        _, der = c.recip_derivs(comb, s.pos[targets], 3)
        qv = s.q[targets]
        dv = (s.dip + muf)[targets]
        tv = s.th[targets]
        F = F - (qv[:, None] * der[1] + np.einsum("nb,nab->na", dv, der[2])
                 + np.einsum("nbc,nabc->na", tv, der[3]) / 3.0)
    F = COULOMB * F
    if sites is not None:
        return None, None, None, F
    e_pol = -0.5 * COULOMB * float(np.sum(mu_pol * E0))
    Tmu = apply_T(sysm, prm, mu_pol, ctx=c)
    e_var = COULOMB * (0.5 * float(np.sum(mu_pol * Tmu)) - float(np.sum(mu_pol * E0)))
    e_elec = electrostatic_energy(sysm, prm, ctx=c)
    return e_pol, e_var, e_elec, F


def virial(sysm, prm, mu_pol, ctx=None):
    """Virial W (3,3, kcal/mol): W_ab = -dE_tot/d eps_ab for the homogeneous
    strain r -> (1 + eps) r of every site (and of the cell when periodic),
    with the multipoles, polarizabilities and mu fixed in the global frame.
    mu is stationary, so at the solution this is the full strain derivative,
    as the forces are the full gradient.  Real space: the pair energies of
    the MM, Mmu and mumu classes (the alpha^-1 and self terms do not depend
    on the geometry); reciprocal: the reciprocal energy of the combined
    density (q, d + mu, Theta).  Cutoff pairs are taken as in the energy
    (a pair crossing the cutoff under strain is not followed)."""
    c = _ctx(sysm, prm, ctx)
    s = c.s
    mult = (s.q, s.dip, s.th)
    mud = (None, c.full(mu_pol), None)
    W = rs.pair_sum(c.pairs, "MM", c.kernel, prm.beta, c.thole, mult, mult, "virial", s.n)
    W += rs.pair_sum(c.pairs, "Mmu", c.kernel, prm.beta, c.thole, mud, mult, "virial", s.n)
    W += rs.pair_sum(c.pairs, "Mmu", c.kernel, prm.beta, c.thole, mult, mud, "virial", s.n)
    W += rs.pair_sum(c.pairs, c.mumu_cls, c.kernel, prm.beta, c.thole, mud, mud, "virial",
                     s.n)
    if prm.periodic:
        comb = (s.q, s.dip + mud[1], s.th)
        if prm.method == "ewald":
            _, Wr = recip.ewald_recip_virial(s.pos, s.box, prm.beta, comb)
        else:
            K = np.broadcast_to(np.asarray(prm.grid, int), (3,))
            _, Wr = recip.spme_virial(s.pos, s.box, K, prm.order, prm.beta, comb)
        W = W + Wr
    return COULOMB * W


def solve(sysm, prm, E0, ctx=None, x0=None):
    """PCG for T mu = E0.  The tolerance always measures alpha r (Debye RMS),
    whichever preconditioner runs."""
    c = _ctx(sysm, prm, ctx)
    mv = lambda v: apply_T(sysm, prm, v, ctx=c)
    measure = lambda r: precond(sysm, r)
    if prm.precond == "molblock":
        blocks = molblock_inverses(sysm, prm, c)
        pc = lambda r: precond_blocks(blocks, r)
    else:
        pc = measure
    if x0 is None:
        x0 = pc(E0)
    return pcg(mv, pc, E0, x0, prm.tol, prm.max_iter, measure=measure)


def tcg(sysm, prm, E0, order, omega=0.0, ctx=None, x0=None):
    """TCG-n dipoles from the guess x0 (default the direct field alpha E0),
    with the optional peek step (see solver.tcg), and E_pol at them in the
    form of Eq. 19.  Returns (mu, E_pol)."""
    c = _ctx(sysm, prm, ctx)
    mv = lambda v: apply_T(sysm, prm, v, ctx=c)
    pc = lambda r: precond(sysm, r)
    mu = sv.tcg(mv, pc, E0, pc(E0) if x0 is None else x0, order, omega)
    return mu, -0.5 * COULOMB * float(np.sum(mu * E0))


def tcg_energy(sysm, prm, order, omega=0.0, x0=None):
    """E_elec + E_pol at the TCG-n dipoles (kcal/mol), the guess x0 (the
    polarizable rows) held fixed, or the direct field alpha E0 of this
    geometry.  Its derivatives, taken by central differences in the tests,
    are the oracle's TCG forces (the analytic TCG derivative is given only
    in the work the paper cites)."""
    c = Context(sysm, prm)
    E0 = permanent_field(sysm, prm, ctx=c)
    _, e_pol = tcg(sysm, prm, E0, order, omega, ctx=c, x0=x0)
    return electrostatic_energy(sysm, prm, ctx=c) + e_pol


def evaluate(sysm, prm, forces=True, with_virial=False):
    """Full evaluation: E0 -> PCG -> energies -> forces (fixed mu), and the
    virial when asked."""
    c = Context(sysm, prm)
    E0 = permanent_field(sysm, prm, ctx=c)
    mu, iters, rho = solve(sysm, prm, E0, ctx=c)
    out = dict(E0=E0, mu=mu, iters=iters, rho=rho)
    if with_virial:
        out["virial"] = virial(sysm, prm, mu, ctx=c)
    if forces:
        e_pol, e_var, e_elec, F = energy_forces(sysm, prm, mu, E0, ctx=c)
        out.update(E_pol=e_pol, E_pol_var=e_var, E_elec=e_elec, forces=F)
    else:
        out["E_pol"] = -0.5 * COULOMB * float(np.sum(mu * E0))
        out["E_elec"] = electrostatic_energy(sysm, prm, ctx=c)
    return out
