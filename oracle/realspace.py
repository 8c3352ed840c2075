"""Real-space pair sums: enumeration of site pairs and class coefficients.

Pairs are ORDERED (i, j, R = r_i - r_j - image shift): per-site quantities
at i sum over every pair starting at i, and energies are half the sum over
all ordered pairs.

Interaction classes (exclusion reading: the paper's T lists a block for every
pair of distinct sites, and E_pol and E_elec are intermolecular terms):
  MM   permanent-permanent (E_elec):     s = 0 for same-molecule pairs,
       undamped;
  Mmu  permanent-induced (field E, mu-permanent forces): s = 0 for
       same-molecule pairs, Thole-damped;
  mumu induced-induced (T): s = 1 for every pair of distinct sites, same
       molecule included, Thole-damped.
Same-molecule exclusion applies to the unshifted (nearest) image only.

Radial coefficients per class, with lambda the Thole factors (1 for MM):
  cluster (bare Coulomb, no cutoff):      c_n = s lambda_{2n+1} c0_n
  periodic (Ewald real space):            c_n = B_n - (1 - s lambda_{2n+1}) c0_n
The periodic form puts back into real space the part of the bare
interaction that the reciprocal sum includes but the class excludes or
damps.
"""
import numpy as np
from scipy.spatial import cKDTree

from . import radial
from .tensors import WEIGHT, deriv_tensor, contract_leading

CHUNK = 2048


class PairSet:
    """Ordered pairs (i, j, R, same)."""

    def __init__(self, i, j, R, same):
        self.i = np.asarray(i, dtype=np.int64)
        self.j = np.asarray(j, dtype=np.int64)
        self.R = np.asarray(R, dtype=float).reshape(-1, 3)
        self.same = np.asarray(same, dtype=bool)

    def __len__(self):
        return len(self.i)


def pairs_cluster(pos, mol):
    n = len(pos)
    ii, jj = np.nonzero(~np.eye(n, dtype=bool))
    R = pos[ii] - pos[jj]
    return PairSet(ii, jj, R, mol[ii] == mol[jj])


def _min_image(d, box):
    return d - box * np.round(d / box)


def pairs_min_image(pos, mol, box, cutoff, subset=None):
    """Ordered pairs within the cutoff under minimum image, plus every
    same-molecule pair (excluded pairs are needed whatever their distance).
    With subset given, only pairs whose first site is in the subset."""
    box = np.asarray(box, float)
    if cutoff >= 0.5 * box.min():
        raise ValueError("cutoff must be below half the box")
    n = len(pos)
    wrapped = np.mod(pos, box)
    tree = cKDTree(wrapped, boxsize=box)
    if subset is None:
        up = tree.query_pairs(cutoff, output_type="ndarray")
        ii = [up[:, 0], up[:, 1]] if len(up) else [np.zeros(0, int)] * 2
        jj = [up[:, 1], up[:, 0]] if len(up) else [np.zeros(0, int)] * 2
        first = np.arange(n)
    else:
        first = np.asarray(subset, int)
        lists = tree.query_ball_point(wrapped[first], cutoff)
        ii = [np.repeat(first, [len(l) for l in lists])]
        jj = [np.concatenate([np.asarray(l, int) for l in lists])]
    # same-molecule pairs (deduplicated below)
    in_first = np.zeros(n, bool)
    in_first[first] = True
    order = np.argsort(mol, kind="stable")
    ms = mol[order]
    starts = np.flatnonzero(np.r_[True, ms[1:] != ms[:-1]])
    ends = np.r_[starts[1:], n]
    extra_i, extra_j = [], []
    for s, e in zip(starts, ends):
        idx = order[s:e]
        for a in idx:
            if not in_first[a]:
                continue
            for b in idx:
                extra_i.append(a)
                extra_j.append(b)
    i = np.concatenate(ii + [np.asarray(extra_i, int)])
    j = np.concatenate(jj + [np.asarray(extra_j, int)])
    keep = i != j
    i, j = i[keep], j[keep]
    key = i * n + j
    _, uniq = np.unique(key, return_index=True)
    i, j = i[uniq], j[uniq]
    R = _min_image(pos[i] - pos[j], box)
    return PairSet(i, j, R, mol[i] == mol[j])


def pairs_images(pos, mol, box, rmax):
    """Every ordered (i, j, image) with |R| < rmax, except i == j unshifted.
    For brute-force Ewald on tiny systems.  box: (3,) edge lengths of an
    orthorhombic cell, or (3,3) lattice vectors as rows (any cell)."""
    box = np.asarray(box, float)
    if box.ndim == 2:
        # image n along a_k moves every point by n / |b_k| across the planes
        # of a_k, with b_k the reciprocal vectors (rows of inv(H)^T)
        recip_len = np.linalg.norm(np.linalg.inv(box).T, axis=1)
        nimg = np.ceil(rmax * recip_len).astype(int) + 1
    else:
        nimg = np.ceil(rmax / box).astype(int) + 1
    I, J, RR, S = [], [], [], []
    n = len(pos)
    base = pos[:, None, :] - pos[None, :, :]
    same_mol = mol[:, None] == mol[None, :]
    for a in range(-nimg[0], nimg[0] + 1):
        for b in range(-nimg[1], nimg[1] + 1):
            for c in range(-nimg[2], nimg[2] + 1):
                shift = (np.array([a, b, c]) @ box if box.ndim == 2
                         else np.array([a, b, c]) * box)
                d = base - shift
                r = np.linalg.norm(d, axis=2)
                zero = (a == 0 and b == 0 and c == 0)
                mask = r < rmax
                if zero:
                    mask &= ~np.eye(n, dtype=bool)
                ii, jj = np.nonzero(mask)
                I.append(ii)
                J.append(jj)
                RR.append(d[ii, jj])
                S.append(same_mol[ii, jj] & zero)
    return PairSet(np.concatenate(I), np.concatenate(J),
                   np.concatenate(RR), np.concatenate(S))


def class_coefficients(cls, r, same, kernel, beta, abar_i, abar_j, a_ij, nmax):
    """[c_0..c_nmax] for the interaction class on these pairs."""
    c0 = radial.bare(r, nmax)
    if cls == "intra":   # same-molecule pairs only, bare kernel
        on = np.where(same, 1.0, 0.0)
        return [on * c0[n] for n in range(nmax + 1)]
    if cls == "MM":
        lam = [np.ones_like(r)] * (nmax + 1)
    else:
        lam = radial.thole_lambdas(r, abar_i, abar_j, a_ij, nmax)
    if cls == "mumu":
        s = np.ones_like(r)
    else:  # MM, Mmu, and mumu_excl (the variant that also excludes
        #    same-molecule induced-induced pairs)
        s = np.where(same, 0.0, 1.0)
    if kernel == "bare":
        return [s * lam[n] * c0[n] for n in range(nmax + 1)]
    B = radial.ewald_real(r, beta, nmax)
    return [B[n] - (1.0 - s * lam[n]) * c0[n] for n in range(nmax + 1)]


def _mlist(q, d, th, idx):
    out = []
    if q is not None:
        out.append((0, q[idx]))
    if d is not None:
        out.append((1, d[idx]))
    if th is not None:
        out.append((2, th[idx]))
    return out


def _interaction(D, Mi, Mj, extra):
    total = 0.0
    for ri, ti in Mi:
        for rj, tj in Mj:
            val = contract_leading(D[ri + rj + extra], [ti, tj])
            total = total + WEIGHT[ri] * WEIGHT[rj] * (-1.0) ** rj * val
    return total


def pair_sum(pairs, cls, kernel, beta, thole, Mi, Mj, what, n_sites,
             pair_mask=None):
    """Generic ordered-pair sum.

    Mi, Mj: (q, d, th) tuples of per-site arrays (None entries allowed) for
    the i side and the j side.  thole: (abar, a) per-site arrays.
    what: 'energy' -> 1/2 sum of U over ordered pairs
          'force'  -> per-site force -dU/dr_i summed over pairs at i (n,3)
          'field'  -> per-site field of the j-side multipoles at i (n,3)
          'potential' -> per-site potential of the j-side multipoles at i (n,)
          'fieldgrad' -> per-site field gradient dE_b/dr_a of the j-side
                      multipoles at i (n,3,3), E = -grad phi
          'virial' -> W_ab = -dE/d eps_ab of the pair energy (3,3) under the
                      homogeneous strain R -> (1 + eps) R of every pair
                      separation with the multipoles fixed in the global
                      frame: -1/2 sum over ordered pairs of (dU/dR)_a R_b
    """
    abar, athole = thole
    maxrank_i = max([k for k, v in enumerate(Mi) if v is not None], default=0)
    maxrank_j = max([k for k, v in enumerate(Mj) if v is not None], default=0)
    extra = {"energy": 0, "potential": 0, "fieldgrad": 2}.get(what, 1)
    nmax = maxrank_i + maxrank_j + extra
    if what == "energy":
        acc = 0.0
    elif what == "virial":
        acc = np.zeros((3, 3))
    elif what == "fieldgrad":
        acc = np.zeros((n_sites, 3, 3))
    elif what == "potential":
        acc = np.zeros(n_sites)
    else:
        acc = np.zeros((n_sites, 3))
    sel = np.arange(len(pairs)) if pair_mask is None else np.flatnonzero(pair_mask)
    for s in range(0, len(sel), CHUNK):
        idx = sel[s:s + CHUNK]
        i = pairs.i[idx]
        j = pairs.j[idx]
        R = pairs.R[idx]
        r = np.linalg.norm(R, axis=1)
        a_ij = np.minimum(athole[i], athole[j])
        c = class_coefficients(cls, r, pairs.same[idx], kernel, beta,
                               abar[i], abar[j], a_ij, nmax)
        D = [deriv_tensor(n, R, c) for n in range(nmax + 1)]
        mi = (_mlist(*Mi, i) if what not in ("field", "fieldgrad", "potential")
              else [(0, np.ones(len(i)))])
        mj = _mlist(*Mj, j)
        val = _interaction(D, mi, mj, extra)
        if what == "energy":
            acc += 0.5 * float(np.sum(val))
        elif what == "virial":
            acc -= 0.5 * np.einsum("pa,pb->ab", val, R)
        elif what == "potential":
            np.add.at(acc, i, val)
        else:
            np.add.at(acc, i, -val)
    return acc
