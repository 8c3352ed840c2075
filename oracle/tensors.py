"""Cartesian derivative tensors of a radial kernel, built from pairings.

For G(R) = c_0(|R|) with c_{n+1} = -c_n'/r, the n-th derivative tensor is
  d^n G / dR_a1..dR_an = sum over all partitions of {a1..an} into p
      disjoint index pairs and s = n - 2p singletons of
      (-1)^(n-p) c_{n-p} * prod(delta over pairs) * prod(R over singletons).
(Each derivative either differentiates a radial factor, which brings
-R_a and raises its order, or an existing R_b, which turns it into a delta.)

The multipole convention (Buckingham traceless quadrupole) used with these
tensors: the potential of site j at R = r - r_j is
  phi_j = [q_j - d_j.grad + 1/3 Theta_j : grad grad] G(R),
and the energy of site i in that potential is
  U = [q_i + d_i.grad + 1/3 Theta_i : grad grad] phi_j(R = r_i - r_j).
"""
import functools
import string

import numpy as np

WEIGHT = (1.0, 1.0, 1.0 / 3.0)   # multipole operator weights by rank


@functools.lru_cache(maxsize=None)
def pairings(n):
    """All (pairs, singles) partitions of range(n)."""
    def rec(items):
        if not items:
            return [((), ())]
        first, rest = items[0], items[1:]
        out = []
        for pairs, singles in rec(rest):
            out.append((pairs, (first,) + singles))
        for k, other in enumerate(rest):
            remaining = rest[:k] + rest[k + 1:]
            for pairs, singles in rec(remaining):
                out.append((((first, other),) + pairs, singles))
        return out
    return tuple(rec(tuple(range(n))))


def deriv_tensor(n, R, c):
    """d^n G/dR^n for P pairs: R (P,3), c list of (P,) arrays -> (P,3,...,3)."""
    P = R.shape[0]
    if n == 0:
        return c[0].copy()
    eye = np.eye(3)
    out = np.zeros((P,) + (3,) * n)
    for pairs, singles in pairings(n):
        p = len(pairs)
        term = ((-1.0) ** (n - p) * c[n - p]).reshape((P,) + (1,) * n)
        for (x, y) in pairs:          # delta_{a_x a_y}, broadcast
            shape = [1] * (n + 1)
            shape[1 + x] = 3
            shape[1 + y] = 3
            term = term * eye.reshape(shape)
        for s in singles:             # R_{a_s}, broadcast
            shape = [P] + [1] * n
            shape[1 + s] = 3
            term = term * R.reshape(shape)
        out += term
    return out


def contract_leading(D, mults):
    """Contract the leading indices of D (P,3^n) with per-pair multipole
    tensors (each (P,), (P,3) or (P,3,3)); return the remaining (P,3^m)."""
    n = D.ndim - 1
    letters = string.ascii_lowercase[:n]
    subs_d = "Z" + letters
    pos = 0
    subs = [subs_d]
    ops = [D]
    for m in mults:
        rank = m.ndim - 1
        subs.append("Z" + letters[pos:pos + rank])
        ops.append(m)
        pos += rank
    out = "Z" + letters[pos:]
    return np.einsum(",".join(subs) + "->" + out, *ops)


def multipole_list(q, d, th):
    """[(rank, weight, tensor)] for the nonzero parts of a multipole set."""
    out = []
    if q is not None:
        out.append((0, q))
    if d is not None:
        out.append((1, d))
    if th is not None:
        out.append((2, th))
    return out
