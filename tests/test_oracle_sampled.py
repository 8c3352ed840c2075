"""The oracle's sampled-row mode equals the rows of its full evaluation.

At the 4,096-, 32,000- and 96,000-water sizes the GPU path is checked
against the oracle on sampled rows only: permanent_field, apply_T and
energy_forces take `sites=` and build their pair list only for pairs that
start at those sites (a ball query per site instead of the all-pairs
query).  The full evaluation is the one pinned by P1-P12; these tests tie
the sampled mode to it, row by row, on boxes small enough to evaluate in
full.  Rows include sites next to the box faces (pairs across the periodic
boundary) and every site of one molecule (the same-molecule pairs that the
sampled list adds by hand).
"""
import numpy as np
import pytest

from oracle.model import System, Params, Context, permanent_field, apply_T, energy_forces
from synth import water_box, config_system


def _rows(s, rng, k):
    """k random sites, plus the sites nearest each box face and all sites of
    molecule 0, sorted and unique."""
    w = np.mod(s.pos, s.box)
    edge = list(np.argmin(w, axis=0)) + list(np.argmax(w, axis=0))
    mol0 = list(np.flatnonzero(s.mol == s.mol[0]))
    pick = list(rng.choice(s.n, k, replace=False))
    return np.unique(np.asarray(pick + edge + mol0, int))


def _check(sysd, kw, seed):
    s = System.from_dict(sysd)
    p = Params(method="spme", tol=1e-10, **kw)
    c = Context(s, p)
    rng = np.random.default_rng(seed)
    E = permanent_field(s, p, ctx=c)
    pv = rng.standard_normal(E.shape)
    Tp = apply_T(s, p, pv, ctx=c)
    mu = 0.1 * rng.standard_normal(E.shape)
    _, _, _, F = energy_forces(s, p, mu, E, ctx=c)

    rows = _rows(s, rng, 12)
    is_pol = np.zeros(s.n, bool)
    is_pol[s.pol] = True
    sub_pol = rows[is_pol[rows]]
    loc = -np.ones(s.n, int)
    loc[s.pol] = np.arange(len(s.pol))
    assert len(sub_pol) >= 6

    Es = permanent_field(s, p, sites=sub_pol)
    Tps = apply_T(s, p, pv, sites=sub_pol)
    _, _, _, Fs = energy_forces(s, p, mu, E, sites=rows)
    # the same pairs in the same order: equal to rounding at most
    assert np.abs(Es - E[loc[sub_pol]]).max() <= 1e-14 * np.abs(E).max()
    assert np.abs(Tps - Tp[loc[sub_pol]]).max() <= 1e-14 * np.abs(Tp).max()
    assert np.abs(Fs - F[rows]).max() <= 1e-14 * np.abs(F).max()


def test_sampled_rows_27_water_box():
    _check(water_box(27, 9.5, 3), dict(beta=0.45, cutoff=4.5, grid=(24,) * 3, order=5), 0)


def test_sampled_rows_box216():
    d, k = config_system("box216")
    _check(d, dict(beta=k["beta"], cutoff=k["cutoff"], grid=(k["grid"],) * 3,
                   order=k["order"]), 1)


def test_sampled_rows_need_the_subset():
    """A planted mistake of the kind the sampled mode could make -- losing
    the same-molecule pairs of its rows -- changes the rows by far more than
    the bar above, so the comparison can see it."""
    sysd = water_box(27, 9.5, 3)
    s = System.from_dict(sysd)
    p = Params(method="spme", tol=1e-10, beta=0.45, cutoff=4.5, grid=(24,) * 3, order=5)
    rows = np.flatnonzero(s.mol == s.mol[0])
    pol_rows = rows[np.isin(rows, s.pol)]
    rng = np.random.default_rng(2)
    pv = rng.standard_normal((len(s.pol), 3))
    full = apply_T(s, p, pv, sites=pol_rows)
    c = Context(s, p, subset=pol_rows)
    keep = ~c.pairs.same
    for name in ("i", "j", "same"):
        setattr(c.pairs, name, getattr(c.pairs, name)[keep])
    c.pairs.R = c.pairs.R[keep]
    broken = apply_T(s, p, pv, ctx=c, sites=pol_rows)
    assert np.abs(broken - full).max() > 1e-3 * np.abs(full).max()
