"""The oracle's TCG forces are central differences of its TCG energy
(model.tcg_energy; the TCG iterate itself is pinned by P12).  Pinned here:
at an order equal to the number of unknowns TCG is the exact solve, so the
differences reproduce the analytic converged forces of energy_forces; at
low orders they do not (the fixed-dipole identity fails there)."""
import numpy as np
import pytest

import oracle
from oracle.model import System, Params, tcg_energy
from synth import water_cluster


def _fd(s, prm, order, omega, sites, h=1e-5, x0=None):
    out = []
    for i, a in sites:
        p = s.pos.copy()
        p[i, a] += h
        ep = tcg_energy(System(**{**s.__dict__, "pos": p}), prm, order, omega, x0)
        p[i, a] -= 2 * h
        em = tcg_energy(System(**{**s.__dict__, "pos": p}), prm, order, omega, x0)
        out.append(-(ep - em) / (2 * h))
    return np.array(out)


def test_full_order_tcg_forces_are_the_converged_forces():
    d = water_cluster(2, 3)
    s = System.from_dict(d)
    prm = Params(method="direct", tol=1e-13)
    n_unknowns = 3 * len(s.pol)
    ref = oracle.evaluate(s, prm)["forces"]
    sites = [(0, 0), (1, 2), (3, 1), (6, 0), (8, 2)]
    fd = _fd(s, prm, n_unknowns, 0.0, sites)
    exact = np.array([ref[i, a] for i, a in sites])
    assert np.abs(fd - exact).max() < 1e-6 * np.abs(ref).max()
    fd1 = _fd(s, prm, 1, 0.0, sites)
    assert np.abs(fd1 - exact).max() > 1e-4 * np.abs(ref).max()
