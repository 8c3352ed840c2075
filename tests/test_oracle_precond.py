"""Pins of the molecular block preconditioner (oracle/model.py
molblock_inverses, solve with precond='molblock').

B1  For a cluster each molecule's block of the preconditioner equals that
    molecule's block of the dense T assembled block by block
    (dense_T_blocks), and the inverses are inverses.
B2  PCG with the block preconditioner converges to the dense solution of
    T mu = E0 (cluster and brute-force Ewald box), with the tolerance still
    measured on alpha r, and in fewer iterations than alpha per site.
B3  Degenerate cases reduce to alpha per site, iterate for iterate: a
    molecule with more than MAX_BLOCK_SITES polarizable sites, and T
    without intramolecular pairs (mumu_intramolecular=False).
B1 and B2 also run on molecules of 1, 2, 4 and 6 polarizable sites
(mixed_molecules), which exercises every block size and the fallback.
"""
import dataclasses

import numpy as np
import pytest

from oracle import model as om
from oracle.model import System, Params, Context
from synth import water_cluster, water_box


def mixed_molecules(d):
    """Water sites regrouped into molecules of 1, 2, 3, 4 and 6 polarizable
    sites (sites O, H1, H2, B1, B2 per water; O, B1 and B2 polarizable)."""
    mol = np.asarray(d["mol"]).copy()
    nw = len(mol) // 5
    assert nw >= 5
    mol[5:10] = mol[0]                 # waters 0 and 1: one molecule, 6 polarizable sites
    mol[10] = nw                       # water 2: O alone (1) and B1, B2 (2)
    mol[11] = nw                       # ... the O keeps one hydrogen
    mol[5 * 3 + 3] = mol[5 * 4]        # B1 of water 3 joins water 4 (4); water 3 keeps 2
    return dict(d, mol=mol)


def _dense_solution(s, prm):
    c = Context(s, prm)
    T = om.dense_T_blocks(s, prm, c)
    E0 = om.permanent_field(s, prm, c)
    return c, T, E0


@pytest.mark.parametrize("regroup", [False, True])
def test_b1_blocks_equal_the_molecular_blocks_of_T_for_a_cluster(regroup):
    d = water_cluster(6, 3)
    s = System.from_dict(mixed_molecules(d) if regroup else d)
    prm = Params(method="direct")
    c, T, _ = _dense_solution(s, prm)
    blocks = om.molblock_inverses(s, prm, c)
    assert sum(len(idx) for idx, _ in blocks) == len(c.pol)
    if regroup:
        assert sorted({len(idx) for idx, _ in blocks}) == [1, 2, 3, 4]
    for idx, Minv in blocks:
        ii = np.concatenate([[3 * k, 3 * k + 1, 3 * k + 2] for k in idx])
        Tb = T[np.ix_(ii, ii)]
        assert np.abs(Minv @ Tb - np.eye(len(ii))).max() < 1e-12
        assert np.abs(Tb - np.linalg.inv(Minv)).max() < 1e-10 * np.abs(Tb).max()


def _iterations(s, prm):
    c, T, E0 = _dense_solution(s, prm)
    mu_ref = np.linalg.solve(T, E0.ravel()).reshape(-1, 3)
    x, it, rho = om.solve(s, prm, E0, ctx=c)
    return x, it, rho, mu_ref


def test_b2_converges_to_the_dense_solution_in_fewer_iterations():
    for d, prm in [(water_cluster(12, 5), Params(method="direct", tol=1e-9)),
                   (mixed_molecules(water_cluster(12, 5)), Params(method="direct", tol=1e-9)),
                   (water_box(27, 9.5, 3), Params(method="ewald", beta=0.45, realspace="images",
                                                  rmax=9.5, tol=1e-9))]:
        s = System.from_dict(d)
        xd, itd, rhod, mu_ref = _iterations(s, prm)
        xb, itb, rhob, _ = _iterations(s, dataclasses.replace(prm, precond="molblock"))
        assert rhob <= prm.tol and rhod <= prm.tol
        scale = np.abs(mu_ref).max()
        assert np.abs(xb - mu_ref).max() <= 1e-7 * scale
        assert np.abs(xd - mu_ref).max() <= 1e-7 * scale
        assert itb < itd, (itb, itd)


def test_b3_degenerate_cases_reduce_to_alpha_per_site():
    d = water_cluster(4, 2)
    prm = Params(method="direct")
    # one molecule of 12 polarizable sites: more than MAX_BLOCK_SITES
    d1 = dict(d, mol=np.zeros_like(d["mol"]))
    for dd, p in [(d1, prm), (d, dataclasses.replace(prm, mumu_intramolecular=False))]:
        s = System.from_dict(dd)
        c = Context(s, p)
        E0 = om.permanent_field(s, p, c)
        xd, itd, _ = om.solve(s, p, E0, ctx=c)
        xb, itb, _ = om.solve(s, dataclasses.replace(p, precond="molblock"), E0, ctx=c)
        assert itb == itd
        assert np.abs(xb - xd).max() <= 1e-13 * np.abs(xd).max()
