"""Radial coefficient functions c_n(r) of the interaction tensors.

Every Cartesian derivative of a radial kernel G(r) is a sum of products of
Kronecker deltas and components of R with scalar radial factors c_n(r),
where c_0 = G and c_{n+1} = -c_n'(r)/r (see tensors.py).  Three kernels:

  bare Coulomb     c_n = (2n-1)!! / r^(2n+1)
  Ewald real space B_0 = erfc(beta r)/r,
                   B_n = [(2n-1) B_{n-1} + (2 beta^2)^n exp(-beta^2 r^2)
                          / (beta sqrt(pi))] / r^2        (Smith's recursion)
  Thole-damped     c_n = lambda_{2n+1}(r) * bare c_n   (n >= 1)

Thole damping (paper, Many-body Polarization and technical appendix: the
field is damped at short range by Thole's function; recalibrated constant
a = 0.28, Calibration section).  The paper gives no formula, so the oracle
takes the exponential form used by AMOEBA (Thole 1981; Ren & Ponder 2003):
  x = a * u^3,  u = r / (abar_i abar_j)^(1/6),  abar = trace(alpha)/3,
  lambda_3 = 1 - exp(-x).
Higher orders follow from requiring every damped tensor to be the exact
derivative of the damped field, i.e. c_{n+1} = -c_n'/r, which gives
  lambda_{2n+3} = lambda_{2n+1} - r/(2n+1) * d lambda_{2n+1}/dr.
Writing lambda_{2n+1} = 1 - P_n(x) exp(-x) (P_1 = 1) and using
dx/dr = 3x/r this is P_{n+1} = P_n + 3x/(2n+1) * (P_n - P_n').
When abar_i abar_j = 0 (a non-polarizable site) lambda = 1.
"""
import math

import numpy as np
from numpy.polynomial import polynomial as npoly
from scipy.special import erfc


def double_factorial_odd(n):
    """(2n-1)!! with (-1)!! = 1."""
    out = 1
    for k in range(1, 2 * n, 2):
        out *= k
    return out


def bare(r, nmax):
    """List [c_0..c_nmax] of the bare Coulomb kernel 1/r."""
    r = np.asarray(r, dtype=float)
    return [double_factorial_odd(n) / r ** (2 * n + 1) for n in range(nmax + 1)]


def ewald_real(r, beta, nmax):
    """List [B_0..B_nmax] of the screened kernel erfc(beta r)/r."""
    r = np.asarray(r, dtype=float)
    r2 = r * r
    g = np.exp(-beta * beta * r2) / (beta * math.sqrt(math.pi))
    out = [erfc(beta * r) / r]
    for n in range(1, nmax + 1):
        out.append(((2 * n - 1) * out[-1] + (2.0 * beta * beta) ** n * g) / r2)
    return out


def thole_polynomials(nmax):
    """Coefficient arrays of P_1..P_nmax (index n-1), lowest order first."""
    polys = [np.array([1.0])]
    for n in range(1, nmax):
        p = polys[-1]
        dp = npoly.polyder(p) if len(p) > 1 else np.array([0.0])
        diff = npoly.polysub(p, dp)
        nxt = npoly.polyadd(p, npoly.polymulx(diff) * (3.0 / (2 * n + 1)))
        polys.append(nxt)
    return polys


def thole_lambdas(r, abar_i, abar_j, a_ij, nmax):
    """List [lambda_1(=1), lambda_3, ..., lambda_{2 nmax + 1}] per pair.

    Entry n multiplies the bare c_n.  n = 0 (the potential) is undamped."""
    r = np.asarray(r, dtype=float)
    prod = np.asarray(abar_i, float) * np.asarray(abar_j, float)
    damped = prod > 0.0
    safe = np.where(damped, prod, 1.0)
    x = np.asarray(a_ij, float) * r ** 3 / np.sqrt(safe)
    ex = np.exp(-x)
    polys = thole_polynomials(max(nmax, 1))
    lam = [np.ones_like(r)]
    for n in range(1, nmax + 1):
        val = 1.0 - npoly.polyval(x, polys[n - 1]) * ex
        lam.append(np.where(damped, val, 1.0))
    return lam
