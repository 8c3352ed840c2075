"""Iterative and direct solvers for T mu = E (paper Eq. 18).

The paper converges the induced dipoles with a preconditioned conjugate
gradient (Computational Details; technical appendix, Polarization).  This is
textbook PCG (Hestenes & Stiefel 1952) with the block-diagonal
preconditioner M^-1 = blockdiag(alpha_i), i.e. the inverse of T's diagonal
blocks.

Convergence measure (reading; the paper gives only a threshold):
  rho = DEBYE * sqrt( sum_i |z_i|^2 / N_pol ),  z = M^-1 r,
an RMS over polarizable sites in Debye.  On exit the residual is recomputed
from scratch (r = E - T x); if that true rho is above the tolerance the
iteration restarts from x.

Vectors are (N_pol, 3) arrays; matvec(p) returns T p; precond(r) returns
alpha r.
"""
import numpy as np

from .units import DEBYE


class NotSPD(RuntimeError):
    pass


def rms_debye(z):
    """RMS over sites in Debye; zero for an empty set of sites."""
    if len(z) == 0:
        return 0.0
    return DEBYE * float(np.sqrt(np.sum(z * z) / len(z)))


def pcg(matvec, precond, rhs, x0, tol, max_iter=200, max_restarts=5, measure=None):
    """Returns (x, iterations, true rho).  The stop tests take the RMS of
    measure(r) (default: the preconditioned residual itself)."""
    if measure is None:
        measure = precond
    x = x0.copy()
    iters = 0
    for _ in range(max_restarts + 1):
        r = rhs - matvec(x)
        z = precond(r)
        if rms_debye(measure(r)) <= tol:
            return x, iters, rms_debye(measure(r))
        p = z.copy()
        rz = float(np.sum(r * z))
        while iters < max_iter:
            q = matvec(p)
            pq = float(np.sum(p * q))
            if pq <= 0.0:
                raise NotSPD("p.Tp <= 0: T is not positive definite")
            gamma = rz / pq
            x = x + gamma * p
            r = r - gamma * q
            z = precond(r)
            iters += 1
            if rms_debye(measure(r)) <= tol:
                break
            rz_new = float(np.sum(r * z))
            p = z + (rz_new / rz) * p
            rz = rz_new
        rho = rms_debye(measure(rhs - matvec(x)))
        if rho <= tol or iters >= max_iter:
            return x, iters, rho
    return x, iters, rho


def tcg(matvec, precond, rhs, x0, order, omega=0.0):
    """Truncated conjugate gradient (TCG-n): a fixed cost instead of a
    convergence test.

    The paper names TCG as the fixed-cost way to converge the dipoles
    (Many-Body Polarization) and leaves its definition to the cited work.
    Reading: TCG-n is the n-th iterate of the PCG above (same guess, same
    preconditioner M^-1 = alpha, no stop test; the closed forms of the cited
    work are this iterate written out), optionally followed by one "peek"
    step x <- x + omega M^-1 r_n with the residual r_n of that iterate.  A
    zero residual ends the steps early (the iterate is then exact).
    Returns x.
    """
    x = x0.copy()
    r = rhs - matvec(x)
    z = precond(r)
    p = z.copy()
    rz = float(np.sum(r * z))
    for _ in range(order):
        if rz == 0.0:
            break
        q = matvec(p)
        pq = float(np.sum(p * q))
        if pq <= 0.0:
            raise NotSPD("p.Tp <= 0: T is not positive definite")
        gamma = rz / pq
        x = x + gamma * p
        r = r - gamma * q
        z = precond(r)
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    if omega != 0.0:
        x = x + omega * z
    return x


def plain_cg(matvec, rhs, x0, tol_abs, max_iter=1000):
    """Unpreconditioned CG to |r|_inf <= tol_abs."""
    x = x0.copy()
    r = rhs - matvec(x)
    p = r.copy()
    rr = float(np.sum(r * r))
    for k in range(max_iter):
        if np.max(np.abs(r)) <= tol_abs:
            return x, k
        q = matvec(p)
        a = rr / float(np.sum(p * q))
        x = x + a * p
        r = r - a * q
        rr_new = float(np.sum(r * r))
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, max_iter


def jacobi(matvec, precond, rhs, x0, tol_abs, max_iter=5000, omega=0.7):
    """Damped block-Jacobi: x <- x + omega * M^-1 (rhs - T x)."""
    x = x0.copy()
    for k in range(max_iter):
        r = rhs - matvec(x)
        if np.max(np.abs(r)) <= tol_abs:
            return x, k
        x = x + omega * precond(r)
    return x, max_iter


def extrapolate(history, k):
    """Guess for the next step from dipole sets taken at equally spaced
    times: the value at t = 0 of the polynomial of degree k' - 1 through
    the k' = min(k, len(history)) newest sets, placed at t = -1, -2, ...
    (history[0] newest).  Written as Lagrange interpolation evaluated at
    t = 0; k' <= 1 returns the newest set.  (The extrapolated guesses of
    the truncated and iterated solvers that Many-Body Polarization cites;
    the polynomial form is this implementation's reading.)"""
    kk = min(int(k), len(history))
    if kk <= 1:
        return np.array(history[0], dtype=float)
    ts = -np.arange(1, kk + 1, dtype=float)
    out = np.zeros_like(np.asarray(history[0], dtype=float))
    for j in range(kk):
        w = 1.0
        for m in range(kk):
            if m != j:
                w *= (0.0 - ts[m]) / (ts[j] - ts[m])
        out += w * np.asarray(history[j], dtype=float)
    return out
