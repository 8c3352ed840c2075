"""Pins of the oracle's building blocks against textbook facts.

* radial coefficients obey c_{n+1} = -c_n'/r (checked by central finite
  differences, for the bare, Ewald and Thole-damped kernels);
* the pairing construction of the derivative tensors equals finite
  differences of the previous rank, and the textbook dipole tensor;
* the multipole operators reproduce the potential of explicit point-charge
  arrangements (a dipole pair and a linear Buckingham quadrupole);
* cardinal B-splines: partition of unity, known knot values, derivative
  identities.
"""
import math

import numpy as np
import pytest

from oracle import radial, recip
from oracle.tensors import deriv_tensor, pairings, contract_leading


def _fd(f, r, h=1e-6):
    return (f(r + h) - f(r - h)) / (2 * h)


@pytest.mark.parametrize("n", range(0, 5))
def test_bare_recursion(n):
    r = np.array([0.7, 1.3, 2.9, 6.1])
    d = _fd(lambda x: radial.bare(x, n)[n], r)
    assert np.allclose(-d / r, radial.bare(r, n + 1)[n + 1], rtol=1e-7)


@pytest.mark.parametrize("n", range(0, 5))
def test_ewald_recursion(n):
    r = np.array([0.5, 1.3, 2.9, 6.1, 8.5])
    beta = 0.4
    d = _fd(lambda x: radial.ewald_real(x, beta, n)[n], r)
    assert np.allclose(-d / r, radial.ewald_real(r, beta, n + 1)[n + 1],
                       rtol=1e-6, atol=1e-12)


def test_ewald_limits():
    # beta -> 0 gives the bare kernel; large r decays like erfc
    r = np.array([1.0, 2.0, 3.0])
    B = radial.ewald_real(r, 1e-7, 4)
    c = radial.bare(r, 4)
    for n in range(5):
        assert np.allclose(B[n], c[n], rtol=1e-6)
    assert radial.ewald_real(np.array([9.0]), 0.4, 0)[0][0] == pytest.approx(
        math.erfc(3.6) / 9.0, rel=1e-14)


@pytest.mark.parametrize("n", range(1, 4))
def test_thole_damped_is_derivative(n):
    """Damped c_{n+1} = -(damped c_n)'/r: each damped tensor is the exact
    derivative of the damped field (Thole 1981 exponential form)."""
    r = np.array([0.45, 0.8, 1.5, 2.5, 4.0])
    ai, aj, a = np.full(5, 0.9), np.full(5, 0.6), np.full(5, 0.28)

    def damped(x, k):
        lam = radial.thole_lambdas(x, ai, aj, a, k)
        return lam[k] * radial.bare(x, k)[k]

    d = _fd(lambda x: damped(x, n), r, h=1e-6)
    assert np.allclose(-d / r, damped(r, n + 1), rtol=1e-6)


def test_thole_field_form():
    """lambda_3 = 1 - exp(-a u^3), u = r/(abar_i abar_j)^(1/6)."""
    r = np.array([0.5, 1.0, 2.0])
    ai, aj = 0.8, 0.5
    lam = radial.thole_lambdas(r, np.full(3, ai), np.full(3, aj),
                               np.full(3, 0.28), 1)
    u = r / (ai * aj) ** (1.0 / 6.0)
    assert np.allclose(lam[1], 1 - np.exp(-0.28 * u ** 3), rtol=1e-14)
    # no damping when one site is not polarizable
    lam0 = radial.thole_lambdas(r, np.zeros(3), np.full(3, aj),
                                np.full(3, 0.28), 3)
    for k in range(4):
        assert np.all(lam0[k] == 1.0)


def test_pairing_counts():
    # number of pairings of n objects into pairs/singletons = telephone numbers
    assert [len(pairings(n)) for n in range(7)] == [1, 1, 2, 4, 10, 26, 76]


@pytest.mark.parametrize("n", range(1, 6))
def test_deriv_tensor_fd(n):
    rng = np.random.default_rng(5)
    R = rng.normal(size=(4, 3)) * 1.5 + 0.3
    beta = 0.5

    def D(Rv, k):
        r = np.linalg.norm(Rv, axis=1)
        return deriv_tensor(k, Rv, radial.ewald_real(r, beta, k))

    h = 1e-5
    full = D(R, n)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (D(R + e, n - 1) - D(R - e, n - 1)) / (2 * h)
        assert np.allclose(full[(slice(None),) + (slice(None),) * (n - 1) + (a,)],
                           fd, rtol=1e-6, atol=1e-9)


def test_dipole_tensor_textbook():
    R = np.array([[0.3, -1.2, 2.0]])
    r = np.linalg.norm(R)
    D2 = deriv_tensor(2, R, radial.bare(np.array([r]), 2))[0]
    ref = (3 * np.outer(R[0], R[0]) - r * r * np.eye(3)) / r ** 5
    assert np.allclose(D2, ref, rtol=1e-14)


def _potential(R, q=None, d=None, th=None):
    """Oracle potential of one multipole at displacement R (field point -
    site): [q - d.grad + 1/3 Theta:grad grad] 1/R."""
    R = np.atleast_2d(R)
    r = np.linalg.norm(R, axis=1)
    c = radial.bare(r, 2)
    out = np.zeros(len(R))
    if q is not None:
        out += q * c[0]
    if d is not None:
        out -= contract_leading(deriv_tensor(1, R, c), [np.tile(d, (len(R), 1))])
    if th is not None:
        out += contract_leading(deriv_tensor(2, R, c),
                                [np.tile(th, (len(R), 1, 1))]) / 3.0
    return out


def test_dipole_matches_charge_pair():
    rng = np.random.default_rng(1)
    dvec = np.array([0.3, -0.2, 0.5])
    h = 1e-3
    qc = 1.0 / h
    pts = rng.normal(size=(6, 3)) * 5 + 1
    exact = np.zeros(len(pts))
    for s in (+1, -1):
        src = 0.5 * s * h * dvec / np.linalg.norm(dvec)
        exact += s * qc * np.linalg.norm(dvec) / np.linalg.norm(pts - src, axis=1)
    assert np.allclose(_potential(pts, d=dvec), exact, rtol=1e-6)


def test_quadrupole_matches_linear_charges():
    """Charges +c at +/-a z and -2c at 0 carry the Buckingham quadrupole
    Theta = 1/2 sum q (3 x x - r^2 I) = c a^2 diag(-1, -1, 2)."""
    c, a = 1.0, 1e-2
    th = c * a * a * np.diag([-1.0, -1.0, 2.0])
    pts = np.array([[3.0, 1.0, 2.0], [-2.0, 4.0, -1.0], [0.5, 0.5, 5.0]])
    exact = (c / np.linalg.norm(pts - [0, 0, a], axis=1)
             + c / np.linalg.norm(pts + [0, 0, a], axis=1)
             - 2 * c / np.linalg.norm(pts, axis=1))
    assert np.allclose(_potential(pts, th=th), exact, rtol=1e-4)


@pytest.mark.parametrize("order", [4, 5, 6])
def test_bspline_partition_of_unity(order):
    w = np.linspace(0.0, 0.999, 37)
    tot = sum(recip.bspline(w + t, order) for t in range(order))
    assert np.allclose(tot, 1.0, atol=1e-14)
    wi = np.linspace(0.01, 0.99, 37)   # derivatives away from the knots
    for nd in range(1, order - 1):
        dsum = sum(recip.bspline(wi + t, order, nd) for t in range(order))
        assert np.allclose(dsum, 0.0, atol=1e-12)


def test_bspline_knots_and_derivative():
    # cubic B-spline (order 4) at the knots: 1/6, 4/6, 1/6
    assert np.allclose(recip.bspline(np.array([1.0, 2.0, 3.0]), 4),
                       [1 / 6, 4 / 6, 1 / 6], atol=1e-15)
    u = np.linspace(0.2, 4.8, 11)
    for nd in range(3):
        fd = (recip.bspline(u + 1e-6, 5, nd) - recip.bspline(u - 1e-6, 5, nd)) / 2e-6
        assert np.allclose(fd, recip.bspline(u, 5, nd + 1), atol=1e-7)


def test_bspline_moduli_nyquist():
    # odd order on an even grid: the raw modulus vanishes at K/2
    K, p = 20, 5
    k = np.arange(p - 1)
    Mk = recip.bspline(k + 1.0, p)
    raw = np.abs(np.exp(1j * np.pi * k) @ Mk) ** 2
    assert raw < 1e-25
    mod = recip.bspline_moduli(K, p)
    assert mod[K // 2] == pytest.approx(0.5 * (mod[K // 2 - 1] + mod[K // 2 + 1]))
    assert mod[0] == pytest.approx(1.0)
