"""Pins of the oracle's extrapolated guess (solver.extrapolate): exact on
polynomial trajectories of degree below the order, the newest set for
orders 0 and 1, and the closed forms of orders 2 to 4."""
import numpy as np
import pytest

from oracle import solver


def _traj(coefs, t):
    return sum(c * t ** p for p, c in enumerate(coefs))


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_exact_on_polynomials_below_the_order(k):
    rng = np.random.default_rng(k)
    coefs = [rng.normal(size=(7, 3)) for _ in range(k)]      # degree k - 1
    hist = [_traj(coefs, -float(j)) for j in range(1, k + 3)]  # newest first
    guess = solver.extrapolate(hist, k)
    assert np.allclose(guess, _traj(coefs, 0.0), rtol=0, atol=1e-11 * 10 ** k)


def test_degree_k_is_not_exact_and_short_history_truncates():
    rng = np.random.default_rng(9)
    coefs = [rng.normal(size=(4, 3)) for _ in range(4)]      # cubic
    hist = [_traj(coefs, -float(j)) for j in range(1, 6)]
    assert not np.allclose(solver.extrapolate(hist, 3), _traj(coefs, 0.0))
    # fewer sets than the order: the available ones
    assert np.allclose(solver.extrapolate(hist[:2], 5), 2 * hist[0] - hist[1])
    for k in (0, 1):
        assert np.array_equal(solver.extrapolate(hist, k), hist[0])


def test_closed_forms_of_low_orders():
    rng = np.random.default_rng(3)
    h = [rng.normal(size=(5, 3)) for _ in range(4)]
    assert np.allclose(solver.extrapolate(h, 2), 2 * h[0] - h[1])
    assert np.allclose(solver.extrapolate(h, 3), 3 * h[0] - 3 * h[1] + h[2])
    assert np.allclose(solver.extrapolate(h, 4), 4 * h[0] - 6 * h[1] + 4 * h[2] - h[3])
