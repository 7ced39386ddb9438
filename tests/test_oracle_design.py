"""Pins of the oracle's design update (optimality criteria for the box and volume
constraints of Section 7.1) against a hand-solved case, fixed points, the optimality
conditions of the update and the descent property at fixed volume."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2505_10168_amd import inputs as I


def test_two_elements_hand_solved():
    # chi = (1/2, 1/2), D = (4, 1), eta = 1/2, no active bounds, mean = 1/2:
    # x_e = chi_e sqrt(D_e / lam) sums to 1 for sqrt(lam) = 3/2, so chi' = (2/3, 1/3)
    chi, g = np.array([0.5, 0.5]), np.array([-4.0, -1.0])
    lam = O.oc_multiplier(chi, g, 0.5, move=1.0, eta=0.5, chi_min=0.0)
    new = O.oc_update(chi, g, 0.5, move=1.0, eta=0.5, chi_min=0.0)
    assert lam == pytest.approx(2.25, rel=1e-14)
    assert np.allclose(new, [2.0 / 3.0, 1.0 / 3.0], rtol=0, atol=1e-15)


def test_uniform_design_and_gradient_is_a_fixed_point():
    chi = np.full(37, 0.4)
    new = O.oc_update(chi, np.full(37, -3.5), 0.4, move=0.2, eta=0.5)
    assert np.abs(new - 0.4).max() <= 1e-15
    assert O.oc_multiplier(chi, np.full(37, -3.5), 0.4) == pytest.approx(3.5, rel=1e-14)


@pytest.mark.parametrize("eta", [0.5, 0.3, 1.0])
def test_optimality_conditions_of_the_step(eta):
    rng = np.random.default_rng(11)
    n, move, cmin, vol = 300, 0.1, 1e-3, 0.45
    chi = rng.uniform(0.0, 1.0, n)
    chi[:10] = 0.0
    chi[10:20] = 1.0
    g = -10 ** rng.uniform(-4, 0, n)
    g[20:30] = rng.uniform(0.0, 1e-2, 10)          # elements that do not help
    new = O.oc_update(chi, g, vol, move, eta, cmin)
    lam = O.oc_multiplier(chi, g, vol, move, eta, cmin)
    lo, hi = np.maximum(cmin, chi - move), np.minimum(1.0, chi + move)
    assert np.all(new >= lo - 1e-15) and np.all(new <= hi + 1e-15)
    assert abs(new.mean() - vol) <= 1e-13
    drive = np.maximum(-g, 0.0)
    inner = (new > lo + 1e-12) & (new < hi - 1e-12)
    assert inner.sum() > 20
    # interior elements: chi' = chi (D / lam)^eta with one lam for all of them
    ratio = (new[inner] / chi[inner]) ** (1.0 / eta) / drive[inner]
    assert np.allclose(ratio, 1.0 / lam, rtol=1e-10, atol=0)
    # elements on a bound: the unclamped value lies beyond it
    x = chi * (drive / lam) ** eta
    at_hi = np.abs(new - hi) <= 1e-15
    at_lo = np.abs(new - lo) <= 1e-15
    assert np.all(x[at_hi & ~at_lo] >= hi[at_hi & ~at_lo] * (1 - 1e-12))
    assert np.all(x[at_lo & ~at_hi] <= lo[at_lo & ~at_hi] * (1 + 1e-12) + 1e-300)
    assert np.all(new[20:30] == lo[20:30])          # D = 0 moves to the lower bound


def test_inactive_volume_bound_takes_the_upper_move_limit():
    rng = np.random.default_rng(2)
    chi = rng.uniform(0.1, 0.9, 64)
    g = -rng.uniform(0.1, 1.0, 64)
    g[::7] = 0.0
    new = O.oc_update(chi, g, 1.0, move=0.15)
    hi, lo = np.minimum(1.0, chi + 0.15), np.maximum(1e-3, chi - 0.15)
    assert np.array_equal(new[g < 0], hi[g < 0])
    assert np.array_equal(new[g == 0], lo[g == 0])


def test_no_descent_direction_moves_everything_down():
    chi = np.linspace(0.0, 1.0, 21)
    new = O.oc_update(chi, np.abs(np.sin(np.arange(21.0))), 0.5, move=0.2)
    assert np.array_equal(new, np.maximum(1e-3, chi - 0.2))


def test_step_is_a_descent_direction_at_fixed_volume():
    # with sum(chi') = sum(chi), g . (chi' - chi) <= 0: elements grow where D > lam and
    # shrink where D < lam, so the sum of (D - lam)(chi' - chi) is non-negative
    rng = np.random.default_rng(5)
    for trial in range(5):
        chi = rng.uniform(0.05, 0.95, 128)
        vol = float(chi.mean())
        g = -10 ** rng.uniform(-3, 0, 128)
        if trial % 2:
            g[rng.integers(0, 128, 12)] = 0.01
        new = O.oc_update(chi, g, vol, move=0.2)
        assert abs(new.mean() - vol) <= 1e-13
        assert float(g @ (new - chi)) < 0.0


def section7_small(n=32):
    mat = O.Material(0.197, 214.0, 1.67e6, 2.41e6)
    return mat, I.paper_heat_load(n, n, 0.1, 10.0)


def test_step_lowers_theta_and_loop_stops_by_the_rule():
    n = 32
    mat, q = section7_small(n)
    chi0 = np.full(n, 0.5)
    designs, thetas = O.design_loop(chi0, mat, n, 0.1, 10.0, q, 1e6, 0.5, max_cycles=200)
    # the first step (a descent direction, move 0.2) lowers Theta
    assert thetas[1] < thetas[0]
    assert thetas[-1] < 0.95 * thetas[0]
    assert all(d.mean() <= 0.5 + 1e-13 for d in designs)
    assert all(d.min() >= 1e-3 - 1e-15 and d.max() <= 1.0 for d in designs[1:])
    # stopped after five consecutive changes below 0.1 %, and not earlier
    assert len(thetas) < 200
    ch = np.abs(np.diff(thetas)) / np.abs(np.asarray(thetas[:-1]))
    assert np.all(ch[-5:] < 1e-3)
    runs = 0
    for c in ch[:-1]:
        runs = runs + 1 if c < 1e-3 else 0
        assert runs < 5
