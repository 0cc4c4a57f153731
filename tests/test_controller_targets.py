"""Training targets of the learned step-size controller (host logic, no
GPU): the hindsight target, and its cap at the explicit stability limit,
whose constant is pinned to the stability function of the oracle's
Dormand-Prince tableau."""
import math

import numpy as np

import oracle
from paper_2309_05331_amd import controller


def _stability(z):
    # R(z) = 1 + z b^T (I - z A)^-1 1 for the explicit tableau (A, b)
    a, b, _, _ = oracle.tableau(oracle.DOPRI5)
    s = b.size
    return 1.0 + z * b @ np.linalg.solve(np.eye(s) - z * a, np.ones(s))


def test_stability_constant_is_where_the_5th_order_solution_reaches_one():
    z = -controller.DOPRI5_REAL_STABILITY
    assert abs(_stability(z) - 1.0) < 1e-4
    # inside the interval the modulus is below one, just outside above
    assert all(abs(_stability(-x)) < 1.0 for x in np.linspace(0.05, 3.3, 200))
    assert abs(_stability(-3.32)) > 1.0


def _trace(h, err, acc, lam):
    """Rows of the device trace layout: h, err, accepted, ..., and the 16
    features with feature 15 = log(h (lambda + 1))."""
    n = len(h)
    tr = np.full((n, 24), np.nan)
    tr[:, 0], tr[:, 1], tr[:, 2] = h, err, acc
    tr[:, 8:24] = 0.0
    tr[:, 23] = np.log(np.asarray(h) * (lam + 1.0))
    return tr


def test_hindsight_target_and_cap():
    h = np.array([0.10, 0.25, 0.28, 0.30])
    err = np.array([0.3, 0.4, 0.05, 0.02])
    acc = np.ones(4)
    lam = 10.0  # stability step 0.330657
    tr = _trace(h, err, acc, lam)
    X, T, W = controller.dataset_from_trace(tr, rho=0.5, reject_weight=2.0)
    want = np.log(h[1:] / h[:-1]) + 0.2 * np.log(0.5 / err[1:])
    np.testing.assert_allclose(T, np.clip(want, math.log(0.2), math.log(5.0)), rtol=1e-12)
    assert np.all(W == 1.0) and X.shape == (3, 16)
    # capped at 0.9 of the stability step 3.30657 / lambda
    _, Tc, _ = controller.dataset_from_trace(tr, rho=0.5, reject_weight=2.0, stab_cap=0.9)
    cap = np.log(0.9 * controller.DOPRI5_REAL_STABILITY / lam / h[:-1])
    np.testing.assert_allclose(Tc, np.clip(np.minimum(want, cap), math.log(0.2), math.log(5.0)), rtol=1e-12)
    assert np.all(Tc <= T + 1e-15) and np.any(Tc < T)
    # a reject after a pair weighs more; rejected attempts give no pair
    tr2 = _trace(h, np.array([0.3, 1.5, 0.05, 0.02]), np.array([1, 0, 1, 1]), lam)
    _, T2, W2 = controller.dataset_from_trace(tr2, rho=0.5, reject_weight=2.0)
    assert T2.size == 2 and list(W2) == [2.0, 1.0]
