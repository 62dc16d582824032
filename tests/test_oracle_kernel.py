"""Pins of the oracle's blob kernel against the properties the paper states
for the 3-point function (eq. delta and the sentences after it)."""
import numpy as np
import pytest

import oracle

SPECIAL = [0.0, 0.13, 0.37, 0.5, -0.5, 0.77, 1.0, 1.4999, -1.2, 2.5e-9]


def _weights(t):
    # Phi at the integer nodes around a point t (units of h)
    js = np.arange(np.floor(t) - 3, np.floor(t) + 4)
    return js, np.array([oracle.phi(j - t) for j in js])


@pytest.mark.parametrize("t", SPECIAL + list(np.random.default_rng(7).uniform(-3, 3, 25)))
def test_moments(t):
    """Zeroth moment 1, first moment 0 (grid independence of J[1] and
    J[r - q]) and discrete L2 norm 1/2 per axis, i.e. int delta_h^2 =
    1/(8 h^3) (after eq. delta)."""
    js, w = _weights(t)
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs(((js - t) * w).sum()) < 1e-15
    assert abs((w * w).sum() - 0.5) < 1e-15


def test_support_and_values(golden):
    """Support of three cells (blob kernel width 3h, Sec. Velocity profiles)
    and int delta_h^2 = 1/V with V = 8 h^3."""
    for r in (1.5, -1.5, 1.6, 2.0, -7.0):
        assert oracle.phi(r) == 0.0
    # one axis contributes sum Phi^2 = 1/2, three axes (1/2)^3 = 1/8
    V = golden["compressible_blob_volume_h3"]["value"]
    js, w = _weights(0.3)
    assert abs((w * w).sum() ** 3 - 1.0 / V) < 1e-15


def test_continuity_c1():
    """Phi is continuous with a continuous derivative at |r| = 1/2 and 3/2."""
    eps = 1e-7
    for r0 in (0.5, 1.5, -0.5, -1.5):
        left, right = oracle.phi(r0 - eps), oracle.phi(r0 + eps)
        assert abs(left - right) < 1e-6
        dl = (oracle.phi(r0 - eps) - oracle.phi(r0 - 2 * eps)) / eps
        dr = (oracle.phi(r0 + 2 * eps) - oracle.phi(r0 + eps)) / eps
        assert abs(dl - dr) < 1e-5


def test_symmetry_and_positivity():
    for r in np.linspace(0, 1.6, 33):
        assert oracle.phi(r) == oracle.phi(-r)
        assert oracle.phi(r) >= 0.0
