"""Pins of the oracle's spreading S and interpolation J (eq. ju, the
definition of S_i after eq. jm, and the properties listed before Sec.
Multiblob dynamics), plus the Faxen second moment of the appendix."""
import numpy as np
import pytest

import oracle
from paper_1407_5600_amd import inputs


def _blobs(seed, M, L, big=False):
    rng = np.random.default_rng(seed)
    q = rng.uniform(0, L, size=(M, 3))
    if big:  # unwrapped coordinates far from the primary box
        q += rng.integers(-50, 50, size=(M, 3)) * L + 1e5
    return q


@pytest.mark.parametrize("L,h,big", [(8, 1.0, False), (12, 0.7, False), (16, 1.0, True), (6, 1.3, False)])
def test_adjointness(L, h, big):
    """<J v, F> = h^3 <v, S F>: J and S are adjoint."""
    M = 40
    q = _blobs(1, M, L * h, big)
    rng = np.random.default_rng(2)
    F = rng.standard_normal((M, 3))
    v = rng.standard_normal((3, L, L, L))
    prm = oracle.params(L, h=h)
    lhs = np.sum(oracle.interpolate(prm, q, v) * F)
    rhs = h ** 3 * np.sum(v * oracle.spread(prm, q, F))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("h", [1.0, 0.5])
def test_total_force_and_constants(h):
    """Zeroth moment: h^3 sum_x S F = F, J[const] = const."""
    L = 10
    q = _blobs(3, 25, L * h)
    F = np.random.default_rng(4).standard_normal((25, 3))
    prm = oracle.params(L, h=h)
    f = oracle.spread(prm, q, F)
    assert np.allclose(h ** 3 * f.reshape(3, -1).sum(1), F.sum(0), atol=1e-12)
    v = np.empty((3, L, L, L))
    v[0], v[1], v[2] = 1.5, -2.0, 0.25
    u = oracle.interpolate(prm, q, v)
    assert np.allclose(u, [1.5, -2.0, 0.25], atol=1e-14)


def test_linear_field_exact():
    """First moment: J[r - q_i] = 0, so a linear field is interpolated to
    its value at q_i exactly (blob well inside the box, no wrap)."""
    L, h = 16, 1.0
    rng = np.random.default_rng(5)
    q = rng.uniform(6, 10, size=(10, 3))
    A = rng.standard_normal((3, 3))
    b = rng.standard_normal(3)
    idx = np.arange(L, dtype=float)
    v = np.empty((3, L, L, L))
    for a in range(3):
        # node of component a at h*(i,j,k) + h/2 e_a
        x = idx[None, None, :] + (0.5 if a == 0 else 0.0)
        y = idx[None, :, None] + (0.5 if a == 1 else 0.0)
        z = idx[:, None, None] + (0.5 if a == 2 else 0.0)
        v[a] = b[a] + A[a, 0] * x + A[a, 1] * y + A[a, 2] * z
    u = oracle.interpolate(oracle.params(L, h=h), q, v)
    assert np.allclose(u, b[None, :] + q @ A.T, atol=1e-12)


@pytest.mark.parametrize("h", [1.0, 0.8])
def test_one_blob_JS_compressible(h, golden):
    """J_i P S_i with P = 1 is exactly V^-1 = 1/(8 h^3) at any position."""
    V = golden["compressible_blob_volume_h3"]["value"]
    L = 8
    for seed in range(5):
        q = _blobs(seed, 1, L * h)
        F = np.array([[0.3, -1.0, 2.0]])
        prm = oracle.params(L, h=h)
        u = oracle.interpolate(prm, q, oracle.spread(prm, q, F))
        assert np.allclose(u, F / (V * h ** 3), rtol=1e-13)


def _second_moment(prm, q, centre):
    """J[(r - centre)^2] for each blob, by interpolating the field
    |x - centre|^2 sampled at each component's own nodes."""
    L, h = prm.L, prm.h
    idx = np.arange(L, dtype=float) * h
    out = 0.0
    for a in range(3):
        x = idx[None, None, :] + (0.5 * h if a == 0 else 0.0) - centre[0]
        y = idx[None, :, None] + (0.5 * h if a == 1 else 0.0) - centre[1]
        z = idx[:, None, None] + (0.5 * h if a == 2 else 0.0) - centre[2]
        v = np.zeros((3, L, L, L))
        v[a] = (x * x + y * y + z * z) / 3.0  # average over components
        out = out + oracle.interpolate(prm, q, v)[:, a]
    return out


def test_faxen_radius_blob(golden):
    """a_F^2 = J[r^2] of one blob (eq. jblob2) lies in [3/4, 1] h^2; its
    average over positions matches the printed a_F = (0.95 +- 0.05) h."""
    g = golden["blob_faxen_radius"]
    L = 16
    prm = oracle.params(L)
    rng = np.random.default_rng(9)
    vals = []
    for _ in range(30):
        q = rng.uniform(7, 9, size=(1, 3))
        vals.append(_second_moment(prm, q, q[0])[0])
    vals = np.array(vals)
    assert np.all(vals >= 0.75 - 1e-12) and np.all(vals <= 1.0 + 1e-12)
    assert abs(np.sqrt(vals).mean() - g["value"]) <= g["tol"]


def test_faxen_radius_multiblob():
    """eq. jm2a traced: J_m[(r - q0)^2] = (1/N) sum_i J_i[(r - q_i)^2]
    + (1/N) sum_i |s_i|^2, exact through the zeroth and first moments."""
    L = 24
    prm = oracle.params(L)
    tmpl = inputs.icosahedron_template(1.0)
    q0 = np.array([11.3, 12.1, 11.8])
    q = q0 + tmpl
    jm = _second_moment(prm, q, q0).mean()
    own = np.array([_second_moment(prm, q[i:i + 1], q[i])[0] for i in range(13)])
    assert abs(jm - (own.mean() + (tmpl ** 2).sum(1).mean())) < 1e-12


def test_icosahedron_gyration(golden):
    """Appendix: for the icosahedron sum_i s_i s_i^T over the 12 vertices is
    (a^2/3) per vertex times the identity; a = 0.9511 d."""
    a = 1.0
    t = inputs.icosahedron_template(a, centre=False)
    G = t.T @ t / 12.0
    assert np.allclose(G, np.eye(3) * a * a / 3.0, atol=1e-14)
    d = min(np.linalg.norm(t[i] - t[j]) for i in range(12) for j in range(i + 1, 12))
    assert abs(a / d - golden["circumradius_over_vertex_distance"]["value"]) < 1e-4


def test_seam_and_periodicity():
    """A blob straddling the periodic seam gives the same result as the
    same blob shifted by whole periods."""
    L = 8
    prm = oracle.params(L)
    q = np.array([[0.2, 7.9, 3.0]])
    F = np.array([[1.0, 2.0, 3.0]])
    f1 = oracle.spread(prm, q, F)
    f2 = oracle.spread(prm, q + np.array([[-3 * L, 5 * L, 11 * L]]), F)
    assert np.allclose(f1, f2, atol=1e-12)
