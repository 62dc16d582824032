"""Pins of the oracle's reverse-mode derivatives (the gradient of a
trajectory loss used for differentiation): each derivative against central
finite differences of the forward function it differentiates, and the
kernel derivative against the moment conditions of the 3-point kernel
(eq. delta and the properties listed after it)."""
import numpy as np
import pytest

import oracle
from paper_1407_5600_amd import inputs


def _cfd(f, x, i, e):
    xp = x.copy()
    xm = x.copy()
    xp.flat[i] += e
    xm.flat[i] -= e
    return (f(xp) - f(xm)) / (2 * e)


@pytest.mark.parametrize("r", [0.0, 0.13, -0.37, 0.5, -0.5, 0.77, -1.2, 1.49, 1.6])
def test_phi_deriv_finite_differences(r):
    e = 1e-6
    fd = (oracle.phi(r + e) - oracle.phi(r - e)) / (2 * e)
    # Phi'' jumps at |r| = 1/2 (Phi is C^1 only): there the central
    # difference is first-order accurate
    tol = 2e-5 if abs(abs(r) - 0.5) < 1e-12 else 1e-8
    assert abs(oracle.phi_deriv(r) - fd) < tol


@pytest.mark.parametrize("x", [0.0, 0.13, 0.37, 0.5, 0.77])
def test_phi_deriv_moments(x):
    """d/dx of sum_j Phi(x - j) = 1 and of sum_j (x - j) Phi(x - j) = 0."""
    js = range(-3, 5)
    s0 = sum(oracle.phi_deriv(x - j) for j in js)
    s1 = sum((x - j) * oracle.phi_deriv(x - j) for j in js)
    assert abs(s0) < 1e-14
    assert abs(s1 + 1.0) < 1e-14


def test_phi_deriv_continuity():
    """Phi is C^1: Phi' is continuous at |r| = 1/2 and 0 at |r| = 3/2."""
    for r in (0.5, -0.5):
        assert abs(oracle.phi_deriv(r - 1e-12) - oracle.phi_deriv(r + 1e-12)) < 1e-5
    assert abs(oracle.phi_deriv(1.5 - 1e-12)) < 1e-5
    assert oracle.phi_deriv(1.5 + 1e-9) == 0.0


@pytest.mark.parametrize("h", [1.0, 0.7])
def test_interpolate_grad_finite_differences(h):
    L = 8
    prm = oracle.params(L, h=h)
    rng = np.random.default_rng(3)
    M = 5
    q = rng.uniform(0, L * h, (M, 3))
    q[0] = [0.01, L * h - 0.02, 3.5 * h]  # straddling the periodic seam
    v = rng.standard_normal((3, L, L, L))
    W = rng.standard_normal((M, 3))
    g = oracle.interpolate_grad(prm, q, v, W)
    e = 1e-6
    for i in range(3 * M):
        fd = _cfd(lambda qq: np.sum(W * oracle.interpolate(prm, qq, v)), q, i, e)
        # q = 3.5 h sits on a kink of Phi'' (a tie of the node sets): there
        # the central difference is first-order accurate
        on_kink = abs(q.flat[i] / h - round(q.flat[i] / h - 0.5) - 0.5) < 1e-9
        tol = 1e-5 if on_kink else 1e-7
        assert abs(g.flat[i] - fd) < tol * max(1.0, abs(fd)), (i, g.flat[i], fd)


def test_spring_adjoint_finite_differences():
    tmpl = inputs.icosahedron_template(1.0)
    pa, pb, r0 = inputs.pair_table(tmpl)
    rng = np.random.default_rng(4)
    P, nb, k = 2, len(tmpl), 37.0
    R = inputs.random_rotations(rng, P)
    q = inputs.place_particles(rng.uniform(0, 10, (P, 3)), tmpl, R)
    q += 0.05 * rng.standard_normal(q.shape)  # off the rest state
    Fbar = rng.standard_normal(q.shape)
    qbar, kbar, r0bar = oracle.spring_adjoint(P, nb, pa, pb, r0, k, q, Fbar)

    def obj(qq, kk=k, rr=r0):
        return np.sum(Fbar * oracle.spring_forces(P, nb, pa, pb, rr, kk, qq, None))

    e = 1e-6
    for i in range(0, q.size, 5):
        fd = _cfd(lambda x: obj(x), q, i, e)
        assert abs(qbar.flat[i] - fd) < 1e-6 * max(1.0, abs(fd))
    fdk = (obj(q, k + e) - obj(q, k - e)) / (2 * e)
    assert abs(kbar - fdk) < 1e-6 * max(1.0, abs(fdk))
    for j in range(0, len(r0), 7):
        fd = _cfd(lambda x: obj(q, k, x), np.array(r0, dtype=float), j, e)
        assert abs(r0bar[j] - fd) < 1e-6 * max(1.0, abs(fd))


def _traj_case(steady=False, zero_mean=False, nsteps=3, L=16, seed=5, h=1.0):
    tmpl = inputs.icosahedron_template(1.0)
    pa, pb, r0 = inputs.pair_table(tmpl)
    rng = np.random.default_rng(seed)
    P, nb = 2, len(tmpl)
    R = inputs.random_rotations(rng, P)
    centres = np.array([[4.3, 5.1, 6.7], [8.9, 7.2, 9.6]])
    q0 = inputs.place_particles(centres, tmpl, R) + 0.02 * rng.standard_normal((P * nb, 3))
    v0 = 0.01 * rng.standard_normal((3, L, L, L))
    G = rng.standard_normal((P * nb, 3))
    V = 0.1 * rng.standard_normal((P, 3))
    prm = oracle.params(L, h=h, dt=0.05, steady=steady, zero_mean=zero_mean or steady)
    sp = {"nb": nb, "pa": pa, "pb": pb, "r0": np.array(r0, dtype=float), "k": 20.0}
    return prm, sp, q0, v0, G, V, nsteps


@pytest.mark.parametrize("mode,h", [("unsteady", 1.0), ("zero_mean", 1.0), ("steady", 1.0),
                                    ("unsteady", 0.8)])
def test_loss_grad_finite_differences(mode, h):
    """Central differences (step 1e-6) of the trajectory loss against the
    reverse sweep, for blob forces, initial positions and velocity, k and
    the rest lengths."""
    prm, sp, q0, v0, G, V, n = _traj_case(steady=mode == "steady",
                                          zero_mean=mode == "zero_mean", h=h)
    loss, g = oracle.loss_grad(prm, sp, q0, v0, G, V, n)
    assert loss > 0

    def L_of(q0_=q0, v0_=v0, G_=G, k_=sp["k"], r0_=sp["r0"]):
        s = dict(sp, k=k_, r0=r0_)
        return oracle.loss_grad(prm, s, q0_, v0_, G_, V, n)[0]

    e = 1e-6
    rng = np.random.default_rng(0)
    checks = []
    for i in rng.choice(G.size, 6, replace=False):
        checks.append((g["G"].flat[i], _cfd(lambda x: L_of(G_=x), G, i, e)))
    for i in rng.choice(q0.size, 6, replace=False):
        checks.append((g["q0"].flat[i], _cfd(lambda x: L_of(q0_=x), q0, i, e)))
    if mode != "steady":
        for i in rng.choice(v0.size, 4, replace=False):
            checks.append((g["v0"].flat[i], _cfd(lambda x: L_of(v0_=x), v0, i, e)))
    checks.append((g["k"], (L_of(k_=sp["k"] + e) - L_of(k_=sp["k"] - e)) / (2 * e)))
    for j in (0, 40, 77):
        checks.append((g["r0"][j], _cfd(lambda x: L_of(r0_=x), sp["r0"], j, e)))
    scale = max(abs(fd) for _, fd in checks)
    for ad, fd in checks:
        assert abs(ad - fd) <= 1e-6 * scale, (ad, fd, scale)
