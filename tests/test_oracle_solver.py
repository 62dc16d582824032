"""Pins of the oracle's fluid solve (eq. vf with the projector P): a dense
real-space solve of the discrete equations on tiny grids, zero discrete
divergence, projector identities, the exact discrete decay of a shear mode
and its continuum limit, the steady response to sinusoidal forcing (the
viscosity measurement of Sec. Stresslet and viscosity) and the mean-mode
momentum balance."""
import numpy as np
import pytest

import oracle


def _ops(L, h):
    """Dense periodic MAC operators: D (cells x faces), G = -D^T and the
    7-point Laplacian acting on each velocity component."""
    N = L ** 3

    def idx(x, y, z):
        return ((z % L) * L + (y % L)) * L + (x % L)

    D = np.zeros((N, 3 * N))
    Lap = np.zeros((N, N))
    for z in range(L):
        for y in range(L):
            for x in range(L):
                c = idx(x, y, z)
                D[c, 0 * N + c] += 1 / h
                D[c, 0 * N + idx(x - 1, y, z)] -= 1 / h
                D[c, 1 * N + c] += 1 / h
                D[c, 1 * N + idx(x, y - 1, z)] -= 1 / h
                D[c, 2 * N + c] += 1 / h
                D[c, 2 * N + idx(x, y, z - 1)] -= 1 / h
                Lap[c, c] -= 6 / h ** 2
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    Lap[c, idx(x + dx, y + dy, z + dz)] += 1 / h ** 2
    G = -D.T
    Lap3 = np.kron(np.eye(3), Lap)
    return D, G, Lap3


@pytest.mark.parametrize("L,h", [(4, 1.0), (3, 0.6)])
def test_dense_unsteady(L, h):
    """Crank-Nicolson: (rho/dt - eta/2 Lap) v' + G pi = (rho/dt + eta/2 Lap) v + f,
    D v' = 0, solved densely."""
    rho, eta, dt = 1.3, 0.7, 0.05
    N = L ** 3
    D, G, Lap3 = _ops(L, h)
    rng = np.random.default_rng(L)
    v = rng.standard_normal(3 * N)
    f = rng.standard_normal(3 * N)
    A = np.zeros((4 * N + 1, 4 * N))
    A[:3 * N, :3 * N] = rho / dt * np.eye(3 * N) - 0.5 * eta * Lap3
    A[:3 * N, 3 * N:] = G
    A[3 * N:4 * N, :3 * N] = D
    A[4 * N, 3 * N:] = 1.0  # pressure gauge
    b = np.zeros(4 * N + 1)
    b[:3 * N] = (rho / dt * np.eye(3 * N) + 0.5 * eta * Lap3) @ v + f
    x = np.linalg.lstsq(A, b, rcond=None)[0]
    prm = oracle.params(L, h=h, rho=rho, eta=eta, dt=dt)
    out = oracle.fluid_solve(prm, v.reshape(3, L, L, L), f.reshape(3, L, L, L))
    assert np.max(np.abs(out.ravel() - x[:3 * N])) < 1e-11


@pytest.mark.parametrize("L,h", [(4, 1.0), (3, 1.4)])
def test_dense_steady(L, h):
    """Steady Stokes: -eta Lap v' + G pi = f, D v' = 0, mean(v') = 0; a mean
    force is dropped (it has no steady periodic solution)."""
    eta = 0.9
    N = L ** 3
    D, G, Lap3 = _ops(L, h)
    rng = np.random.default_rng(L + 10)
    f = rng.standard_normal(3 * N)
    f0 = f.reshape(3, N) - f.reshape(3, N).mean(1, keepdims=True)
    A = np.zeros((4 * N + 4, 4 * N))
    A[:3 * N, :3 * N] = -eta * Lap3
    A[:3 * N, 3 * N:] = G
    A[3 * N:4 * N, :3 * N] = D
    for c in range(3):
        A[4 * N + c, c * N:(c + 1) * N] = 1.0
    A[4 * N + 3, 3 * N:] = 1.0
    b = np.zeros(4 * N + 4)
    b[:3 * N] = f0.ravel()
    x = np.linalg.lstsq(A, b, rcond=None)[0]
    prm = oracle.params(L, h=h, eta=eta, steady=True, zero_mean=True)
    out = oracle.fluid_solve(prm, np.zeros((3, L, L, L)), f.reshape(3, L, L, L))
    assert np.max(np.abs(out.ravel() - x[:3 * N])) < 1e-11


@pytest.mark.parametrize("L", [8, 12, 9])
def test_divergence_free(L):
    rng = np.random.default_rng(L)
    prm = oracle.params(L, rho=1.0, eta=0.5, dt=0.1)
    out = oracle.fluid_solve(prm, rng.standard_normal((3, L, L, L)), rng.standard_normal((3, L, L, L)))
    assert np.max(np.abs(oracle.divergence(prm, out))) < 1e-12 * np.max(np.abs(out)) * L


def test_projector_identities():
    """eta = 0, f = 0: v' = P v.  P P = P and P G p = 0."""
    L = 8
    prm = oracle.params(L, rho=1.0, eta=0.0, dt=1.0)
    rng = np.random.default_rng(3)
    z = np.zeros((3, L, L, L))
    Pv = oracle.fluid_solve(prm, rng.standard_normal((3, L, L, L)), z)
    PPv = oracle.fluid_solve(prm, Pv, z)
    assert np.max(np.abs(PPv - Pv)) < 1e-13
    p = rng.standard_normal((L, L, L))
    # G = -D^T: (G p)_a at the face c + e_a/2 is (p[c + e_a] - p[c]) / h
    Gp = np.stack([np.roll(p, -1, axis=2) - p, np.roll(p, -1, axis=1) - p, np.roll(p, -1, axis=0) - p])
    out = oracle.fluid_solve(prm, z, Gp)
    assert np.max(np.abs(out)) < 1e-13


@pytest.mark.parametrize("m", [1, 3])
def test_shear_mode_decay(m):
    """v_x = A sin(2 pi m y / L): each Crank-Nicolson step multiplies the
    amplitude by g = (1 - nu dt lam / 2) / (1 + nu dt lam / 2) with
    lam = (4/h^2) sin^2(pi m / L), exactly; lam -> k^2 recovers the paper's
    exp(-nu k^2 t) decay as h -> 0."""
    L, h, rho, eta, dt, steps = 32, 1.0, 1.0, 1.0, 0.5, 4
    nu = eta / rho
    y = np.arange(L) * h
    v = np.zeros((3, L, L, L))
    v[0] = np.sin(2 * np.pi * m * y / (L * h))[None, :, None]
    prm = oracle.params(L, h=h, rho=rho, eta=eta, dt=dt)
    z = np.zeros_like(v)
    out = v
    for _ in range(steps):
        out = oracle.fluid_solve(prm, out, z)
    lam = 4 / h ** 2 * np.sin(np.pi * m / L) ** 2
    g = (1 - nu * dt * lam / 2) / (1 + nu * dt * lam / 2)
    assert np.max(np.abs(out - g ** steps * v)) < 1e-13
    if m == 1:
        k2 = (2 * np.pi / (L * h)) ** 2
        cont = np.exp(-nu * k2 * dt * steps)
        assert abs(g ** steps - cont) / cont < 2e-3


def test_steady_sinusoid_viscosity():
    """f = f0 sin(k y) x: steady v_x = f0 sin(k y) / (eta lam); the paper's
    viscosity estimate eta = f0 / (k^2 v_x) holds up to (k h)^2 / 12."""
    L, h, eta, f0 = 32, 1.0, 2.5, 0.3
    y = np.arange(L) * h
    k = 2 * np.pi / (L * h)
    f = np.zeros((3, L, L, L))
    f[0] = f0 * np.sin(k * y)[None, :, None]
    prm = oracle.params(L, h=h, eta=eta, steady=True, zero_mean=True)
    out = oracle.fluid_solve(prm, np.zeros_like(f), f)
    lam = 4 / h ** 2 * np.sin(np.pi / L) ** 2
    assert np.max(np.abs(out[0] - f[0] / (eta * lam))) < 1e-12
    assert np.max(np.abs(out[1:])) < 1e-14
    vx = f0 / (eta * lam)
    eta_est = f0 / (k ** 2 * vx)
    assert abs(eta_est - eta) / eta < (k * h) ** 2 / 12 * 1.01


def test_mean_mode():
    """Unsteady: mean(v') = mean(v) + dt/rho mean(f) (momentum balance);
    zero_mean holds it at zero."""
    L = 6
    rng = np.random.default_rng(1)
    v = rng.standard_normal((3, L, L, L))
    f = rng.standard_normal((3, L, L, L))
    prm = oracle.params(L, rho=2.0, eta=0.3, dt=0.1)
    out = oracle.fluid_solve(prm, v, f)
    assert np.allclose(out.reshape(3, -1).mean(1), v.reshape(3, -1).mean(1) + 0.05 * f.reshape(3, -1).mean(1), atol=1e-14)
    prm0 = oracle.params(L, rho=2.0, eta=0.3, dt=0.1, zero_mean=True)
    assert np.allclose(oracle.fluid_solve(prm0, v, f).reshape(3, -1).mean(1), 0.0, atol=1e-14)
