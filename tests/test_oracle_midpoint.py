"""The oracle's second-order step (midpoint predictor-corrector rebuilt from
eqs. vf, ju and blob1 with m_e = 0) pinned by what fixes it independently of
its code: the order of convergence in dt against a fine-step solution (2 for
the midpoint step, 1 for the first-order step), the exact momentum balance of
eq. vf and the exact translation of blobs in a uniform flow."""
import numpy as np
import pytest

import oracle
from paper_1407_5600_amd import inputs

L = 12
T = 0.4


def _case(steady):
    t = inputs.icosahedron_template(1.0)
    pa, pb, r0 = inputs.pair_table(t)
    sp = {"nb": 13, "pa": pa, "pb": pb, "r0": r0, "k": 100.0}
    rng = np.random.default_rng(3)
    c = np.array([[5.3, 6.1, 4.7], [8.2, 3.9, 7.6]])
    # deformed particles (springs ringing) in a random solenoidal flow
    q0 = inputs.place_particles(c, t, inputs.random_rotations(rng, 2)) \
        + 0.05 * rng.standard_normal((26, 3))
    v0 = oracle.fluid_solve(oracle.params(L, eta=0.0), 0.3 * rng.standard_normal((3, L, L, L)),
                            np.zeros((3, L, L, L)))
    Fe = np.array([[1.0, 0.5, 0.0], [-0.5, 0.0, 1.0]])

    def run(scheme, nst):
        prm = oracle.params(L, dt=T / nst, steady=steady, zero_mean=steady)
        r = oracle.step(prm, sp, q0, np.zeros_like(v0) if steady else v0, Fe, nst,
                        scheme=scheme)
        return r["q"], r["v"]
    return run


@pytest.mark.parametrize("steady", [False, True])
def test_orders_of_convergence(steady):
    run = _case(steady)
    qref, vref = run("midpoint", 256)
    for scheme, order in (("euler", 1), ("midpoint", 2)):
        eq = [np.abs(run(scheme, n)[0] - qref).max() for n in (16, 32, 64)]
        rates = np.log2(np.array(eq[:-1]) / np.array(eq[1:]))
        assert np.all(np.abs(rates - order) < 0.25), (scheme, eq, rates)
    if not steady:
        ev = [np.abs(run("midpoint", n)[1] - vref).max() for n in (16, 32, 64)]
        rates = np.log2(np.array(ev[:-1]) / np.array(ev[1:]))
        assert np.all(np.abs(rates - 2) < 0.25), (ev, rates)


def test_midpoint_momentum_balance():
    """Mean mode evolved: the momentum grows by dt sum Fext per step exactly
    (the springs cancel pairwise), with the forces taken at q*."""
    w = inputs.random_suspension(5, 12, 3)
    prm = oracle.params(w.L, rho=w.rho, eta=w.eta, dt=w.dt)
    r = oracle.step(prm, w.springs(), w.q, np.zeros((3, w.L, w.L, w.L)), w.Fext, 4,
                    scheme="midpoint")
    assert np.abs(r["diag"][:3] - 4 * w.dt * w.Fext.sum(0)).max() < 1e-13
    assert np.abs(r["diag"][3:6] - w.Fext.sum(0)).max() < 1e-12


@pytest.mark.parametrize("scheme", ["euler", "midpoint"])
def test_uniform_flow_translates_blobs(scheme):
    """No forces, uniform v: the blobs move by n dt U exactly (J interpolates
    constants exactly; the solve leaves the mean mode alone)."""
    w = inputs.random_suspension(6, 12, 2)
    U = np.array([0.3, -0.2, 0.1])
    v0 = np.broadcast_to(U[:, None, None, None], (3, w.L, w.L, w.L)).copy()
    sp = dict(w.springs(), k=0.0)
    prm = oracle.params(w.L, rho=w.rho, eta=w.eta, dt=w.dt)
    r = oracle.step(prm, sp, w.q, v0, np.zeros_like(w.Fext), 5, scheme=scheme)
    assert np.abs(r["q"] - (w.q + 5 * w.dt * U)).max() < 1e-12
    assert np.abs(r["v"] - v0).max() < 1e-13
