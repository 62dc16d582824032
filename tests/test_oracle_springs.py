"""Pins of the oracle's spring forces: F = -grad E by central differences,
zero net internal force, zero force in the template state, and the template
geometry itself (Fig. 1, Sec. Multiblob particle model)."""
import numpy as np

import oracle
from paper_1407_5600_amd import inputs


def _energy(q, pa, pb, r0, k, nb):
    P = q.shape[0] // nb
    E = 0.0
    for p in range(P):
        for a, b, r in zip(pa, pb, r0):
            d = q[p * nb + b] - q[p * nb + a]
            E += 0.5 * k * (np.sqrt(d @ d) - r) ** 2
    return E


def _setup(seed=0, P=3):
    tmpl = inputs.icosahedron_template(1.0)
    pa, pb, r0 = inputs.pair_table(tmpl)
    rng = np.random.default_rng(seed)
    R = inputs.random_rotations(rng, P)
    q = inputs.place_particles(rng.uniform(0, 20, (P, 3)), tmpl, R)
    return tmpl, pa, pb, r0, q, rng


def test_template_pairs():
    """78 pairs; rest lengths 1.0515 a (30 edges), 1.7013 a (30), 2 a (6
    antipodes), a (12 centre pairs)."""
    tmpl, pa, pb, r0, _, _ = _setup()
    assert len(pa) == 78
    vals, counts = np.unique(np.round(r0, 4), return_counts=True)
    assert list(vals) == [1.0, 1.0515, 1.7013, 2.0]
    assert list(counts) == [12, 30, 30, 6]


def test_rest_state_only_external():
    tmpl, pa, pb, r0, q, rng = _setup()
    Fext = rng.standard_normal((3, 3))
    F = oracle.spring_forces(3, 13, pa, pb, r0, 100.0, q, Fext)
    assert np.allclose(F, np.repeat(Fext / 13.0, 13, axis=0), atol=1e-12)


def test_minus_gradient_and_net_force():
    tmpl, pa, pb, r0, q, rng = _setup(1)
    q = q + 0.05 * rng.standard_normal(q.shape)
    k = 100.0
    F = oracle.spring_forces(3, 13, pa, pb, r0, k, q, None)
    eps = 1e-6
    G = np.zeros_like(q)
    for i in range(q.shape[0]):
        for c in range(3):
            qp = q.copy(); qp[i, c] += eps
            qm = q.copy(); qm[i, c] -= eps
            G[i, c] = (_energy(qp, pa, pb, r0, k, 13) - _energy(qm, pa, pb, r0, k, 13)) / (2 * eps)
    assert np.max(np.abs(F + G)) < 1e-6 * max(1.0, np.max(np.abs(F)))
    # internal forces sum to zero per particle
    assert np.max(np.abs(F.reshape(3, 13, 3).sum(1))) < 1e-12 * np.max(np.abs(F))


def test_stretched_pair_direction():
    """Two blobs stretched apart attract along their separation."""
    q = np.array([[0.0, 0, 0], [2.0, 0, 0]])
    F = oracle.spring_forces(1, 2, [0], [1], [1.5], 10.0, q, None)
    assert np.allclose(F, [[5.0, 0, 0], [-5.0, 0, 0]])
