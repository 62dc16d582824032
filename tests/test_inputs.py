"""Checks of the seeded input generators (no method arithmetic here)."""
import numpy as np
from scipy.spatial import cKDTree

from paper_1407_5600_amd import inputs


def test_template():
    t = inputs.icosahedron_template(1.0)
    assert t.shape == (13, 3)
    assert np.allclose(np.linalg.norm(t[:12], axis=1), 1.0)
    assert np.allclose(t[12], 0.0)
    assert np.allclose(t.mean(0), 0.0, atol=1e-15)


def test_particle_count_for_fraction():
    assert inputs.particles_for_fraction(128, 0.3) == 36669
    assert inputs.particles_for_fraction(256, 0.4) == 391139


def test_rsa_nonoverlap_and_determinism():
    rng = np.random.default_rng(5)
    c = inputs.rsa_centres(rng, 24.0, 200)
    tr = cKDTree(c % 24.0, boxsize=24.0)
    assert len(tr.query_pairs(3.2 - 1e-12)) == 0
    c2 = inputs.rsa_centres(np.random.default_rng(5), 24.0, 200)
    assert np.array_equal(c, c2)


def test_lattice_nonoverlap():
    c = inputs.lattice_centres(np.random.default_rng(1), 40.0, 1500)
    tr = cKDTree(c, boxsize=40.0)
    assert len(tr.query_pairs(3.2 - 1e-12)) == 0


def test_rotations_orthonormal():
    R = inputs.random_rotations(np.random.default_rng(0), 50)
    assert np.allclose(np.einsum("pij,pkj->pik", R, R), np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(R), 1.0)


def test_single_workload():
    w = inputs.single()
    assert w.L == 32 and w.M == 13 and w.P == 1
    assert np.allclose(w.Fext, [[1, 0, 0]])
    assert len(w.pa) == 78


def test_hard_sphere_centres_no_overlap_and_moved():
    """Monte Carlo hard-sphere configurations: n centres in the box, every
    minimum-image pair at least 2R apart, and the sweeps moved the spheres
    away from their starting configuration."""
    from paper_1407_5600_amd import inputs as I
    L, R = 24.0, 1.62
    n = I.particles_for_fraction(L, 0.15, R)
    c0 = I.hard_sphere_centres(np.random.default_rng(5), L, n, R, sweeps=0)
    c = I.hard_sphere_centres(np.random.default_rng(5), L, n, R, sweeps=10)
    assert c.shape == (n, 3) and np.all((c >= 0) & (c < L))
    d = c[:, None] - c[None]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, np.inf)
    assert r.min() >= 2 * R
    assert np.abs(c - c0).max() > 0.1


def test_hard_sphere_sweeps_keep_spheres_apart():
    """The checkerboard Monte Carlo moves spheres (from a dense lattice start)
    without ever letting two come closer than dmin, with an acceptance near
    its target."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(3)
    L, n, dmin = 48.0, 2000, 3.2
    c = inputs.lattice_centres(rng, L, n, dmin=dmin)
    c0 = c.copy()
    out = inputs.hard_sphere_sweeps(rng, c, L, dmin, 8, 0.2)
    assert len(out["acceptance"]) == 8 and 0.2 < np.mean(out["acceptance"][2:]) < 0.6
    assert not cKDTree(c % L, boxsize=L).query_pairs(dmin * (1 - 1e-12))
    d = c - c0
    d -= L * np.round(d / L)
    assert np.sqrt((d * d).sum(1)).mean() > 0.1


def test_cached_reloads_array_extras(tmp_path, monkeypatch):
    monkeypatch.setenv("MB_INPUT_CACHE", str(tmp_path))
    a = inputs.cached("diff")
    b = inputs.cached("diff")  # from the file
    for k in ("centres", "rotations", "V"):
        assert np.array_equal(a.extra[k], b.extra[k])
    assert np.array_equal(a.q, b.q)


def test_pair_sweep_boxes():
    """Boxes of the pair sweep: edges from the set, the two centres along x
    at the drawn separation about the box middle, forces +-x; the rotated
    variant keeps every box (edge, separation, centres) and only turns the
    particles about their centres."""
    tmpl = inputs.icosahedron_template(inputs.CIRCUMRADIUS_OVER_EDGE)
    a = inputs.pair_sweep(seed=7, nbox=40, template=tmpl)
    b = inputs.pair_sweep(seed=7, nbox=40, template=tmpl, rotate=True)
    nb = tmpl.shape[0]
    for x, y in zip(a, b):
        assert x["L"] in (24, 32, 48, 64) and 2.0 <= x["sep"] <= 6.0
        assert x["L"] == y["L"] and x["sep"] == y["sep"]
        np.testing.assert_array_equal(x["c"], y["c"])
        d = x["c"][1] - x["c"][0]
        np.testing.assert_allclose(d, [x["sep"], 0.0, 0.0], atol=1e-12)
        assert np.all(np.abs(x["c"].mean(0) - x["L"] / 2) <= 0.5)
        np.testing.assert_array_equal(x["Fext"], [[1.0, 0, 0], [-1.0, 0, 0]])
        for j in (0, 1):
            qa, qb = x["q"][j * nb:(j + 1) * nb], y["q"][j * nb:(j + 1) * nb]
            np.testing.assert_allclose(qa.mean(0), x["c"][j], atol=1e-12)
            np.testing.assert_allclose(qb.mean(0), x["c"][j], atol=1e-12)
            # same shape: pairwise blob distances agree
            da = np.linalg.norm(qa[:, None] - qa[None], axis=-1)
            db = np.linalg.norm(qb[:, None] - qb[None], axis=-1)
            np.testing.assert_allclose(da, db, atol=1e-12)
        assert not np.allclose(x["q"], y["q"])
