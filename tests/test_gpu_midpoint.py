"""The second-order step (MB_SCHEME_MIDPOINT) on the GPU against the oracle's
midpoint step, its order of convergence measured on the GPU, and its
captured-graph replays against eager steps."""
import sys

import numpy as np
import pytest

import oracle
from paper_1407_5600_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_5600_amd  # noqa: F401
    return torch


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def _case(torch, w, prec, nsteps, mode="unsteady", v0=None, f_fluid=None):
    from paper_1407_5600_amd import Grid, Springs
    steady = mode == "steady"
    g = Grid(w.L, precision=prec, mode=mode, zero_mean=steady, max_blobs=w.M, rho=w.rho,
             eta=w.eta, dt=w.dt, scheme="midpoint")
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    q = dev(torch, w.q)
    v = g.field() if v0 is None else torch.from_numpy(v0).to(g.field_dtype).cuda()
    vstart = v.double().cpu().numpy()
    u = torch.zeros_like(q)
    U0 = torch.zeros((w.P, 3), dtype=torch.float64, device="cuda")
    diag = torch.zeros(7, dtype=torch.float64, device="cuda")
    if f_fluid is None:
        g.step(sp, q, v, dev(torch, w.Fext), nsteps, u, U0, diag)
        ff = None
    else:
        fd = torch.from_numpy(f_fluid).to(g.field_dtype).cuda()
        g.step_forced(sp, q, v, fd, Fext=dev(torch, w.Fext), nsteps=nsteps, u_out=u,
                      U0_out=U0, diag_out=diag)
        ff = fd.double().cpu().numpy()
    torch.cuda.synchronize()
    prm = oracle.params(w.L, rho=w.rho, eta=w.eta, dt=w.dt, steady=steady, zero_mean=steady)
    r = oracle.step(prm, w.springs(), w.q, vstart, w.Fext, nsteps, f_fluid=ff,
                    scheme="midpoint")
    tol = TOL[prec]
    errs = {"u": rel(u.cpu().numpy(), r["u"]), "U0": rel(U0.cpu().numpy(), r["U0"]),
            "v": rel(v.double().cpu().numpy(), r["v"])}
    # positions: the GPU adds the two halves of the update one at a time,
    # the oracle their sum, each rounded to the ulp of |q|
    qg = q.cpu().numpy()
    dq_ref = r["q"] - w.q
    ulp = np.spacing(np.abs(r["q"]).max())
    bound = tol * np.abs(dq_ref).max() + 3 * nsteps * ulp
    say(prec, mode, " ".join(f"{k} {e:.2e}" for k, e in errs.items()),
        f"dq max err {np.abs(qg - r['q']).max():.2e} (bound {bound:.2e})")
    for k, e in errs.items():
        assert e < tol, (k, e)
    assert np.abs(qg - r["q"]).max() <= bound
    d = diag.cpu().numpy()
    Fmag = np.abs(oracle.spring_forces(w.P, w.nb, w.pa, w.pb, w.r0, w.k, r["q"], w.Fext)).sum(0)
    assert np.abs(d[3:6] - r["diag"][3:6]).max() < tol * np.linalg.norm(Fmag)
    if not steady:
        pscale = w.rho * np.abs(r["v"]).sum(axis=(1, 2, 3))
        assert np.abs(d[:3] - r["diag"][:3]).max() < tol * np.linalg.norm(pscale)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("mode", ["unsteady", "steady"])
def test_midpoint_vs_oracle(torch_cuda, prec, mode):
    torch = torch_cuda
    say("midpoint", prec, mode)
    w = inputs.random_suspension(31, 32, 40)
    L = w.L
    v0 = None
    if mode == "unsteady":
        v0 = oracle.fluid_solve(oracle.params(L, eta=0.0),
                                0.1 * np.random.default_rng(5).standard_normal((3, L, L, L)),
                                np.zeros((3, L, L, L)))
    _case(torch, w, prec, 3, mode, v0=v0)


def test_midpoint_forced_vs_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1407_5600_amd.stokes import shear_force_field
    say("midpoint forced steady")
    w = inputs.random_suspension(32, 24, 15)
    _case(torch, w, "fp64", 3, "steady", f_fluid=shear_force_field(w.L, 0.2))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_midpoint_dense_full_size(torch_cuda, prec):
    """The 128^3, phi = 0.3 suspension (476,697 blobs), one midpoint step,
    every output against the oracle."""
    torch = torch_cuda
    say("midpoint dense 128^3", prec)
    w = inputs.cached("dense")
    _case(torch, w, prec, 1)


@pytest.mark.parametrize("mode", ["unsteady", "steady"])
def test_orders_of_convergence_on_gpu(torch_cuda, mode):
    """Two deformed particles in a random flow over T = 0.4: positions
    converge at rate 2 with the midpoint scheme and at rate 1 with the
    first-order one (float64 GPU runs against a fine-step GPU run)."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid, Springs
    say("convergence", mode)
    steady = mode == "steady"
    L, T = 16, 0.4
    t = inputs.icosahedron_template(1.0)
    pa, pb, r0 = inputs.pair_table(t)
    sp = Springs(13, pa, pb, r0, 100.0)
    rng = np.random.default_rng(3)
    c = np.array([[5.3, 6.1, 4.7], [9.2, 10.9, 8.6]])
    q0 = inputs.place_particles(c, t, inputs.random_rotations(rng, 2)) \
        + 0.05 * rng.standard_normal((26, 3))
    v0 = np.zeros((3, L, L, L)) if steady else oracle.fluid_solve(
        oracle.params(L, eta=0.0), 0.3 * rng.standard_normal((3, L, L, L)),
        np.zeros((3, L, L, L)))
    Fe = np.array([[1.0, 0.5, 0.0], [-0.5, 0.0, 1.0]])

    def run(scheme, n):
        g = Grid(L, dt=T / n, mode=mode, zero_mean=steady, max_blobs=26, scheme=scheme)
        q = dev(torch, q0)
        v = dev(torch, v0)
        g.step(sp, q, v, dev(torch, Fe), n)
        return q.cpu().numpy()
    qref = run("midpoint", 256)
    for scheme, order in (("euler", 1), ("midpoint", 2)):
        e = [np.abs(run(scheme, n) - qref).max() for n in (16, 32, 64)]
        rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        say(scheme, [f"{x:.3e}" for x in e], np.round(rates, 3).tolist())
        assert np.all(np.abs(rates - order) < 0.25)


def test_midpoint_graph_replays_match_eager(torch_cuda):
    """Batch grids on the midpoint scheme stepped by the captured graph and
    eagerly: bitwise equal after every replay."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid, Springs
    from paper_1407_5600_amd.binding import step_graph
    say("midpoint graph replays")
    tmpl = inputs.icosahedron_template(1.0)
    pa, pb, r0 = inputs.pair_table(tmpl)
    sp = Springs(13, pa, pb, r0, 100.0)
    specs = [(24, 3, "fp64", "unsteady"), (32, 2, "mixed", "steady")]
    G, E, qs, qe, vs, ve, fe = [], [], [], [], [], [], []
    for L, nbox, prec, mode in specs:
        boxes = inputs.pair_sweep(seed=L, nbox=10 * nbox, sizes=(L,))[:nbox]
        q = np.concatenate([b["q"] for b in boxes])
        for lg, lq, lv in ((G, qs, vs), (E, qe, ve)):
            g = Grid(L, precision=prec, mode=mode, zero_mean=mode == "steady",
                     max_blobs=len(q), nbox=nbox, scheme="midpoint")
            lg.append(g)
            lq.append(dev(torch, q))
            lv.append(g.field())
        fe.append(dev(torch, np.concatenate([b["Fext"] for b in boxes])))
    for reps in (4, 1, 3):
        step_graph(G, [sp, sp], qs, vs, fe, None, reps)
        for g, q, v, F in zip(E, qe, ve, fe):
            g.step(sp, q, v, F, reps)
        torch.cuda.synchronize()
        for a, b in zip(qs + vs, qe + ve):
            assert torch.equal(a, b)


def test_adjoint_rejects_midpoint(torch_cuda):
    torch = torch_cuda
    from paper_1407_5600_amd import Grid, MultiblobError, Springs
    tmpl = inputs.icosahedron_template(1.0)
    pa, pb, r0 = inputs.pair_table(tmpl)
    sp = Springs(13, pa, pb, r0, 100.0)
    g = Grid(16, max_blobs=13, scheme="midpoint")
    q = dev(torch, inputs.place_particles(np.full((1, 3), 8.0), tmpl))
    v = g.field()
    with pytest.raises(MultiblobError):
        g.step_adjoint(sp, q, v, torch.zeros_like(q), g.field())
