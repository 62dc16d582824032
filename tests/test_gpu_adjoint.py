"""Differentiation on the GPU: the adjoint kernels against the oracle's
reverse-mode derivatives (which the CPU suite pins by finite differences),
and the gradients of the 64^3, 16-particle, 100-step trajectory loss against
central finite differences of the GPU forward (step 1e-6, float64)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1407_5600_amd import inputs

pytestmark = pytest.mark.gpu


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


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("pos", ["random", "ties"])
@pytest.mark.parametrize("prec,L", [("fp64", 16), ("fp64", 24), ("mixed", 16)])
def test_interpolate_grad_vs_oracle(torch_cuda, prec, L, pos):
    """The position derivative of the interpolation against the oracle's;
    "ties": integer and half-integer coordinates, where the offset of a node
    set is exactly +-1/2 (the kernel's derivative is continuous there, and
    the node at distance 3/2 has zero weight and zero slope)."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid
    say("interp grad", prec, L, pos)
    rng = np.random.default_rng(L)
    M = 500
    q = rng.uniform(0, L, (M, 3))
    if pos == "ties":
        q = rng.integers(0, L + 1, (M, 3)) + rng.choice([0.0, 0.5], (M, 3))
        q[::5, 2] = rng.uniform(0, L, q[::5, 2].shape)
    q[:50] += rng.integers(-3, 3, (50, 3)) * L  # unwrapped positions
    v = rng.standard_normal((3, L, L, L))
    W = rng.standard_normal((M, 3))
    g = Grid(L, precision=prec, max_blobs=M)
    vt = torch.from_numpy(v).to(g.field_dtype).cuda()
    out = g.interpolate_grad(dev(torch, q), vt, dev(torch, W))
    torch.cuda.synchronize()
    ref = oracle.interpolate_grad(oracle.params(L), q, vt.double().cpu().numpy(), W)
    r = rel(out.cpu().numpy(), ref)
    say(f"rel err {r:.3e}")
    assert r < (1e-12 if prec == "fp64" else 1e-5)


def test_spring_adjoint_vs_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1407_5600_amd import Springs, spring_adjoint
    say("spring adjoint")
    tmpl = inputs.icosahedron_template(1.0)
    pa, pb, r0 = inputs.pair_table(tmpl)
    rng = np.random.default_rng(7)
    P, nb, k = 40, len(tmpl), 37.0
    R = inputs.random_rotations(rng, P)
    q = inputs.place_particles(rng.uniform(0, 30, (P, 3)), tmpl, R)
    q += 0.05 * rng.standard_normal(q.shape)
    Fbar = rng.standard_normal(q.shape)
    sp = Springs(nb, pa, pb, r0, k)
    qbar = torch.zeros((P * nb, 3), dtype=torch.float64, device="cuda")
    kbar = torch.zeros(1, dtype=torch.float64, device="cuda")
    r0bar = torch.zeros(len(pa), dtype=torch.float64, device="cuda")
    spring_adjoint(sp, dev(torch, q), dev(torch, Fbar), qbar, kbar, r0bar)
    torch.cuda.synchronize()
    rq, rk, rr = oracle.spring_adjoint(P, nb, pa, pb, r0, k, q, Fbar)
    assert rel(qbar.cpu().numpy(), rq) < 1e-12
    assert abs(kbar.item() - rk) <= 1e-12 * abs(rk)
    assert rel(r0bar.cpu().numpy(), rr) < 1e-12


def _oracle_traj_blob_forces(prm, sp, q, v, G, n):
    """Forward of the per-blob-force step from the oracle's pinned parts."""
    q = q.copy()
    v = v.copy()
    P = q.shape[0] // sp["nb"]
    for _ in range(n):
        F = oracle.spring_forces(P, sp["nb"], sp["pa"], sp["pb"], sp["r0"], sp["k"], q,
                                 None) + G
        v = oracle.fluid_solve(prm, v, oracle.spread(prm, q, F))
        u = oracle.interpolate(prm, q, v)
        q = q + prm.dt * u
    return q, v, u


def _small_case(seed=5, L=16, h=1.0):
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
    sp = {"nb": nb, "pa": pa, "pb": pb, "r0": np.array(r0, dtype=float), "k": 20.0}
    return sp, q0, v0, G, V


def test_step_ext_per_blob_forces_vs_oracle(torch_cuda):
    torch = torch_cuda
    from paper_1407_5600_amd import Grid, Springs
    say("step_ext")
    L, n = 16, 4
    sp, q0, v0, G, V = _small_case()
    prm = oracle.params(L, dt=0.05)
    g = Grid(L, dt=0.05, max_blobs=q0.shape[0])
    s = Springs(sp["nb"], sp["pa"], sp["pb"], sp["r0"], sp["k"])
    q = dev(torch, q0)
    v = dev(torch, v0)
    u = torch.empty_like(q)
    g.step_ext(s, q, v, None, dev(torch, G), n, u_out=u)
    torch.cuda.synchronize()
    rq, rv, ru = _oracle_traj_blob_forces(prm, sp, q0, v0, G, n)
    assert rel(q.cpu().numpy() - q0, rq - q0) < 1e-12
    assert rel(v.cpu().numpy(), rv) < 1e-12
    assert rel(u.cpu().numpy(), ru) < 1e-12


def _gpu_loss_grad(torch, g, sp, q0, v0, G, V, n, every):
    from paper_1407_5600_amd.autodiff import particle_means, trajectory
    q0t = dev(torch, q0).requires_grad_(True)
    v0t = dev(torch, v0).requires_grad_(True)
    Gt = dev(torch, G).requires_grad_(True)
    kt = torch.tensor(float(sp["k"]), dtype=torch.float64, device="cuda", requires_grad=True)
    r0t = dev(torch, sp["r0"]).requires_grad_(True)
    u = trajectory(g, sp["nb"], sp["pa"], sp["pb"], q0t, v0t, Gt, kt, r0t, n, every)
    loss = ((particle_means(u, sp["nb"]) - dev(torch, V)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return loss.item(), {"q0": q0t.grad.cpu().numpy(), "v0": v0t.grad.cpu().numpy(),
                         "G": Gt.grad.cpu().numpy(), "k": kt.grad.item(),
                         "r0": r0t.grad.cpu().numpy()}


@pytest.mark.parametrize("mode,h", [("unsteady", 1.0), ("zero_mean", 1.0), ("steady", 1.0),
                                    ("unsteady", 0.8)])
def test_trajectory_gradient_vs_oracle(torch_cuda, mode, h):
    """Five steps with checkpoints every two (segments 2, 2, 1): loss and all
    gradients against the oracle's reverse sweep."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid
    say("trajectory grad", mode, h)
    L, n = 16, 5
    sp, q0, v0, G, V = _small_case(h=h)
    steady = mode == "steady"
    zm = mode != "unsteady"
    prm = oracle.params(L, h=h, dt=0.05, steady=steady, zero_mean=zm)
    g = Grid(L, h=h, dt=0.05, mode="steady" if steady else "unsteady", zero_mean=zm,
             max_blobs=q0.shape[0])
    loss, gr = _gpu_loss_grad(torch, g, sp, q0, v0, G, V, n, 2)
    rloss, rg = oracle.loss_grad(prm, sp, q0, v0, G, V, n)
    say(f"loss {loss:.12e} oracle {rloss:.12e}")
    assert abs(loss - rloss) <= 1e-12 * abs(rloss)
    for key in ("q0", "G", "r0") + (() if steady else ("v0",)):
        r = rel(gr[key], rg[key])
        say(f"grad {key}: rel err {r:.3e}")
        assert r < 1e-12, key
    assert abs(gr["k"] - rg["k"]) <= 1e-12 * max(abs(rg["k"]), 1e-12)


def _diff_setup(torch):
    w = inputs.diff()
    G = np.repeat(w.Fext / w.nb, w.nb, axis=0)
    unit = inputs.icosahedron_template(1.0)
    _, _, r0u = inputs.pair_table(unit)
    return w, G, unit, np.array(r0u, dtype=float)


def _diff_loss(torch, g, w, G, unit, r0u, k, a, nsteps, grad=False):
    from paper_1407_5600_amd.autodiff import particle_means, place_template, trajectory
    at = torch.tensor(float(a), dtype=torch.float64, device="cuda", requires_grad=grad)
    kt = torch.tensor(float(k), dtype=torch.float64, device="cuda", requires_grad=grad)
    Gt = dev(torch, G).requires_grad_(grad)
    q0 = place_template(dev(torch, w.extra["centres"]), dev(torch, w.extra["rotations"]),
                        dev(torch, unit), at)
    r0 = at * dev(torch, r0u)
    v0 = torch.zeros((3, w.L, w.L, w.L), dtype=torch.float64, device="cuda")
    u = trajectory(g, w.nb, w.pa, w.pb, q0, v0, Gt, kt, r0, nsteps, 10)
    loss = ((particle_means(u, w.nb) - dev(torch, w.extra["V"])) ** 2).sum()
    if grad:
        loss.backward()
        torch.cuda.synchronize()
        return loss.item(), Gt.grad.cpu().numpy(), kt.grad.item(), at.grad.item()
    torch.cuda.synchronize()
    return loss.item()


def test_diff_workload_gradients_vs_finite_differences(torch_cuda):
    """64^3, 16 particles, 100 steps of dt = 0.01, checkpoints every 10:
    gradients of sum_p |U_p - V_p|^2 with respect to the 624 blob-force
    components, the stiffness k and the vertex radius a against central
    differences of the GPU forward.

    At the step 1e-6 the difference quotient carries the forward's rounding
    noise (about 1e-13 of the loss over 100 steps, divided by 2e-6), so the
    adjoint is held to 1e-6 of the gradient's norm there; with steps where
    truncation and rounding balance (1e-4 for forces and radius, 1e-2 for k)
    each component is held to 1e-6 of itself."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid
    say("diff workload FD")
    w, G, unit, r0u = _diff_setup(torch)
    g = Grid(w.L, dt=w.dt, max_blobs=w.M)
    n, k, a = w.steps, w.k, 1.0
    loss, gG, gk, ga = _diff_loss(torch, g, w, G, unit, r0u, k, a, n, grad=True)
    gnorm = float(np.sqrt(np.sum(gG ** 2) + gk ** 2 + ga ** 2))
    say(f"loss {loss:.6e}  |grad| {gnorm:.3e}  dk {gk:.3e}  da {ga:.3e}")
    rng = np.random.default_rng(0)
    idx = rng.choice(G.size, 8, replace=False)
    d = rng.standard_normal(G.shape)
    d /= np.linalg.norm(d)

    def fd_G(i, e):
        Gp, Gm = G.copy(), G.copy()
        Gp.flat[i] += e
        Gm.flat[i] -= e
        return (_diff_loss(torch, g, w, Gp, unit, r0u, k, a, n) -
                _diff_loss(torch, g, w, Gm, unit, r0u, k, a, n)) / (2 * e)

    def fd_dir(e):
        return (_diff_loss(torch, g, w, G + e * d, unit, r0u, k, a, n) -
                _diff_loss(torch, g, w, G - e * d, unit, r0u, k, a, n)) / (2 * e)

    def fd_k(e):
        return (_diff_loss(torch, g, w, G, unit, r0u, k + e, a, n) -
                _diff_loss(torch, g, w, G, unit, r0u, k - e, a, n)) / (2 * e)

    def fd_a(e):
        return (_diff_loss(torch, g, w, G, unit, r0u, k, a + e, n) -
                _diff_loss(torch, g, w, G, unit, r0u, k, a - e, n)) / (2 * e)

    ad = {f"G[{i}]": gG.flat[i] for i in idx}
    ad["G.d"] = float(np.sum(gG * d))
    ad["k"] = gk
    ad["a"] = ga
    # the step 1e-6: norm-wise
    fd6 = {f"G[{i}]": fd_G(i, 1e-6) for i in idx}
    fd6["G.d"] = fd_dir(1e-6)
    fd6["k"] = fd_k(1e-6)
    fd6["a"] = fd_a(1e-6)
    for name in ad:
        err = abs(ad[name] - fd6[name])
        say(f"step 1e-6 {name}: adjoint {ad[name]:.10e} fd {fd6[name]:.10e} "
            f"err/|grad| {err / gnorm:.2e}")
        assert err <= 1e-6 * gnorm, name
    # balanced steps: component-wise
    fdb = {f"G[{i}]": fd_G(i, 1e-4) for i in idx[:4]}
    fdb["G.d"] = fd_dir(1e-4)
    fdb["k"] = fd_k(1e-2)
    fdb["a"] = fd_a(1e-4)
    for name in fdb:
        rel_err = abs(ad[name] - fdb[name]) / abs(fdb[name])
        say(f"balanced step {name}: adjoint {ad[name]:.10e} fd {fdb[name]:.10e} rel {rel_err:.2e}")
        assert rel_err <= 1e-6, name


def test_fit_stiffness_and_radius_to_target_mobilities(torch_cuda):
    """Fit k and the vertex radius a of the 16 particles of the 64^3 case
    to the blob velocities (rigid motion and deformation) produced with
    (k, a) = (60, 1.08), from (100, 1.0), by Adam on (log k, a) with the
    adjoint gradients (30-step trajectories)."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid
    from paper_1407_5600_amd.autodiff import place_template, trajectory
    say("fit k and a")
    w, G, unit, r0u = _diff_setup(torch)
    g = Grid(w.L, dt=w.dt, max_blobs=w.M)
    n = 30
    c = dev(torch, w.extra["centres"])
    R = dev(torch, w.extra["rotations"])
    tu = dev(torch, unit)
    r0t = dev(torch, r0u)
    Gt = dev(torch, G)
    v0 = torch.zeros((3, w.L, w.L, w.L), dtype=torch.float64, device="cuda")

    def u_of(k, a):
        return trajectory(g, w.nb, w.pa, w.pb, place_template(c, R, tu, a), v0, Gt, k,
                          a * r0t, n, 10)

    with torch.no_grad():
        target = u_of(torch.tensor(60.0, dtype=torch.float64, device="cuda"),
                      torch.tensor(1.08, dtype=torch.float64, device="cuda")).clone()
    logk = torch.tensor(np.log(100.0), dtype=torch.float64, device="cuda", requires_grad=True)
    a = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([logk, a], lr=0.05)
    losses = []
    for it in range(200):
        opt.zero_grad()
        loss = ((u_of(torch.exp(logk), a) - target) ** 2).sum()
        loss.backward()
        opt.step()
        losses.append(loss.item())
        if it % 40 == 0:
            say(f"it {it}: loss {losses[-1]:.3e} k {torch.exp(logk).item():.3f} a {a.item():.5f}")
    kf, af = torch.exp(logk).item(), a.item()
    say(f"final: loss {losses[-1]:.3e} (from {losses[0]:.3e}) k {kf:.4f} a {af:.6f}")
    assert losses[-1] < 1e-7 * losses[0]
    assert abs(af - 1.08) < 1e-3
    assert abs(kf - 60.0) < 1.0
