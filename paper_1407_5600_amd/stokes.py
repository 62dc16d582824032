"""Stokes-limit measurements with the multiblob step (steady Stokes mode).

The steady mode of the solve (the fluid momentum relaxes at once, the
Sc -> infinity limit the paper uses for its hydrodynamic measurements) drives
the paper's own experiments on synthetic configurations:

* hydrodynamic radius against the icosahedron vertex distance d: a particle
  pulled by a small force relaxes its springs until it translates rigidly;
  R_H(L) = F / (6 pi eta U_0) in the periodic box, extrapolated to the
  infinite box with eq. rhinf (Sec. Hydrodynamic radius, Table 2);
* pair mobilities: two particles pulled with opposite forces along or across
  their line of centres; the velocity of particle 1 gives A~ and B~ of Sec.
  Mutual friction and lubrication forces, whose interaction part is compared
  with the two-sphere functions A(r), B(r) of eq. ab (four reflections);
* suspension viscosity: a periodic force density f0 sin(k_j y) x on the
  fluid over hard-sphere Monte Carlo configurations, eta = f0 / (k_j^2 v_x)
  from the amplitude v_x of the x-velocity profile after the springs have
  adapted to the strain (Sec. Stresslet and Viscosity), compared with
  Einstein's 1 + 5/2 phi and Batchelor's + 6.2 phi^2.

Every box of a measurement is a box of a batch grid, so one launch per
kernel advances all orientations, separations or configurations together.
Velocities are read from the displacement of the particle centres over the
averaging window (the mean blob velocity of each step moves the centre by
dt U_0 exactly).
"""
import math
import time

import numpy as np

from . import inputs
from .binding import Grid, Springs, step_graph

HASIMOTO = 2.837  # eq. rhinf (printed as 2.84)


def _template(d):
    """Filled icosahedron of vertex distance d (circumradius 0.95106 d)."""
    return inputs.icosahedron_template(inputs.CIRCUMRADIUS_OVER_EDGE * d)


def _springs(tmpl, k):
    pa, pb, r0 = inputs.pair_table(tmpl)
    return Springs(tmpl.shape[0], pa, pb, r0, k)


def _particle(d, k):
    tmpl = _template(d)
    return tmpl, _springs(tmpl, k)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _centres(torch, q, nb):
    return q.view(-1, nb, 3).mean(1)


def _run(grids, springs, qs, vs, fs, nsteps):
    if nsteps > 0:
        step_graph(grids, springs, qs, vs, fs, None, nsteps)


def inf_box_radius(RL, L):
    """R_H(infinity) from the periodic-box value (eq. rhinf)."""
    return RL / (1.0 + HASIMOTO * RL / L)


def radius_setup(d_values, L, orientations, force=0.01, seed=7):
    """Inputs of the hydrodynamic-radius measurement: per d, the template,
    the blobs of `orientations` particles (random rotation, centre at L/2
    plus a random offset within a cell, one per box) and their pulling
    forces (force along x)."""
    rng = np.random.default_rng(seed)
    out = []
    for d in d_values:
        tmpl = _template(d)
        R = inputs.random_rotations(rng, orientations)
        c = L / 2.0 + rng.uniform(0.0, 1.0, size=(orientations, 3))
        F = np.zeros((orientations, 3))
        F[:, 0] = force
        out.append((d, tmpl, inputs.place_particles(c, tmpl, R), F))
    return out


def hydrodynamic_radius(d_values=(1.0, 1.5, 2.0, 2.5, 3.0), L=32, orientations=8,
                        force=0.01, dt=0.05, relax=2000, average=400, k=100.0,
                        eta=1.0, precision="fp64", seed=7):
    """R_H(L) and R_H(infinity) of the filled icosahedron for each vertex
    distance d, averaged over random orientations and positions within the
    cell.  One batch grid per d (one particle per box), all advanced by one
    graph-captured step."""
    import torch
    grids, sprs, qs, vs, fs = [], [], [], [], []
    for d, tmpl, q, F in radius_setup(d_values, L, orientations, force, seed):
        sp = _springs(tmpl, k)
        g = Grid(L, eta=eta, dt=dt, precision=precision, mode="steady", zero_mean=True,
                 max_blobs=q.shape[0], nbox=orientations)
        grids.append(g), sprs.append(sp), qs.append(_dev(torch, q))
        vs.append(g.field()), fs.append(_dev(torch, F))
    t0 = time.perf_counter()
    _run(grids, sprs, qs, vs, fs, relax)
    X0 = [_centres(torch, q, sp.nb).clone() for q, sp in zip(qs, sprs)]
    _run(grids, sprs, qs, vs, fs, average)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = {"L": L, "orientations": orientations, "steps": relax + average, "dt": dt,
           "force": force, "precision": precision, "seconds": elapsed, "d": []}
    for d, q, sp, x0 in zip(d_values, qs, sprs, X0):
        U = ((_centres(torch, q, sp.nb) - x0) / (average * dt)).cpu().numpy()
        RL = force / (6.0 * math.pi * eta * U[:, 0])
        Rinf = inf_box_radius(RL, L)
        out["d"].append({"d": d, "R_H_L": float(RL.mean()), "R_H": float(Rinf.mean()),
                         "R_H_min": float(Rinf.min()), "R_H_max": float(Rinf.max()),
                         "transverse_over_parallel": float(np.abs(U[:, 1:]).max()
                                                           / np.abs(U[:, 0]).min())})
    return out


def sphere_A(r, R):
    """Normal pair function A(r) of eq. ab with the coefficient of the 1/r
    term read as 3/2 (the printed 3/3 is garbled: 3/2 is the Oseen term
    along the line of centres)."""
    x = R / r
    return 1.0 - 1.5 * x + x ** 3 - 3.75 * x ** 4


def sphere_B(r, R):
    """Tangential pair function B(r) of eq. ab."""
    x = R / r
    return 1.0 - 0.75 * x - 0.5 * x ** 3


def pair_mobility(separations=(4.0, 5.0, 6.0, 8.0, 10.0, 12.0), d=1.0, L=64,
                  direction="normal", force=0.01, dt=0.05, relax=1000, average=200,
                  k=100.0, eta=1.0, precision="fp64", seed=9):
    """Two particles at separation r along x pulled with F1 = -F2 = F n
    (n = x: 'normal', the lubrication set-up; n = y: 'tangential'), one box
    per separation, and beside each pair a box holding particle 1 alone at
    the same place and orientation.  Returns A~ = 6 pi eta U1.n / F per
    separation (B~ for the tangential direction) and the interaction part
        mu12~ = 6 pi eta (U_alone - U1).n / F + 2.837 / L,
    whose two-sphere value is (1 - A(r)) / R_s (or (1 - B(r)) / R_s).  The
    periodic images shift the self and the pair mobility by the same
    -2.837 / (6 pi eta L) (eq. rhinf), restored by the last term; the
    matched lone particle cancels the dependence of the self term on the
    position within the cell.  The remainder is O(r^2 / L^3)."""
    import torch
    rng = np.random.default_rng(seed)
    tmpl, sp = _particle(d, k)
    n = np.array([1.0, 0.0, 0.0]) if direction == "normal" else np.array([0.0, 1.0, 0.0])
    nsep = len(separations)
    R = inputs.random_rotations(rng, nsep)
    cen, Fp = [], []
    for r in separations:
        mid = L / 2.0 + rng.uniform(0.0, 1.0, size=3)
        cen += [mid - [r / 2.0, 0.0, 0.0], mid + [r / 2.0, 0.0, 0.0]]
        Fp += [force * n, -force * n]
    cen = np.array(cen)
    q2 = inputs.place_particles(cen, tmpl, np.repeat(R, 2, 0))
    g2 = Grid(L, eta=eta, dt=dt, precision=precision, mode="steady", zero_mean=True,
              max_blobs=q2.shape[0], nbox=nsep)
    q1 = inputs.place_particles(cen[0::2], tmpl, R)
    g1 = Grid(L, eta=eta, dt=dt, precision=precision, mode="steady", zero_mean=True,
              max_blobs=q1.shape[0], nbox=nsep)
    grids = [g2, g1]
    qs = [_dev(torch, q2), _dev(torch, q1)]
    vs = [g2.field(), g1.field()]
    fs = [_dev(torch, np.array(Fp)), _dev(torch, np.tile(force * n, (nsep, 1)))]
    t0 = time.perf_counter()
    _run(grids, [sp, sp], qs, vs, fs, relax)
    X0 = [_centres(torch, q, sp.nb).clone() for q in qs]
    _run(grids, [sp, sp], qs, vs, fs, average)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    U2 = ((_centres(torch, qs[0], sp.nb) - X0[0]) / (average * dt)).cpu().numpy()
    U1 = ((_centres(torch, qs[1], sp.nb) - X0[1]) / (average * dt)).cpu().numpy()
    c = 6.0 * math.pi * eta / force
    At = c * (U2[0::2] @ n)
    alone = c * (U1 @ n)
    return {"direction": direction, "d": d, "L": L, "separations": list(separations),
            "A_tilde": At.tolist(),
            "R_H": float(np.mean(inf_box_radius(1.0 / alone, L))),
            "interaction": (alone - At + HASIMOTO / L).tolist(), "precision": precision,
            "steps": relax + average, "seconds": elapsed}


def pair_interaction_sphere(r, R, direction="normal"):
    """(1 - A(r)) / R or (1 - B(r)) / R: the pair part of 6 pi eta U1 / F for
    two spheres of radius R (eq. ab)."""
    r = np.asarray(r, dtype=np.float64)
    f = sphere_A if direction == "normal" else sphere_B
    return (1.0 - f(r, R)) / R


def _lone_velocities(torch, q, L_box, F_x, tmpl, k, precision, eta=1.0, dt=0.01):
    """x-velocity of each particle of each pair box when alone in a box of
    the same edge, with the same blob positions (q: (nbox, 2 nb, 3)) and the
    same force (F_x: (nbox, 2)); steady Stokes, zero mean, one step from
    those positions: (nbox, 2) array."""
    sp = _springs(tmpl, k)
    nb = tmpl.shape[0]
    out = np.zeros((len(L_box), 2))
    for L in sorted(set(int(x) for x in L_box)):
        idx = [i for i, x in enumerate(L_box) if int(x) == L]
        ql = np.concatenate([q[i] for i in idx])  # particle 1, particle 2 of each box
        F = np.zeros((2 * len(idx), 3))
        F[:, 0] = np.asarray(F_x)[idx].reshape(-1)
        g = Grid(L, eta=eta, dt=dt, precision=precision, mode="steady", zero_mean=True,
                 max_blobs=ql.shape[0], nbox=2 * len(idx))
        U0 = torch.empty((2 * len(idx), 3), dtype=torch.float64, device="cuda")
        g.step(sp, _dev(torch, ql), g.field(), _dev(torch, F), 1, U0_out=U0)
        out[idx] = U0[:, 0].view(-1, 2).cpu().numpy()
        g.close()
    return out


def pair_sweep_interaction(torch, q, L_box, F_x, U_rel, tmpl, k=100.0, R_s=1.62,
                           precision="mixed", eta=1.0, dt=0.01):
    """Pair part of the mobility of two particles pulled apart along their
    line of centres (x), from the relative velocity U_rel = (U1 - U2).x of
    each pair box at blob positions q (nbox, 2 nb, 3) (steady Stokes, zero
    mean, forces F_x (nbox, 2) = (F, -F)), against eq. ab.  With particle j
    alone at the same blob positions (x-velocity U_ja, same force), the pair
    mobility along x in the periodic box is
    mu12(L) = [(U_1a - U_2a) - U_rel] / (2F), which cancels the dependence
    of the self terms on the place within the cell; the image shift
    -2.837 / (6 pi eta L) of eq. rhinf, common to self and pair terms, is
    added back:
        6 pi eta mu12 = 6 pi eta [(U_1a - U_2a) - U_rel] / (2F) + 2.837 / L,
    to be compared with (1 - A(r)) / R_s for two spheres of radius R_s at
    the centre distance r (remainder O(r^2 / L^3)).  Returns per box r, L,
    the measured and the two-sphere values."""
    q = np.asarray(q, dtype=np.float64)
    nb = tmpl.shape[0]
    Ua = _lone_velocities(torch, q, L_box, F_x, tmpl, k, precision, eta, dt)
    F = np.abs(np.asarray(F_x)[:, 0])
    L = np.asarray(L_box, dtype=np.float64)
    c1, c2 = q[:, :nb].mean(1), q[:, nb:].mean(1)
    d = c2 - c1
    d -= L[:, None] * np.round(d / L[:, None])  # minimum image
    r = np.linalg.norm(d, axis=1)
    meas = 6.0 * math.pi * eta * ((Ua[:, 0] - Ua[:, 1]) - np.asarray(U_rel)) / (2.0 * F) \
        + HASIMOTO / L
    return {"r": r, "L": L, "interaction": meas,
            "sphere": pair_interaction_sphere(r, R_s, "normal")}


def pair_sweep_measure(torch, boxes, tmpl, steps=1000, k=100.0, R_s=1.62,
                       precision="mixed", eta=1.0, dt=0.05):
    """The sweep boxes (inputs.pair_sweep) as batch grids by edge, steady
    Stokes with zero mean, advanced `steps` steps by one graph-captured
    step each; then the relative velocity of each box's pair and its pair
    part against eq. ab (pair_sweep_interaction)."""
    sp = _springs(tmpl, k)
    nb = tmpl.shape[0]
    grids, qs, vs, fs, order = [], [], [], [], []
    for L in sorted({b["L"] for b in boxes}):
        idx = [i for i, b in enumerate(boxes) if b["L"] == L]
        g = Grid(L, eta=eta, dt=dt, precision=precision, mode="steady", zero_mean=True,
                 max_blobs=2 * nb * len(idx), nbox=len(idx))
        grids.append(g), order.append(idx), vs.append(g.field())
        qs.append(_dev(torch, np.concatenate([boxes[i]["q"] for i in idx])))
        fs.append(_dev(torch, np.concatenate([boxes[i]["Fext"] for i in idx])))
    _run(grids, [sp] * len(grids), qs, vs, fs, steps)
    rel = np.zeros(len(boxes))
    q_at = np.zeros((len(boxes), 2 * nb, 3))
    for g, q, v, F, idx in zip(grids, qs, vs, fs, order):
        q_at[idx] = q.view(len(idx), 2 * nb, 3).cpu().numpy()
        U0 = torch.empty((2 * len(idx), 3), dtype=torch.float64, device="cuda")
        g.step(sp, q, v, F, 1, U0_out=U0)
        rel[idx] = (U0[0::2, 0] - U0[1::2, 0]).cpu().numpy()
    F_x = np.array([b["Fext"][:, 0] for b in boxes])
    return pair_sweep_interaction(torch, q_at, [b["L"] for b in boxes], F_x, rel, tmpl, k,
                                  R_s, precision, eta, dt)


def shear_force_field(L, f0, j=1, h=1.0, nbox=1):
    """Force density f0 sin(k_j y) x on the staggered grid, k_j = 2 pi j /
    (L h): the x component lives on the x faces, whose y coordinate is the
    row index times h.  Shape (3, L, L, L) or (nbox, 3, L, L, L)."""
    y = np.arange(L) * h
    f = np.zeros((3, L, L, L))
    f[0] = f0 * np.sin(2.0 * math.pi * j * y / (L * h))[None, :, None]
    return f if nbox == 1 else np.broadcast_to(f, (nbox,) + f.shape).copy()


def profile_amplitude(vx, L, j=1, h=1.0):
    """Amplitude of the sin(k_j y) component of the x velocity, per box
    (vx: (..., L, L, L) torch tensor): (2 / N) sum v_x sin(k_j y)."""
    import torch
    y = torch.arange(L, dtype=torch.float64, device=vx.device) * h
    s = torch.sin(2.0 * math.pi * j * y / (L * h)).view(L, 1)
    return (vx.double() * s).sum(dim=(-1, -2, -3)) * (2.0 / L ** 3)


def einstein_batchelor(phi):
    """eta / eta0 = 1 + 5/2 phi + 6.2 phi^2 (Sec. Stresslet and Viscosity)."""
    phi = np.asarray(phi, dtype=np.float64)
    return 1.0 + 2.5 * phi + 6.2 * phi ** 2


def viscosity(phi_values=(0.05, 0.1, 0.15, 0.2), d=1.0, L=32, configs=16, R_HS=1.62,
              j=1, f0=1e-5, dt=0.02, relax=1500, average=100, k=100.0, eta=1.0,
              precision="fp64", mc_sweeps=20, seed=11):
    """Relative viscosity eta(phi) / eta0 of a suspension of d-icosahedra at
    hard-sphere radius R_HS: per phi, `configs` independent hard-sphere
    Monte Carlo configurations (one box each of one batch grid, random
    orientations), forced by f0 sin(k_j y) x on the fluid; after `relax`
    steps the amplitude of the x-velocity profile is averaged over
    `average` steps and set against the particle-free amplitude
    f0 / (eta lambda_j), lambda_j = (4 / h^2) sin^2(pi j / L) (the discrete
    symbol of -Laplacian, whose continuum limit k_j^2 the paper's formula
    uses)."""
    import torch
    rng = np.random.default_rng(seed)
    tmpl, sp = _particle(d, k)
    lam = 4.0 * math.sin(math.pi * j / L) ** 2
    A0 = f0 / (eta * lam)
    out = {"d": d, "L": L, "configs": configs, "R_HS": R_HS, "j": j, "f0": f0, "dt": dt,
           "steps": relax + average, "precision": precision, "phi": [], "seconds": 0.0}
    for phi in phi_values:
        n = inputs.particles_for_fraction(L, phi, R_HS)
        cs = [inputs.hard_sphere_centres(rng, float(L), n, R_HS, sweeps=mc_sweeps)
              for _ in range(configs)]
        Rs = inputs.random_rotations(rng, n * configs)
        q = inputs.place_particles(np.concatenate(cs), tmpl, Rs)
        g = Grid(L, eta=eta, dt=dt, precision=precision, mode="steady", zero_mean=True,
                 max_blobs=q.shape[0], nbox=configs)
        qd = _dev(torch, q)
        v = g.field()
        ff = torch.from_numpy(shear_force_field(L, f0, j, nbox=configs)).to(
            device=v.device, dtype=v.dtype).reshape(g.field_shape)
        t0 = time.perf_counter()
        g.step_forced(sp, qd, v, ff, nsteps=relax)
        amp = torch.zeros(configs, dtype=torch.float64, device=v.device)
        vv = v.view(configs, 3, L, L, L)
        for _ in range(average):
            g.step_forced(sp, qd, v, ff, nsteps=1)
            amp += profile_amplitude(vv[:, 0], L, j)
        amp = (amp / average).cpu().numpy()
        out["seconds"] += time.perf_counter() - t0
        rel = A0 / amp
        out["phi"].append({"phi": phi, "particles": n, "eta_rel": float(rel.mean()),
                           "eta_rel_min": float(rel.min()), "eta_rel_max": float(rel.max()),
                           "einstein_batchelor": float(einstein_batchelor(phi))})
    return out
