"""Benchmark of the multiblob step on one MI355X.

Workload (default): the dense suspension -- periodic 128^3 MAC grid, h = 1,
36,669 thirteen-blob icosahedral particles (476,697 blobs) at volume
fraction 0.3 (effective radius 1.6 h), random sequential addition, uniformly
random orientations, Fext ~ N(0, 1) per particle, dt = 0.01, rho = eta = 1,
springs k = 100 on all 78 pairs.  Synthetic, seeded inputs resident in HBM
before the timed region.

One step = springs + binning + spreading + the FFT fluid solve with the
projection + interpolation and the position update + the momentum and
divergence reductions (everything mb_step runs).  `value` is the mixed
precision step rate; the float64 step rate on the same GPU is reported
beside it.  The dominant kernel's duration is measured live in the timed
region with HIP events around that kernel only, and set against the HBM
roofline with the kernel's algorithmic bytes.  The oracle (float64, its
OpenMP build on the host's cores) is timed on a bounded sample of the same
workload as the CPU baseline.

Also measured: the large suspension (256^3, phi = 0.4, 5,084,807 blobs),
100 steps in each precision from the same state, with the mixed result's
error against the float64 one (key "large"); the second-order (midpoint)
scheme's step rate on the same workload (key "midpoint"); the steady-Stokes measurements (hydrodynamic
radius against d, suspension viscosity) timed whole (key "stokes"); one loss
and gradient evaluation of the differentiation case, 64^3, 16 particles, 100
float64 steps through the adjoint kernels (key "diff"); and
(key "batch") the pair-mobility sweep, 512 boxes of edge
24/32/48/64 with two particles each, grouped by edge into four grids of equal
boxes and advanced by a graph-captured step of all four, against the same
boxes advanced one grid per box.

Prints one JSON line.  `--gpus N` with N > 1 exits: the step has a one-GPU
path only.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def algorithmic_bytes(L, M, P, prec, steady=False):
    """Bytes each kernel of one step must move at minimum (one read or write
    of every array it consumes or produces), per launch."""
    s = 4 if prec == "mixed" else 8
    recg = 16 if prec == "mixed" else 32      # geometry record (fractions, cell)
    rec = recg + 3 * s                        # + force record
    N = L ** 3
    field = 3 * N * s
    spec = 3 * L * L * (L // 2 + 1) * 2 * s
    ntiles = (L // 16 if L % 16 == 0 else L // 8) * (L // 8) ** 2  # 16x8x8 tiles
    return {
        "bin_count": 24 * M + 4 * M + 4 * M + 4 * M,  # q, previous order, tile, rank
        "scan_reduce": 4 * ntiles,
        "scan_apply": 12 * ntiles,
        "springs_scatter": 24 * M + 24 * P + 12 * M + rec * M,
        "spread": rec * M + field,
        "fft_x_fwd": (1 if steady else 2) * field + spec,
        "fft_xy_inv": spec + field,  # inverse y and x in one plane pass
        "fft_y_fwd": 2 * spec,
        "fft_z_spectral": 2 * spec,
        "fft_y_inv": 2 * spec,
        "fft_x_inv": spec + field,
        "interp_step": field + recg * M + 4 * M + 48 * M,
    }


def library_sources_sha256():
    """SHA-256 over the library's kernel and interface sources (the key under
    which measured HBM traffic is stored)."""
    import glob
    import hashlib
    src = sorted(glob.glob(os.path.join(ROOT, "paper_1407_5600_amd", "csrc", "*.hip")) +
                 glob.glob(os.path.join(ROOT, "paper_1407_5600_amd", "csrc", "*.h")) +
                 glob.glob(os.path.join(ROOT, "include", "*.h")))
    h = hashlib.sha256()
    for p in src:
        h.update(os.path.relpath(p, ROOT).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE scaled by the
    copy calibration) from the stored counter summary of the dense workload,
    or None when there is none or the library sources changed since."""
    path = os.path.join(ROOT, "profiles", "dense128_traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != library_sources_sha256():
        return None
    k = t.get("kernels", {}).get(kernel)
    return round(k["read_bytes"] + k["write_bytes"]) if k else None


def run_steps(torch, g, sp, q, v, Fe, n):
    # one call of n steps (steps after a call's first take their binning
    # from the previous step's interpolation), returning the diagnostics
    # (momentum, net force, max |Dv|) of the last step
    if n > 0:
        diag = torch.zeros(7, dtype=torch.float64, device=q.device)
        g.step(sp, q, v, Fe, n, diag_out=diag)


def bench_precision(torch, w, prec, steps, warmup, live_kernel=None):
    from paper_1407_5600_amd import Grid, Springs
    g = Grid(w.L, h=w.h, rho=w.rho, eta=w.eta, dt=w.dt, precision=prec, max_blobs=w.M)
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    q = torch.from_numpy(w.q.copy()).cuda()
    v = g.field()
    Fe = torch.from_numpy(w.Fext).cuda()
    run_steps(torch, g, sp, q, v, Fe, warmup)
    torch.cuda.synchronize()
    # calibration pass: every kernel timed (each launch records its own
    # start and end), to find the dominant one
    g.set_timing("all")
    ncal = 20
    run_steps(torch, g, sp, q, v, Fe, ncal)
    kt = g.kernel_times()
    g.set_timing(None)
    per_step = {k: ms / ncal for k, (ms, n) in kt.items()}
    avg = {k: ms / n for k, (ms, n) in kt.items()}
    dominant = live_kernel or max(per_step, key=per_step.get)
    # timed region of the headline: no events, one call of all the steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(torch, g, sp, q, v, Fe, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the same steps again with the dominant kernel's launches timed (on the
    # stream they run on), for its live duration
    g.set_timing([dominant])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    run_steps(torch, g, sp, q, v, Fe, steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    live = g.kernel_times()
    g.set_timing(None)
    ms, n = live[dominant]
    assert bool(torch.isfinite(v).all()), "non-finite velocity"
    return {
        "ms_per_step": (t1 - t0) * 1e3 / steps,
        "timed_pass_ms_per_step": (t3 - t2) * 1e3 / steps,
        "per_step_ms": per_step,
        "avg_launch_ms": avg,
        "dominant": dominant,
        "dominant_live_ms": ms / n,
        "dominant_launches": n,
    }


def bench_midpoint(torch, w, steps, warmup):
    """Step rate of the second-order (midpoint) scheme on the same workload."""
    from paper_1407_5600_amd import Grid, Springs
    out = {}
    for prec in ("mixed", "fp64"):
        g = Grid(w.L, h=w.h, rho=w.rho, eta=w.eta, dt=w.dt, precision=prec, max_blobs=w.M,
                 scheme="midpoint")
        sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
        q = torch.from_numpy(w.q.copy()).cuda()
        v = g.field()
        Fe = torch.from_numpy(w.Fext).cuda()
        run_steps(torch, g, sp, q, v, Fe, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_steps(torch, g, sp, q, v, Fe, steps)
        torch.cuda.synchronize()
        out[prec + "_steps_per_s"] = round(steps / (time.perf_counter() - t0), 2)
    return out


def bench_large(torch, steps):
    """The large suspension (256^3, phi = 0.4, 391,139 particles, 5,084,807
    blobs): `steps` steps from rest in each precision from the same state,
    timed, and the mixed result's error against the float64 one (norm-wise
    relative: displacements, final fluid velocity, last-step particle
    velocities)."""
    import numpy as np
    from paper_1407_5600_amd import Grid, Springs, inputs
    w = inputs.cached("large")
    out = {"workload": f"large suspension {w.L}^3 h=1, {w.P} particles x {w.nb} blobs "
                       f"({w.M} blobs), phi={w.extra.get('phi', '')}, dt={w.dt}, k={w.k}",
           "steps": steps}
    fin = {}
    for prec in ("mixed", "fp64"):
        g = Grid(w.L, h=w.h, rho=w.rho, eta=w.eta, dt=w.dt, precision=prec, max_blobs=w.M)
        sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
        Fe = torch.from_numpy(w.Fext).cuda()
        # one untimed step on a copy of the state (first binning)
        qw = torch.from_numpy(w.q.copy()).cuda()
        vw = g.field()
        g.step(sp, qw, vw, Fe, 1)
        del qw, vw
        q = torch.from_numpy(w.q.copy()).cuda()
        v = g.field()
        U0 = torch.zeros((w.P, 3), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(sp, q, v, Fe, steps, U0_out=U0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[prec + "_steps_per_s"] = round(steps / dt, 2)
        fin[prec] = {"dq": q.cpu().numpy() - w.q, "v": v.double().cpu().numpy(),
                     "U0": U0.cpu().numpy()}
        del g, sp, q, v, U0, Fe
        torch.cuda.empty_cache()

    def rel(a, b):
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    out["mixed_over_fp64"] = round(out["mixed_steps_per_s"] / out["fp64_steps_per_s"], 3)
    out["mixed_vs_fp64_rel_err"] = {k: rel(fin["mixed"][k], fin["fp64"][k])
                                    for k in ("dq", "v", "U0")}
    return out


def bench_stokes(torch, oracle_sample=True):
    """The steady-Stokes measurements at their default sizes, timed whole
    (input generation excluded), with box-steps/s; the oracle timed on a few
    steps of one such box."""
    from paper_1407_5600_amd import stokes
    rh = stokes.hydrodynamic_radius()
    vis = stokes.viscosity()
    out = {
        "hydrodynamic_radius": {
            "boxes": len(rh["d"]) * rh["orientations"], "L": rh["L"], "steps": rh["steps"],
            "seconds": round(rh["seconds"], 4),
            "box_steps_per_s": round(len(rh["d"]) * rh["orientations"] * rh["steps"]
                                     / rh["seconds"], 1),
            "R_H": {str(d["d"]): round(d["R_H"], 4) for d in rh["d"]}},
        "viscosity": {
            "boxes": len(vis["phi"]) * vis["configs"], "L": vis["L"], "steps": vis["steps"],
            "seconds": round(vis["seconds"], 4),
            "box_steps_per_s": round(len(vis["phi"]) * vis["configs"] * vis["steps"]
                                     / vis["seconds"], 1),
            "eta_rel": {str(p["phi"]): round(p["eta_rel"], 4) for p in vis["phi"]}},
    }
    if oracle_sample:
        import numpy as np
        import oracle
        from paper_1407_5600_amd import inputs
        setup = stokes.radius_setup((1.0,), rh["L"], 1)[0]
        pa, pb, r0 = inputs.pair_table(setup[1])
        prm = oracle.params(rh["L"], dt=rh["dt"], steady=True, zero_mean=True)
        n = 5
        t0 = time.perf_counter()
        oracle.step(prm, {"nb": 13, "pa": pa, "pb": pb, "r0": r0, "k": 100.0}, setup[2],
                    np.zeros((3, rh["L"], rh["L"], rh["L"])), setup[3], n)
        out["oracle_box_steps_per_s"] = round(n / (time.perf_counter() - t0), 2)
        out["oracle_sample"] = f"{n} float64 steps of one {rh['L']}^3 radius box, one thread"
    return out


def bench_diff(torch, reps=3, oracle_sample=True):
    """The differentiation case (64^3, 16 particles, 100 float64 steps of
    dt = 0.01, checkpoints every 10): the loss sum_p |U_p - V_p|^2 alone and
    with its gradients (624 blob-force components, stiffness, vertex radius)
    by the library's adjoint kernels through torch.autograd; median wall
    time of `reps` evaluations after one warm-up.  The oracle's reverse
    sweep is timed on a few steps of the same case (one thread)."""
    import numpy as np
    from paper_1407_5600_amd import Grid, inputs
    from paper_1407_5600_amd.autodiff import particle_means, place_template, trajectory
    w = inputs.diff()
    G = np.repeat(w.Fext / w.nb, w.nb, axis=0)
    unit = inputs.icosahedron_template(1.0)
    _, _, r0u = inputs.pair_table(unit)

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()

    g = Grid(w.L, h=w.h, rho=w.rho, eta=w.eta, dt=w.dt, max_blobs=w.M)
    cen, rot, V = dev(w.extra["centres"]), dev(w.extra["rotations"]), dev(w.extra["V"])
    unit_t, r0u_t = dev(unit), dev(np.asarray(r0u, dtype=float))

    def once(grad):
        a = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=grad)
        k = torch.tensor(float(w.k), dtype=torch.float64, device="cuda", requires_grad=grad)
        Gt = dev(G).requires_grad_(grad)
        q0 = place_template(cen, rot, unit_t, a)
        v0 = torch.zeros((3, w.L, w.L, w.L), dtype=torch.float64, device="cuda")
        u = trajectory(g, w.nb, w.pa, w.pb, q0, v0, Gt, k, a * r0u_t, w.steps, 10)
        loss = ((particle_means(u, w.nb) - V) ** 2).sum()
        if grad:
            loss.backward()
        torch.cuda.synchronize()

    out = {"workload": f"diff: {w.L}^3, {w.P} particles x {w.nb} blobs, {w.steps} steps of "
                       f"dt {w.dt}, checkpoints every 10, float64"}
    for key, grad in (("loss_seconds", False), ("loss_and_gradient_seconds", True)):
        once(grad)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            once(grad)
            ts.append(time.perf_counter() - t0)
        out[key] = round(sorted(ts)[len(ts) // 2], 4)
    if oracle_sample:
        import oracle
        prm = oracle.params(w.L, h=w.h, rho=w.rho, eta=w.eta, dt=w.dt)
        n = 5
        t0 = time.perf_counter()
        oracle.loss_grad(prm, w.springs(), w.q, np.zeros((3, w.L, w.L, w.L)), G,
                         w.extra["V"], n)
        sec = time.perf_counter() - t0
        out["oracle_loss_and_gradient_seconds_per_step"] = round(sec / n, 4)
        out["oracle_sample"] = (f"{n} float64 steps of the same case, loss and reverse sweep, "
                                f"one thread")
    return out


# Child process of the CPU baseline: times single float64 oracle steps of the
# cached workload with the OpenMP build (the library path and thread count
# come from the environment), until `budget` seconds or `max_steps` steps,
# at least `min_steps`; prints the step times as JSON.
_CPU_CHILD = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
from paper_1407_5600_amd import inputs
w = inputs.cached(sys.argv[2])
budget, min_steps, max_steps = float(sys.argv[3]), int(sys.argv[4]), int(sys.argv[5])
prm = oracle.params(w.L, h=w.h, rho=w.rho, eta=w.eta, dt=w.dt)
q, v = w.q.copy(), np.zeros((3, w.L, w.L, w.L))
times = []
t_start = time.perf_counter()
while len(times) < max_steps and (len(times) < min_steps or
                                   time.perf_counter() - t_start < budget):
    t0 = time.perf_counter()
    r = oracle.step(prm, w.springs(), q, v, w.Fext, 1)
    times.append(time.perf_counter() - t0)
    q, v = r["q"], r["v"]
print(json.dumps(times))
"""


def cpu_baseline(workload, budget_s=12.0, min_steps=3, max_steps=30):
    """The float64 oracle (plain C, its OpenMP build at -O3) timed on the
    host's cores: single steps of the same workload from rest, the median
    step time.  Threads: the CPUs this process may run on, capped by
    OMP_NUM_THREADS when the environment sets it."""
    import statistics
    import subprocess
    from oracle import build as obuild
    if not os.path.exists(obuild.LIB_OMP):
        obuild.build(openmp=True)
    ncpu = len(os.sched_getaffinity(0))
    threads = ncpu
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = max(1, min(ncpu, int(os.environ["OMP_NUM_THREADS"])))
    env = dict(os.environ, MBO_ORACLE_LIB=obuild.LIB_OMP, OMP_NUM_THREADS=str(threads),
               OMP_PROC_BIND="close")
    r = subprocess.run([sys.executable, "-c", _CPU_CHILD, ROOT, workload, str(budget_s),
                        str(min_steps), str(max_steps)], env=env, capture_output=True,
                       text=True, check=True)
    times = json.loads(r.stdout.strip().splitlines()[-1])
    med = statistics.median(times)
    return {"value": 1.0 / med, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(times)} single float64 steps of the same workload from rest, "
                      f"median step time; C oracle built -O3 -fopenmp, {threads} threads",
            "step_seconds": [round(t, 4) for t in times], "affinity_cpus": ncpu,
            "host_cpu": host_cpu()}


def host_cpu():
    """The host CPU as lscpu reports it (model name, sockets, cores per
    socket, threads per core), else /proc/cpuinfo's model name, or None."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    keys = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
            "CPU(s)", "CPU max MHz")
    got = {k: info[k] for k in keys if k in info}
    if got:
        return got
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return {"Model name": line.split(":", 1)[1].strip()}
    except OSError:
        pass
    return None


R_NOSLIP = 1.62  # no-slip radius of the d = h icosahedron (Table 2)


def bench_batch(torch, nbox, steps, sample=32):
    """Pair-mobility sweep: nbox boxes of edge 24/32/48/64 with two d = h
    icosahedra each (one random orientation per box) pulled towards each
    other along their line of centres, steady Stokes with dt = 0.05 (the
    Stokes-limit set-up of the paper's pair measurements), mixed precision,
    grouped by edge into four batch grids stepped by one graph-captured step
    per time step; against the same boxes stepped one grid per box (a
    sample of them, eager).  Each box's relative velocity at the end gives
    the pair mobility, compared with the two-sphere function of eq. ab for
    separations beyond 2.5 R_s."""
    import numpy as np
    from paper_1407_5600_amd import Grid, Springs, inputs, stokes
    from paper_1407_5600_amd.binding import step_graph
    tmpl = inputs.icosahedron_template(inputs.CIRCUMRADIUS_OVER_EDGE * 1.0)
    boxes = inputs.pair_sweep(nbox=nbox, template=tmpl, rotate=True)
    pa, pb, r0 = inputs.pair_table(tmpl)
    sp = Springs(len(tmpl), pa, pb, r0, 100.0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    kw = dict(precision="mixed", mode="steady", zero_mean=True, dt=0.05)
    grids, qs, vs, fs, order = [], [], [], [], []
    for L in sorted({b["L"] for b in boxes}):
        idx = [i for i, b in enumerate(boxes) if b["L"] == L]
        g = Grid(L, max_blobs=26 * len(idx), nbox=len(idx), **kw)
        grids.append(g)
        qs.append(dev(np.concatenate([boxes[i]["q"] for i in idx])))
        vs.append(g.field())
        fs.append(dev(np.concatenate([boxes[i]["Fext"] for i in idx])))
        order.append(idx)
    cells = sum(b["L"] ** 3 for b in boxes)
    step_graph(grids, [sp] * len(grids), qs, vs, fs, None, 2)  # warm-up, capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_graph(grids, [sp] * len(grids), qs, vs, fs, None, steps)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for g, q, v, F in zip(grids, qs, vs, fs):
        g.step(sp, q, v, F, steps)
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / steps
    # relative velocity (U1 - U2).x per box after the run (one more step),
    # and the blob positions it is taken at
    rel_u = np.zeros(nbox)
    q_at = np.zeros((nbox, 2 * len(tmpl), 3))
    for g, q, v, F, idx in zip(grids, qs, vs, fs, order):
        q_at[idx] = q.view(len(idx), 2 * len(tmpl), 3).cpu().numpy()
        U0 = torch.empty((2 * len(idx), 3), dtype=torch.float64, device="cuda")
        g.step(sp, q, v, F, 1, U0_out=U0)
        rel_u[idx] = (U0[0::2, 0] - U0[1::2, 0]).cpu().numpy()
    # pair part of the mobility per box against eq. ab (untimed: each
    # particle alone in a box of its own at the same blob positions)
    F_x = np.array([b["Fext"][:, 0] for b in boxes])
    pi = stokes.pair_sweep_interaction(torch, q_at, [b["L"] for b in boxes], F_x, rel_u,
                                       tmpl, R_s=R_NOSLIP, dt=0.05)
    far = pi["r"] > 2.5 * R_NOSLIP
    err = np.abs(pi["interaction"] - pi["sphere"]) / pi["sphere"]
    stat = lambda m: ({"boxes": int(m.sum()), "rel_err_mean": round(float(err[m].mean()), 4),
                       "rel_err_max": round(float(err[m].max()), 4)} if m.any() else
                      {"boxes": 0})
    eq_ab = {"r_min": round(2.5 * R_NOSLIP, 3), "all": stat(far),
             "by_L": {int(L): stat(far & (pi["L"] == L)) for L in sorted(set(pi["L"]))},
             "r_below_4.5": stat(far & (pi["r"] < 4.5)), "r_from_4.5": stat(pi["r"] >= 4.5)}
    # one grid per box, a sample of the boxes
    samp = boxes[:sample]
    sg = [Grid(b["L"], max_blobs=26, **kw) for b in samp]
    sq = [dev(b["q"]) for b in samp]
    sv = [g.field() for g in sg]
    sf = [dev(b["Fext"]) for b in samp]
    for g, q, v, F in zip(sg, sq, sv, sf):
        g.step(sp, q, v, F, 2)
    torch.cuda.synchronize()
    ns = max(5, steps // 10)
    t0 = time.perf_counter()
    for _ in range(ns):
        for g, q, v, F in zip(sg, sq, sv, sf):
            g.step(sp, q, v, F, 1)
    torch.cuda.synchronize()
    per_box_step = (time.perf_counter() - t0) / (ns * len(samp))
    sample_cells = sum(b["L"] ** 3 for b in samp)
    return {"workload": f"pair sweep: {nbox} boxes of edge 24/32/48/64 (seeded), 2 d = h "
                        f"icosahedra each at x-separation U[2,6], forces +-(1,0,0), steady "
                        f"Stokes, dt 0.05, mixed",
            "boxes": nbox, "cells": int(cells), "steps": steps,
            "batched_graph_ms_per_step": round(t_batch * 1e3, 4),
            "box_steps_per_s": round(nbox / t_batch, 1),
            "batched_eager_ms_per_step": round(t_eager * 1e3, 4),
            "one_grid_per_box_ms_per_box_step": round(per_box_step * 1e3, 4),
            "one_grid_per_box_sample": f"{len(samp)} boxes ({sample_cells} cells), eager",
            "speedup_vs_one_grid_per_box": round(per_box_step * nbox / t_batch, 2),
            "relative_velocity_x": {"mean": float(rel_u.mean()), "min": float(rel_u.min()),
                                    "max": float(rel_u.max())},
            "pair_mobility_vs_eq_ab": eq_ab}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="dense", choices=["dense", "large", "single"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU time budget of the oracle baseline (at least 3 steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None,
                    help="run one precision (profiling)")
    ap.add_argument("--batch-boxes", type=int, default=512,
                    help="boxes of the batched pair-sweep measurement (0: skip it)")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--large-steps", type=int, default=100,
                    help="steps per precision of the 256^3 phi = 0.4 suspension (0: skip it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the midpoint-scheme and steady-Stokes measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device-to-device copy of 2^28 bytes, the "
                         "reference for scaling FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the step runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1407_5600_amd import inputs
    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)  # elementwise copy: reads and writes 256 MiB
        torch.cuda.synchronize()
        del src, dst
    w = inputs.cached(args.workload)
    res = {}
    for prec in (["mixed", "fp64"] if args.only is None else [args.only]):
        print(f"[bench] {prec} {args.workload} L={w.L} M={w.M}", file=sys.stderr, flush=True)
        res[prec] = bench_precision(torch, w, prec, args.steps, args.warmup)
        print(f"[bench] {prec}: {res[prec]['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)

    head = res.get("mixed") or res["fp64"]
    head_prec = "mixed" if "mixed" in res else "fp64"
    ab = algorithmic_bytes(w.L, w.M, w.P, head_prec)
    dom = head["dominant"]
    dom_bytes = ab.get(dom)
    achieved = dom_bytes / (head["dominant_live_ms"] * 1e-3) / 1e9 if dom_bytes else None
    kernels = {}
    for k, ms in head["per_step_ms"].items():
        b = ab.get(k)
        kernels[k] = {"ms_per_step": round(ms, 5),
                      "avg_launch_ms": round(head["avg_launch_ms"][k], 5),
                      "alg_GBps": round(b / (head["avg_launch_ms"][k] * 1e-3) / 1e9, 1) if b else None}
    t_s = head["avg_launch_ms"].get("spread", 0.0)
    t_j = head["avg_launch_ms"].get("interp_step", 0.0)
    out = {
        "metric": "steps/s at 128^3 phi=0.3 (FP32 mixed vs FP64); blob S+J/s; HBM GB/s",
        "value": round(1e3 / head["ms_per_step"], 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-mixed" if head_prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} suspension {w.L}^3 h=1, {w.P} particles x {w.nb} blobs"
                               f" ({w.M} blobs), phi={w.extra.get('phi', '')}, dt={w.dt}, k={w.k}",
                   "L": w.L, "particles": w.P, "blobs": w.M, "precision": head_prec},
        "fp64_steps_per_s": round(1e3 / res["fp64"]["ms_per_step"], 2) if "fp64" in res else None,
        "mixed_over_fp64": (round(res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"], 3)
                            if "fp64" in res and "mixed" in res else None),
        "blob_SJ_per_s": round(w.M / ((t_s + t_j) * 1e-3), 1) if t_s + t_j > 0 else None,
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": (measured_traffic(dom)
                                 if args.workload == "dense" and head_prec == "mixed" else None),
                     "alg_bytes_per_launch": dom_bytes,
                     "live_avg_launch_ms": round(head["dominant_live_ms"], 5),
                     "live_launches": head["dominant_launches"],
                     "live_pass_ms_per_step": round(head["timed_pass_ms_per_step"], 5)},
    }
    if "fp64" in res:
        out["kernels_fp64"] = {k: round(ms, 5) for k, ms in res["fp64"]["per_step_ms"].items()}
    if args.only is None and args.workload == "dense" and args.large_steps > 0:
        print(f"[bench] large suspension ({args.large_steps} steps per precision)",
              file=sys.stderr, flush=True)
        out["large"] = bench_large(torch, args.large_steps)
    if args.only is None and args.workload == "dense" and not args.no_extras:
        print("[bench] midpoint scheme", file=sys.stderr, flush=True)
        out["midpoint"] = bench_midpoint(torch, w, max(10, args.steps // 4), 5)
        print("[bench] steady-Stokes measurements", file=sys.stderr, flush=True)
        out["stokes"] = bench_stokes(torch, oracle_sample=not args.no_cpu_baseline)
        print("[bench] differentiation case", file=sys.stderr, flush=True)
        out["diff"] = bench_diff(torch, oracle_sample=not args.no_cpu_baseline)
    if args.batch_boxes > 0 and args.only is None:
        print(f"[bench] batched pair sweep ({args.batch_boxes} boxes)", file=sys.stderr,
              flush=True)
        out["batch"] = bench_batch(torch, args.batch_boxes, args.batch_steps)
    if not args.no_cpu_baseline and args.workload != "large":
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
