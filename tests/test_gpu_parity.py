"""GPU parity: every call of the HIP library against the oracle on the same
seeded inputs.  Tolerances are norm-wise relative per output array,
||x - x_ref||_2 / ||x_ref||_2: 1e-12 for the float64 path and 1e-5 for the
mixed path (float32 fields), the targets the method's precision variants
are held to; element-wise bounds are checked against the array maximum."""
import math
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
    import paper_1407_5600_amd  # noqa: F401  (loads the library, fails loudly)
    return torch


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def check(name, got, ref, prec, floor=0.0):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    r = np.linalg.norm((got - ref).ravel()) / max(np.linalg.norm(ref.ravel()), floor, 1e-300)
    tol = TOL[prec]
    say(f"{name}: rel err {r:.3e} (tol {tol:.0e})")
    assert r <= tol, f"{name}: relative error {r:.3e} > {tol:.0e}"
    scale = max(np.max(np.abs(ref)), 1e-300)
    assert np.max(np.abs(got - ref)) <= 10 * tol * max(scale, floor)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def grid(L, prec, max_blobs=0, **kw):
    from paper_1407_5600_amd import Grid
    return Grid(L, precision=prec, max_blobs=max_blobs, **kw)


def blobs(seed, M, L, mode):
    rng = np.random.default_rng(seed)
    q = rng.uniform(0, L, size=(M, 3))
    if mode == "seam":
        q[: M // 2] = rng.choice([0.0, L - 1e-9, 1e-12, L / 2.0], size=(M // 2, 3)) + \
            rng.uniform(-0.6, 0.6, size=(M // 2, 3))
    elif mode == "unwrapped":
        q += rng.integers(-40, 40, size=(M, 3)) * L
    elif mode == "one_cell":
        q = 5.0 + rng.uniform(0.0, 1.0, size=(M, 3))
    elif mode == "ties":
        # integer and half-integer coordinates: the offset t of eq. delta's
        # node sets is exactly +-1/2 on the cell-centred axes or on the
        # component's own (half-cell shifted) axis, where the rounding of the
        # nearest node can go either way; at the seam (0, L/2, L) and
        # unwrapped far from the box
        base = rng.integers(0, L + 1, size=(M, 3)).astype(np.float64)
        base[: M // 4] = rng.choice([0.0, float(L // 2), float(L)], size=(M // 4, 3))
        q = base + rng.choice([0.0, 0.5], size=(M, 3))
        q[M // 2:] += rng.integers(-40, 40, size=(M - M // 2, 3)) * L
        q[::7, 1] = rng.uniform(0, L, size=q[::7, 1].shape)  # ties on two axes only
    return q


SIZES = [8, 16, 24, 32, 48, 64]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("L", SIZES)
@pytest.mark.parametrize("mode", ["uniform", "seam", "unwrapped", "one_cell", "ties"])
def test_spread(torch_cuda, prec, L, mode):
    torch = torch_cuda
    say("spread", prec, L, mode)
    M = 700
    q = blobs(L * 7 + len(mode), M, L, mode)
    F = np.random.default_rng(L).standard_normal((M, 3))
    g = grid(L, prec, M)
    f = g.spread(dev(torch, q), dev(torch, F))
    torch.cuda.synchronize()
    ref = oracle.spread(oracle.params(L), q, F)
    check(f"spread {prec} L={L} {mode}", f.double().cpu().numpy(), ref, prec)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_spread_h_and_empty(torch_cuda, prec):
    torch = torch_cuda
    say("spread h/empty", prec)
    L, h = 32, 0.7
    q = blobs(3, 400, L * h, "uniform")
    F = np.random.default_rng(4).standard_normal((400, 3))
    g = grid(L, prec, 400, h=h)
    f = g.spread(dev(torch, q), dev(torch, F))
    ref = oracle.spread(oracle.params(L, h=h), q, F)
    check(f"spread h={h}", f.double().cpu().numpy(), ref, prec)
    z = g.spread(dev(torch, np.zeros((0, 3))), dev(torch, np.zeros((0, 3))))
    torch.cuda.synchronize()
    assert float(z.abs().max()) == 0.0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("L", SIZES)
@pytest.mark.parametrize("mode", ["uniform", "seam", "unwrapped", "one_cell", "ties"])
def test_interpolate(torch_cuda, prec, L, mode):
    torch = torch_cuda
    say("interp", prec, L, mode)
    M = 700
    q = blobs(L * 11 + len(mode), M, L, mode)
    v = np.random.default_rng(L + 1).standard_normal((3, L, L, L))
    g = grid(L, prec, M)
    vt = torch.from_numpy(v).to(g.field_dtype).cuda()
    u = g.interpolate(dev(torch, q), vt)
    torch.cuda.synchronize()
    vin = vt.double().cpu().numpy()  # the field as the GPU sees it
    ref = oracle.interpolate(oracle.params(L), q, vin)
    check(f"interp {prec} L={L} {mode}", u.cpu().numpy(), ref, prec)


def test_spring_forces(torch_cuda):
    torch = torch_cuda
    from paper_1407_5600_amd import Springs, spring_forces
    say("springs")
    w = inputs.random_suspension(21, 24, 30)
    rng = np.random.default_rng(0)
    q = w.q + 0.03 * rng.standard_normal(w.q.shape)
    sp = Springs(13, w.pa, w.pb, w.r0, w.k)
    F = spring_forces(sp, dev(torch, q), dev(torch, w.Fext))
    torch.cuda.synchronize()
    ref = oracle.spring_forces(w.P, 13, w.pa, w.pb, w.r0, w.k, q, w.Fext)
    check("springs", F.cpu().numpy(), ref, "fp64")
    F0 = spring_forces(sp, dev(torch, q), None)
    ref0 = oracle.spring_forces(w.P, 13, w.pa, w.pb, w.r0, w.k, q, None)
    check("springs no Fext", F0.cpu().numpy(), ref0, "fp64")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("L", SIZES + [96])
@pytest.mark.parametrize("mode", ["unsteady", "unsteady0", "steady", "ideal"])
def test_fluid_solve(torch_cuda, prec, L, mode):
    torch = torch_cuda
    say("solve", prec, L, mode)
    rng = np.random.default_rng(L + len(mode))
    v = rng.standard_normal((3, L, L, L))
    f = rng.standard_normal((3, L, L, L)) + 0.3
    kw = dict(rho=1.3, eta=0.7, dt=0.05)
    if mode == "unsteady0":
        kw["zero_mean"] = True
    if mode == "steady":
        kw.update(mode="steady", zero_mean=True)
    if mode == "ideal":
        kw["eta"] = 0.0
    g = grid(L, prec, 0, **kw)
    vt = torch.from_numpy(v).to(g.field_dtype).cuda()
    ft = torch.from_numpy(f).to(g.field_dtype).cuda()
    out = g.fluid_solve(vt, ft)
    torch.cuda.synchronize()
    prm = oracle.params(L, rho=kw["rho"], eta=kw["eta"], dt=kw["dt"],
                        steady=mode == "steady", zero_mean=kw.get("zero_mean", False))
    ref = oracle.fluid_solve(prm, vt.double().cpu().numpy(), ft.double().cpu().numpy())
    check(f"solve {prec} L={L} {mode}", out.double().cpu().numpy(), ref, prec)
    # in place (v_in == v_out)
    g.fluid_solve(vt, ft, vt)
    torch.cuda.synchronize()
    check(f"solve in place {prec} L={L} {mode}", vt.double().cpu().numpy(), ref, prec)


@pytest.mark.parametrize("prec,L", [("mixed", 128), ("mixed", 144), ("fp64", 128)])
def test_fluid_solve_plane_pass_sizes(torch_cuda, prec, L):
    """The largest sizes whose inverse y and x transforms run as one plane
    per block (float32 L = 144 and float64 L = 128 with one block per CU),
    against the oracle on random fields."""
    torch = torch_cuda
    say("solve plane pass", prec, L)
    rng = np.random.default_rng(1000 + L)
    kw = dict(rho=1.3, eta=0.7, dt=0.05)
    g = grid(L, prec, 0, **kw)
    vt = torch.from_numpy(rng.standard_normal((3, L, L, L))).to(g.field_dtype).cuda()
    ft = torch.from_numpy(rng.standard_normal((3, L, L, L)) + 0.3).to(g.field_dtype).cuda()
    out = g.fluid_solve(vt, ft)
    torch.cuda.synchronize()
    prm = oracle.params(L, rho=kw["rho"], eta=kw["eta"], dt=kw["dt"])
    ref = oracle.fluid_solve(prm, vt.double().cpu().numpy(), ft.double().cpu().numpy())
    check(f"solve {prec} L={L}", out.double().cpu().numpy(), ref, prec)


@pytest.mark.parametrize("prec,L", [("fp64", 144), ("fp64", 192)])
def test_fluid_solve_z_pass_widths(torch_cuda, prec, L):
    """Float64 sizes above 128, whose z pass takes eight ky columns per block
    (one block per CU), against the oracle on random fields."""
    torch = torch_cuda
    say("solve z widths", prec, L)
    rng = np.random.default_rng(2000 + L)
    kw = dict(rho=1.3, eta=0.7, dt=0.05)
    g = grid(L, prec, 0, **kw)
    vt = torch.from_numpy(rng.standard_normal((3, L, L, L))).to(g.field_dtype).cuda()
    ft = torch.from_numpy(rng.standard_normal((3, L, L, L)) + 0.3).to(g.field_dtype).cuda()
    out = g.fluid_solve(vt, ft)
    torch.cuda.synchronize()
    prm = oracle.params(L, rho=kw["rho"], eta=kw["eta"], dt=kw["dt"])
    ref = oracle.fluid_solve(prm, vt.double().cpu().numpy(), ft.double().cpu().numpy())
    check(f"solve {prec} L={L}", out.double().cpu().numpy(), ref, prec)


_SOLVE_REFS = {}


def _solve_inputs_and_ref(L):
    """Random fields rounded to float32 (so that both precisions solve the
    same input) and the oracle's solve of them; computed once per size."""
    if L not in _SOLVE_REFS:
        rng = np.random.default_rng(3000 + L)
        v = rng.standard_normal((3, L, L, L)).astype(np.float32).astype(np.float64)
        f = (rng.standard_normal((3, L, L, L)) + 0.3).astype(np.float32).astype(np.float64)
        prm = oracle.params(L, rho=1.3, eta=0.7, dt=0.05)
        say(f"oracle solve {L}^3")
        _SOLVE_REFS.clear()
        _SOLVE_REFS[L] = (v, f, oracle.fluid_solve(prm, v, f))
    return _SOLVE_REFS[L]


@pytest.mark.parametrize("L,prec", [(72, "fp64"), (72, "mixed"), (216, "fp64"),
                                    (216, "mixed"), (288, "fp64"), (288, "mixed")])
def test_fluid_solve_radix3_sizes(torch_cuda, L, prec):
    """Sizes with factors 9 and 27 (72 = 8*9, 216 = 8*27, 288 = 32*9), whose
    transforms take two or three radix-3 stages, against the oracle."""
    torch = torch_cuda
    say("solve radix-3 size", prec, L)
    v, f, ref = _solve_inputs_and_ref(L)
    g = grid(L, prec, 0, rho=1.3, eta=0.7, dt=0.05)
    vt = torch.from_numpy(v).to(g.field_dtype).cuda()
    ft = torch.from_numpy(f).to(g.field_dtype).cuda()
    out = g.fluid_solve(vt, ft)
    torch.cuda.synchronize()
    check(f"solve {prec} L={L}", out.double().cpu().numpy(), ref, prec)


def _mode_sum(torch, L, modes, coef):
    """sum over modes m of Re(c_a exp(2 pi i m.(i,j,k)/L)) per component a,
    on the GPU in float64 ([3][L][L][L], x fastest); coef[n] is the complex
    3-vector of mode n."""
    idx = torch.arange(L, dtype=torch.int64, device="cuda")
    out = torch.zeros((3, L, L, L), dtype=torch.float64, device="cuda")
    for m, c in zip(modes, coef):
        # the phase index m.(i,j,k) mod L is exact in integers
        ph = (m[2] * idx[:, None, None] + m[1] * idx[None, :, None] + m[0] * idx[None, None, :]) % L
        ang = ph.to(torch.float64) * (2 * math.pi / L)
        cs, sn = torch.cos(ang), torch.sin(ang)
        for a in range(3):
            out[a] += c[a].real * cs - c[a].imag * sn
        del ph, ang, cs, sn
    return out


@pytest.mark.parametrize("prec,L", [("fp64", 256), ("mixed", 256), ("fp64", 384),
                                    ("mixed", 384), ("fp64", 432), ("mixed", 432),
                                    ("fp64", 512), ("mixed", 512)])
def test_fluid_solve_large_mode_sums(torch_cuda, prec, L):
    """The largest grids, checked by a property that holds at any size: the
    solve maps each Fourier mode m of v and f to the same mode,
    v'(m) = P(m) [(rho/dt - eta |D(m)|^2/2) v(m) + f(m)] / (rho/dt +
    eta |D(m)|^2/2), with D_b(m) = (1 - exp(-2 pi i m_b/L))/h and
    P = I - conj(D) D^T/|D|^2, and the mean by v' = v + (dt/rho) f.  The
    fields are sums of eight random modes (every axis, not divergence-free)
    plus a constant; the whole output is compared."""
    torch = torch_cuda
    say("solve mode sums", prec, L)
    rho, eta, dt, h = 1.3, 0.7, 0.05, 1.0
    rng = np.random.default_rng(4000 + L)
    modes = [tuple(int(x) for x in rng.integers(-L // 2 + 1, L // 2, size=3)) for _ in range(8)]
    modes = [m for m in dict.fromkeys(modes) if any(m)]
    cv = rng.standard_normal((len(modes), 3)) + 1j * rng.standard_normal((len(modes), 3))
    cf = rng.standard_normal((len(modes), 3)) + 1j * rng.standard_normal((len(modes), 3))
    v0, f0 = rng.standard_normal(3), rng.standard_normal(3)
    resp = []
    for m, a, b in zip(modes, cv, cf):
        D = (1 - np.exp(-2j * np.pi * np.array(m) / L)) / h
        d2 = float(np.sum(np.abs(D) ** 2))
        Pm = np.eye(3) - np.outer(np.conj(D), D) / d2
        resp.append(Pm @ ((rho / dt - eta * d2 / 2) * a + b) / (rho / dt + eta * d2 / 2))
    g = grid(L, prec, 0, rho=rho, eta=eta, dt=dt)
    v = _mode_sum(torch, L, modes, cv) + torch.tensor(v0, device="cuda")[:, None, None, None]
    f = _mode_sum(torch, L, modes, cf) + torch.tensor(f0, device="cuda")[:, None, None, None]
    vt, ft = v.to(g.field_dtype), f.to(g.field_dtype)
    del v, f
    out = g.fluid_solve(vt, ft)
    del vt, ft
    exp = _mode_sum(torch, L, modes, resp)
    exp += torch.tensor(v0 + dt / rho * f0, device="cuda")[:, None, None, None]
    err = (torch.linalg.vector_norm(out.double() - exp) / torch.linalg.vector_norm(exp)).item()
    say(f"mode sums L={L} {prec}: rel err {err:.3e} (tol {TOL[prec]:.0e})")
    assert err <= TOL[prec]
    del out, exp, g
    torch.cuda.empty_cache()


def _step_case(torch, w, prec, nsteps, v0=None, ref=None, **kw):
    from paper_1407_5600_amd import Springs
    g = grid(w.L, prec, w.M, rho=w.rho, eta=w.eta, dt=w.dt, **kw)
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    q = dev(torch, w.q)
    v = g.field() if v0 is None else torch.from_numpy(v0).to(g.field_dtype).cuda()
    vstart = v.double().cpu().numpy()
    Fe = dev(torch, w.Fext)
    u = torch.zeros_like(q)
    U0 = torch.zeros((w.P, 3), dtype=torch.float64, device="cuda")
    diag = torch.zeros(7, dtype=torch.float64, device="cuda")
    g.step(sp, q, v, Fe, nsteps, u, U0, diag)
    torch.cuda.synchronize()
    prm = oracle.params(w.L, rho=w.rho, eta=w.eta, dt=w.dt,
                        steady=kw.get("mode") == "steady",
                        zero_mean=kw.get("zero_mean", False))
    r = ref if ref is not None else oracle.step(prm, w.springs(), w.q, vstart, w.Fext, nsteps)
    name = f"step {w.name} {prec} n={nsteps}"
    check(name + " u", u.cpu().numpy(), r["u"], prec)
    check(name + " U0", U0.cpu().numpy(), r["U0"], prec)
    check(name + " v", v.double().cpu().numpy(), r["v"], prec)
    # Positions: q + dt u is rounded to the ulp of |q| on both sides (one
    # rounding with a fused multiply-add on the GPU, two on the CPU), so the
    # displacement agrees to the tolerance plus a few position ulps per step.
    qg = q.cpu().numpy()
    dq_ref = r["q"] - w.q
    ulp = np.spacing(np.abs(r["q"]).max())
    bound = TOL[prec] * np.abs(dq_ref).max() + 2 * nsteps * ulp
    err = np.abs(qg - r["q"]).max()
    say(f"{name} dq: max err {err:.3e} (bound {bound:.3e}), rel "
        f"{np.linalg.norm(qg - w.q - dq_ref) / np.linalg.norm(dq_ref):.3e}")
    assert err <= bound
    d = diag.cpu().numpy()
    # momentum is zero up to rounding when the mean mode is held at zero;
    # its error is measured against the summed magnitude of the field
    pscale = w.rho * w.h ** 3 * np.abs(r["v"]).sum(axis=(1, 2, 3))
    check(name + " momentum", d[:3], r["diag"][:3], prec,
          floor=np.linalg.norm(pscale))
    # the net force is a cancelling sum; its error is measured against the
    # summed magnitude of the blob forces (evaluated at the final positions)
    Fmag = np.abs(oracle.spring_forces(w.P, w.nb, w.pa, w.pb, w.r0, w.k, r["q"], w.Fext)).sum(0)
    check(name + " sumF", d[3:6], r["diag"][3:6], prec,
          floor=np.linalg.norm(Fmag))
    assert d[6] < (1e-10 if prec == "fp64" else 1e-3) * max(1.0, np.abs(r["v"]).max())
    g.last = {"u": u.cpu().numpy(), "U0": U0.cpu().numpy(), "v": v.double().cpu().numpy(),
              "q": qg}
    return g, r


def test_step_single_particle_fp64(torch_cuda):
    """The single-particle workload: 200 steps in float64 against the oracle."""
    torch = torch_cuda
    say("step single fp64 200")
    w = inputs.single()
    _step_case(torch, w, "fp64", 200)


def test_step_single_particle_mixed(torch_cuda):
    torch = torch_cuda
    say("step single mixed 20")
    w = inputs.single()
    _step_case(torch, w, "mixed", 20)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("L,P", [(24, 20), (32, 60), (48, 150)])
def test_step_suspension(torch_cuda, prec, L, P):
    torch = torch_cuda
    say("step suspension", prec, L, P)
    w = inputs.random_suspension(100 + L, L, P)
    v0 = oracle.fluid_solve(oracle.params(L, eta=0.0), np.random.default_rng(L).standard_normal((3, L, L, L)) * 0.1,
                            np.zeros((3, L, L, L)))
    _step_case(torch, w, prec, 3, v0=v0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_step_steady_stokes(torch_cuda, prec):
    torch = torch_cuda
    say("step steady", prec)
    w = inputs.random_suspension(7, 32, 25)
    _step_case(torch, w, prec, 3, mode="steady", zero_mean=True)


def test_step_zero_mean_and_no_external_force(torch_cuda):
    torch = torch_cuda
    say("step zero_mean")
    w = inputs.random_suspension(8, 24, 10)
    w.Fext[:] = 0.0
    # a decaying divergence-free flow carries the blobs; no force acts
    L = w.L
    v0 = oracle.fluid_solve(oracle.params(L, eta=0.0), np.random.default_rng(3).standard_normal((3, L, L, L)),
                            np.zeros((3, L, L, L)))
    for prec in ("fp64", "mixed"):
        _step_case(torch, w, prec, 2, v0=v0, zero_mean=True)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_step_dense_full_size(torch_cuda, prec):
    """The 128^3, phi = 0.3 suspension (36,669 particles, 476,697 blobs), one
    step in the launch configuration the benchmark times, every output
    compared with the oracle."""
    torch = torch_cuda
    say("step dense 128^3", prec)
    w = inputs.cached("dense")
    _step_case(torch, w, prec, 1)


def test_step_large_full_size(torch_cuda):
    """The 256^3, phi = 0.4 suspension (391,139 particles, 5,084,807 blobs):
    one step in float64 and one in mixed precision, in the launch
    configuration the benchmark times, each against the same oracle step
    (every output); the mixed step's error against the float64 step is
    printed."""
    torch = torch_cuda
    w = inputs.cached("large")
    L = w.L
    say(f"step large {L}^3: oracle step of {w.M} blobs (about a minute on one core)")
    prm = oracle.params(L, rho=w.rho, eta=w.eta, dt=w.dt)
    ref = oracle.step(prm, w.springs(), w.q, np.zeros((3, L, L, L)), w.Fext, 1)
    say("step large: oracle done")
    last = {}
    for prec in ("fp64", "mixed"):
        say(f"step large {L}^3 {prec}")
        g, _ = _step_case(torch, w, prec, 1, ref=ref)
        last[prec] = g.last
        del g
        torch.cuda.empty_cache()
    for k in ("u", "U0", "v"):
        say(f"step large: mixed vs float64 {k}: rel err {rel(last['mixed'][k], last['fp64'][k]):.3e}")
    dq = {p: last[p]["q"] - w.q for p in last}
    say(f"step large: mixed vs float64 dq: rel err {rel(dq['mixed'], dq['fp64']):.3e}")
    assert rel(last["mixed"]["U0"], last["fp64"]["U0"]) < TOL["mixed"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_spread_independent_of_blob_order(torch_cuda, prec):
    """Spreading sums in fixed point, so the field does not depend on the
    order of the blobs (nor of the atomic additions): a permuted input gives
    the same bits, and so does a repeated call."""
    torch = torch_cuda
    say("spread order", prec)
    L, M = 32, 3000
    q = blobs(1, M, L, "uniform")
    F = np.random.default_rng(2).standard_normal((M, 3))
    perm = np.random.default_rng(3).permutation(M)
    g = grid(L, prec, M)
    a = g.spread(dev(torch, q), dev(torch, F)).cpu().numpy()
    b = g.spread(dev(torch, q[perm]), dev(torch, F[perm])).cpu().numpy()
    c = g.spread(dev(torch, q), dev(torch, F)).cpu().numpy()
    assert np.array_equal(a, b) and np.array_equal(a, c)
    check(f"spread order {prec}", a, oracle.spread(oracle.params(L), q, F), prec)


@pytest.mark.parametrize("prec,M", [("mixed", 70000), ("fp64", 70000), ("fp64", 1100000)])
def test_spread_crowded_tile(torch_cuda, prec, M):
    """More records in one tile than the fast fixed-point forms are sized
    for: mixed falls back to 64-bit integer sums above 2048 records, float64
    coarsens its quantum above ~27,000 and falls back to float64 LDS atomics
    above 2^20; next to tiles of ordinary density."""
    torch = torch_cuda
    say("spread crowded tile", prec, M)
    L = 8 if M > 100000 else 16
    rng = np.random.default_rng(9)
    q = 4.0 + rng.uniform(0.0, 2.0, size=(M, 3))
    q[:10] = rng.uniform(0, L, size=(10, 3))
    F = rng.standard_normal((M, 3))
    g = grid(L, prec, M)
    f = g.spread(dev(torch, q), dev(torch, F))
    torch.cuda.synchronize()
    ref = oracle.spread(oracle.params(L), q, F)
    check(f"spread crowded {prec} M={M}", f.double().cpu().numpy(), ref, prec)


@pytest.mark.parametrize("M", [1, 262, 263, 269, 526, 263 * 269])
def test_spread_box_tile_record_counts(torch_cuda, M):
    """Float32 spreading takes the k-th record of a box tile at position
    (k P) mod n, P = 263, or 269 where 263 divides the tile's count n, or 1
    where 269 does too: every record must be taken exactly once.  At L = 16
    one box tile holds every blob, so n = M; 263 * 269 records also take
    the 64-bit sums (more than 2048)."""
    torch = torch_cuda
    say("spread box-tile record count", M)
    L = 16
    rng = np.random.default_rng(M)
    q = rng.uniform(0.0, L, size=(M, 3))
    F = rng.standard_normal((M, 3))
    g = grid(L, "mixed", M)
    perm = rng.permutation(M)
    a = g.spread(dev(torch, q), dev(torch, F)).cpu().numpy()
    b = g.spread(dev(torch, q[perm]), dev(torch, F[perm])).cpu().numpy()
    assert np.array_equal(a, b)
    check(f"spread record count M={M}", a, oracle.spread(oracle.params(L), q, F), "mixed")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["suspension", "steady", "batch", "tile8", "fast", "crowded",
                                  "crowded_fast"])
def test_step_call_binning_carry_is_exact(torch_cuda, prec, case):
    """Within one call of several first-order steps, each step after the
    first takes its binning from the interpolation that moved the blobs.
    Spreading sums in fixed point and the rest works per blob, per cell or
    per tile, so the result equals that of one call per step bit for bit
    (suspension, steady Stokes, a batch of boxes, small tiles; "fast": blobs
    that move more than a tile per step, which take the global-atomic path;
    "crowded": several hundred blobs per tile, more than the block's
    threads, whose extra records are counted in a second pass).  The last
    step leaves the counts at zero: a following call bins afresh."""
    from paper_1407_5600_amd import Springs
    torch = torch_cuda
    say("binning carry", prec, case)
    nbox, kw = 1, {}
    if case == "batch":
        nbox = 3
        ws = [inputs.random_suspension(40 + b, 32, 40) for b in range(nbox)]
        w = ws[0]
        q0 = np.concatenate([x.q for x in ws])
        Fe = np.concatenate([x.Fext for x in ws])
    elif case.startswith("crowded"):
        # 400 overlapping particles in [4, 12)^3 of a 64^3 box: ~1,300 blobs
        # in each of the 4 tiles (16x8x8) they cover; with the flow (1.25
        # tiles per step along x) some move beyond the neighbour tiles
        w = inputs.random_suspension(33, 64, 1)
        rng = np.random.default_rng(34)
        P = 400
        tmpl = w.q - w.q.mean(axis=0)
        cent = rng.uniform(4.0, 12.0, size=(P, 1, 3))
        q0 = (cent + tmpl[None, :, :]).reshape(-1, 3)
        Fe = rng.standard_normal((P, 3))
    else:
        w = inputs.random_suspension(31, 48, 150)
        q0, Fe = w.q, w.Fext
        if case == "steady":
            kw = {"mode": "steady", "zero_mean": True}

    M = q0.shape[0]
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    out = []
    for calls in ([5], [1, 1, 1, 1, 1], [2, 3]):
        g = grid(w.L, prec, M, rho=w.rho, eta=w.eta, dt=w.dt, nbox=nbox, **kw)
        if case == "tile8":
            g.set_tiles(8, 8, 8)
        q = dev(torch, q0)
        v = g.field()
        if case.endswith("fast"):
            v[0] += 2000.0  # a uniform flow carries the blobs 20 cells per step
        F = dev(torch, Fe)
        diag = torch.zeros(7, dtype=torch.float64, device="cuda")
        U0 = torch.zeros((M // w.nb, 3), dtype=torch.float64, device="cuda")
        for n in calls:
            g.step(sp, q, v, F, n, None, U0, diag)
        torch.cuda.synchronize()
        out.append([x.cpu().numpy() for x in (q, v, U0, diag)])
        if calls == [5] and case.endswith("fast"):
            moved = np.abs(out[0][0] - q0).max()
            say(f"binning carry fast: max move {moved:.2f} cells over 5 steps")
            assert moved > 5 * 16, "the fast case must move blobs beyond a tile per step"
    for o in out[1:]:
        for a, b in zip(out[0], o):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["suspension", "batch", "midpoint"])
def test_step_call_particle_order_is_exact(torch_cuda, prec, case):
    """A call of many steps runs them with the particles reordered by tile
    (its own copy of the positions, scattered back at the end).  Its
    positions, fluid velocity, blob and particle velocities and momentum
    equal those of one call per step bit for bit; the net force, a float64
    sum over blocks of particles, agrees to rounding."""
    from paper_1407_5600_amd import Springs
    torch = torch_cuda
    say("particle order", prec, case)
    nbox, n = 1, 10
    if case == "batch":
        nbox = 3
        ws = [inputs.random_suspension(60 + b, 32, 40) for b in range(nbox)]
        w = ws[0]
        q0 = np.concatenate([x.q for x in ws])
        Fe = np.concatenate([x.Fext for x in ws])
    else:
        w = inputs.random_suspension(62, 48, 150)
        q0, Fe = w.q, w.Fext
    M = q0.shape[0]
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    out = []
    for calls in ([n], [1] * n):
        g = grid(w.L, prec, M, rho=w.rho, eta=w.eta, dt=w.dt, nbox=nbox,
                 scheme="midpoint" if case == "midpoint" else "euler")
        q = dev(torch, q0)
        v = g.field()
        F = dev(torch, Fe)
        u = torch.zeros_like(q)
        U0 = torch.zeros((M // w.nb, 3), dtype=torch.float64, device="cuda")
        diag = torch.zeros(7, dtype=torch.float64, device="cuda")
        for k in calls:
            g.step(sp, q, v, F, k, u, U0, diag)
        torch.cuda.synchronize()
        out.append([x.cpu().numpy() for x in (q, v, u, U0, diag)])
    for a, b in zip(out[0][:4], out[1][:4]):
        assert np.array_equal(a, b)
    assert np.array_equal(out[0][4][:3], out[1][4][:3]) and out[0][4][6] == out[1][4][6]
    assert np.allclose(out[0][4][3:6], out[1][4][3:6], rtol=0, atol=1e-12 * np.abs(Fe).sum())
