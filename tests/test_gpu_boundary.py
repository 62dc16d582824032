"""The boundary's set-up and error contract on the GPU: a caller-given
workspace (mb_workspace_size / mb_grid_set_workspace) gives the same bits as
the library's own scratch, check_finite reports non-finite positions and
forces as MB_ERR_NONFINITE, deterministic grids repeat bit for bit, and
misaligned pointers are rejected."""
import ctypes
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


def _run_steps(torch, g, w, nsteps, tiles=None):
    from paper_1407_5600_amd import Springs
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    if tiles:
        g.set_tiles(*tiles)
    q = dev(torch, w.q)
    v = g.field()
    U0 = torch.zeros((w.P, 3), dtype=torch.float64, device="cuda")
    diag = torch.zeros(7, dtype=torch.float64, device="cuda")
    g.step(sp, q, v, dev(torch, w.Fext), nsteps, None, U0, diag)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (q, v, U0, diag)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_torch_workspace_gives_the_same_bits(torch_cuda, prec):
    """A grid whose scratch is a torch tensor (external_workspace, then
    mb_grid_set_workspace) steps exactly as one with library scratch, also
    after a tile-shape change and after moving to a second workspace."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid
    say("torch workspace", prec)
    w = inputs.random_suspension(61, 48, 120)
    kw = dict(precision=prec, max_blobs=w.M, rho=w.rho, eta=w.eta, dt=w.dt)
    ref = _run_steps(torch, Grid(w.L, **kw), w, 4)
    g = Grid(w.L, workspace="torch", **kw)
    assert g.workspace.numel() == g.workspace_size() > 0
    got = _run_steps(torch, g, w, 4)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    ref8 = _run_steps(torch, Grid(w.L, **kw), w, 3, tiles=(8, 8, 8))
    got8 = _run_steps(torch, g, w, 3, tiles=(8, 8, 8))
    for a, b in zip(ref8, got8):
        assert np.array_equal(a, b)
    # a second, larger workspace tensor of the caller's
    buf = torch.empty(g.workspace_size() + 4096, dtype=torch.uint8, device="cuda")
    g.set_workspace(buf)
    got8b = _run_steps(torch, g, w, 3)
    for a, b in zip(ref8, got8b):
        assert np.array_equal(a, b)
    r = oracle.step(oracle.params(w.L, rho=w.rho, eta=w.eta, dt=w.dt), w.springs(), w.q,
                    np.zeros((3, w.L, w.L, w.L)), w.Fext, 4)
    assert rel(got[2], r["U0"]) < TOL[prec]


def test_workspace_contract(torch_cuda):
    torch = torch_cuda
    from paper_1407_5600_amd import Grid, MultiblobError, binding
    say("workspace contract")
    L = 32
    g = Grid(L, max_blobs=26)
    g.desc.external_workspace = 1
    h = ctypes.c_void_p()
    assert binding.lib().mb_grid_create(ctypes.byref(g.desc), ctypes.byref(h)) == binding.MB_OK
    bare = h
    f = g.field()
    q = torch.zeros((26, 3), dtype=torch.float64, device="cuda")
    # no workspace yet: every call is refused
    st = binding.lib().mb_spread(bare, 26, ctypes.c_void_p(q.data_ptr()),
                                 ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                 None)
    assert st == binding.MB_ERR_INVALID
    n = binding.lib().mb_workspace_size(ctypes.byref(g.desc), 1)
    buf = torch.empty(n + 512, dtype=torch.uint8, device="cuda")
    lib = binding.lib()
    assert lib.mb_grid_set_workspace(bare, ctypes.c_void_p(buf.data_ptr()), n - 256) == \
        binding.MB_ERR_INVALID  # too small
    assert lib.mb_grid_set_workspace(bare, ctypes.c_void_p(buf.data_ptr() + 8), n) == \
        binding.MB_ERR_INVALID  # misaligned
    assert lib.mb_grid_set_workspace(bare, ctypes.c_void_p(buf.data_ptr()), n) == binding.MB_OK
    st = lib.mb_spread(bare, 26, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                       ctypes.c_void_p(f.data_ptr()), None)
    torch.cuda.synchronize()
    assert st == binding.MB_OK and float(f.abs().max()) == 0.0
    assert lib.mb_grid_destroy(bare) == binding.MB_OK
    # misaligned field and blob pointers
    v = torch.zeros(3 * L ** 3 + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(MultiblobError):
        binding._check(lib.mb_fluid_solve(g.handle, ctypes.c_void_p(v.data_ptr() + 8),
                                          ctypes.c_void_p(v.data_ptr()),
                                          ctypes.c_void_p(v.data_ptr()), None), "solve")
    qq = torch.zeros(27 * 3, dtype=torch.float64, device="cuda")
    u = torch.zeros((26, 3), dtype=torch.float64, device="cuda")
    assert lib.mb_interpolate(g.handle, 26, ctypes.c_void_p(qq.data_ptr() + 24),
                              ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                              None) == binding.MB_ERR_INVALID


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("bad", ["nan_position", "inf_force", "coincident_blobs"])
def test_check_finite(torch_cuda, prec, bad):
    """check_finite: a NaN position, an infinite external force or two blobs
    of a particle at the same place (a spring of zero length) make the step
    report MB_ERR_NONFINITE; the flag is cleared, so a finite state then
    steps normally and matches a grid without the check."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid, MultiblobError, Springs, binding
    say("check_finite", prec, bad)
    w = inputs.random_suspension(71, 32, 20)
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    kw = dict(precision=prec, max_blobs=w.M, rho=w.rho, eta=w.eta, dt=w.dt)
    g = Grid(w.L, check_finite=True, **kw)
    q0 = w.q.copy()
    Fe = w.Fext.copy()
    if bad == "nan_position":
        q0[17, 1] = np.nan
    elif bad == "inf_force":
        Fe[3, 0] = np.inf
    else:
        q0[13 * 5 + 2] = q0[13 * 5 + 7]
    q = dev(torch, q0)
    v = g.field()
    with pytest.raises(MultiblobError) as ex:
        g.step(sp, q, v, dev(torch, Fe), 2)
    assert ex.value.status == binding.MB_ERR_NONFINITE
    if bad == "nan_position":
        with pytest.raises(MultiblobError) as ex:
            g.spread(q, dev(torch, np.ones_like(q0)))
        assert ex.value.status == binding.MB_ERR_NONFINITE
        with pytest.raises(MultiblobError) as ex:
            g.interpolate(q, g.field())
        assert ex.value.status == binding.MB_ERR_NONFINITE
    # a finite state after the failure: same bits as an unchecked grid
    out = []
    for gg in (g, Grid(w.L, **kw)):
        q = dev(torch, w.q)
        v = gg.field()
        U0 = torch.zeros((w.P, 3), dtype=torch.float64, device="cuda")
        gg.step(sp, q, v, dev(torch, w.Fext), 3, None, U0)
        torch.cuda.synchronize()
        out.append((q.cpu().numpy(), v.cpu().numpy(), U0.cpu().numpy()))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_deterministic_crowded_float64_spreading(torch_cuda):
    """More than 2^20 records in one float64 spreading tile: the default grid
    sums them with float64 LDS atomics, a deterministic grid in 64-bit fixed
    point; the deterministic result repeats bit for bit (also with the blobs
    permuted) and both agree with the oracle."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid
    say("deterministic crowded spreading")
    L, M = 8, 1100000
    rng = np.random.default_rng(9)
    q = 4.0 + rng.uniform(0.0, 2.0, size=(M, 3))
    F = rng.standard_normal((M, 3))
    perm = rng.permutation(M)
    ref = oracle.spread(oracle.params(L), q, F)
    g = Grid(L, precision="fp64", max_blobs=M, deterministic=True)
    a = g.spread(dev(torch, q), dev(torch, F)).cpu().numpy()
    b = g.spread(dev(torch, q[perm]), dev(torch, F[perm])).cpu().numpy()
    c = g.spread(dev(torch, q), dev(torch, F)).cpu().numpy()
    assert np.array_equal(a, b) and np.array_equal(a, c)
    e = rel(a, ref)
    say(f"deterministic crowded: rel err {e:.3e}")
    assert e < TOL["fp64"]


def test_deterministic_adjoint_sums(torch_cuda):
    """mb_step_adjoint on a deterministic grid: the stiffness and rest-length
    derivatives are summed per block in a fixed order, so two reverse
    sweeps give the same bits; they agree with a default grid's (float64
    atomics) to rounding."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid, Springs
    say("deterministic adjoint sums")
    w = inputs.random_suspension(81, 32, 60)
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    qbar0 = np.random.default_rng(3).standard_normal((w.M, 3))
    outs = {}
    for det in (True, False):
        g = Grid(w.L, max_blobs=w.M, rho=w.rho, eta=w.eta, dt=w.dt, deterministic=det)
        q = dev(torch, w.q)
        v = g.field()
        g.step(sp, q, v, dev(torch, w.Fext), 1)
        runs = []
        for _ in range(2):
            qbar = dev(torch, qbar0)
            vbar = torch.ones_like(v)
            kbar = torch.zeros(1, dtype=torch.float64, device="cuda")
            r0bar = torch.zeros(len(w.pa), dtype=torch.float64, device="cuda")
            g.step_adjoint(sp, dev(torch, w.q), v, qbar, vbar, Fext=dev(torch, w.Fext),
                           kbar=kbar, r0bar=r0bar)
            torch.cuda.synchronize()
            runs.append((kbar.cpu().numpy(), r0bar.cpu().numpy(), qbar.cpu().numpy()))
        outs[det] = runs
    (k1, r1, q1), (k2, r2, q2) = outs[True]
    assert np.array_equal(k1, k2) and np.array_equal(r1, r2) and np.array_equal(q1, q2)
    kd, rd, qd = outs[False][0]
    say(f"kbar det {k1[0]:.15e} atomics {kd[0]:.15e}")
    assert abs(k1[0] - kd[0]) <= 1e-12 * abs(kd[0])
    assert rel(r1, rd) < 1e-12 and rel(q1, qd) < 1e-12


def test_springs_set_params(torch_cuda):
    """mb_springs_set_params: a table given new rest lengths and stiffness
    computes what a new table with them computes."""
    torch = torch_cuda
    from paper_1407_5600_amd import Springs, spring_forces
    say("springs set params")
    w = inputs.random_suspension(91, 24, 10)
    q = dev(torch, w.q + 0.05 * np.random.default_rng(1).standard_normal(w.q.shape))
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    r0n = np.asarray(w.r0) * 1.07
    sp.set_params(r0n, 37.5)
    got = spring_forces(sp, q, dev(torch, w.Fext)).cpu().numpy()
    ref = spring_forces(Springs(w.nb, w.pa, w.pb, r0n, 37.5), q,
                        dev(torch, w.Fext)).cpu().numpy()
    assert np.array_equal(got, ref)
    exp = oracle.spring_forces(w.P, w.nb, w.pa, w.pb, r0n, 37.5, q.cpu().numpy(), w.Fext)
    assert rel(got, exp) < TOL["fp64"]
