"""Tile shapes of the binning, spreading and interpolation: every shape with
kernels against the oracle (spread, interpolation, interpolation gradient,
steps), and the autotuner (leaves the caller's state alone, keeps a shape
that fits, steps correctly afterwards)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1407_5600_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}
SHAPES = [(16, 8, 8), (8, 8, 8), (32, 8, 8), (16, 16, 8), (16, 8, 16), (8, 16, 16)]


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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", SHAPES)
def test_tile_shape_vs_oracle(torch_cuda, prec, shape):
    torch = torch_cuda
    from paper_1407_5600_amd import Grid, Springs
    say("tiles", shape, prec)
    w = inputs.random_suspension(40, 32, 60)
    L = w.L
    rng = np.random.default_rng(7)
    F = rng.standard_normal((w.M, 3))
    vfield = rng.standard_normal((3, L, L, L))
    W = rng.standard_normal((w.M, 3))
    g = Grid(L, precision=prec, max_blobs=w.M, rho=w.rho, eta=w.eta, dt=w.dt)
    g.set_tiles(*shape)
    assert g.tiles == shape
    prm = oracle.params(L, rho=w.rho, eta=w.eta, dt=w.dt)
    q = dev(torch, w.q)
    f = g.spread(q, dev(torch, F))
    vd = torch.from_numpy(vfield).to(g.field_dtype).cuda()
    u = g.interpolate(q, vd)
    gr = torch.zeros_like(q)
    g.interpolate_grad(q, vd, dev(torch, W), gr)
    torch.cuda.synchronize()
    vref = vd.double().cpu().numpy()
    tol = TOL[prec]
    e = {"spread": rel(f.double().cpu().numpy(), oracle.spread(prm, w.q, F)),
         "interp": rel(u.cpu().numpy(), oracle.interpolate(prm, w.q, vref)),
         "interp_grad": rel(gr.cpu().numpy(), oracle.interpolate_grad(prm, w.q, vref, W))}
    # steps
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    qs = dev(torch, w.q)
    v = g.field()
    U0 = torch.zeros((w.P, 3), dtype=torch.float64, device="cuda")
    g.step(sp, qs, v, dev(torch, w.Fext), 3, U0_out=U0)
    torch.cuda.synchronize()
    r = oracle.step(prm, w.springs(), w.q, np.zeros((3, L, L, L)), w.Fext, 3)
    e["step v"] = rel(v.double().cpu().numpy(), r["v"])
    e["step U0"] = rel(U0.cpu().numpy(), r["U0"])
    say(" ".join(f"{k} {x:.2e}" for k, x in e.items()))
    for k, x in e.items():
        assert x < tol, (k, x)


def test_set_tiles_rejects_unsupported(torch_cuda):
    from paper_1407_5600_amd import Grid, MultiblobError
    g = Grid(24, max_blobs=26)
    for shape in [(16, 8, 8), (32, 8, 8), (8, 8, 4), (12, 8, 8), (16, 16, 16)]:
        with pytest.raises(MultiblobError):
            g.set_tiles(*shape)   # 16 and 32 do not divide 24; no kernels for the rest
    assert g.tiles == (8, 8, 8)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_autotune_dense(torch_cuda, prec):
    """On the 128^3 suspension: the tuner keeps a shape that fits, leaves
    the caller's q and v unchanged, and the next steps agree with the
    oracle."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid, Springs
    w = inputs.cached("dense")
    g = Grid(w.L, precision=prec, max_blobs=w.M, rho=w.rho, eta=w.eta, dt=w.dt)
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    q = dev(torch, w.q)
    v = g.field()
    Fe = dev(torch, w.Fext)
    q_before = q.clone()
    shape = g.autotune(sp, q, v, Fe, nsteps=5)
    torch.cuda.synchronize()
    say("autotune", prec, shape)
    assert tuple(shape) in SHAPES and g.tiles == tuple(shape)
    assert torch.equal(q, q_before) and not bool(v.abs().max() > 0)
    U0 = torch.zeros((w.P, 3), dtype=torch.float64, device="cuda")
    g.step(sp, q, v, Fe, 1, U0_out=U0)
    torch.cuda.synchronize()
    r = oracle.step(oracle.params(w.L, rho=w.rho, eta=w.eta, dt=w.dt), w.springs(), w.q,
                    np.zeros((3, w.L, w.L, w.L)), w.Fext, 1)
    assert rel(U0.cpu().numpy(), r["U0"]) < TOL[prec]
