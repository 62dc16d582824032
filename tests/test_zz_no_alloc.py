"""The allocation-free step (mb_step_noalloc, its workspace in the library's
static device array) against mb_step on a grid of the same description:
two calls in a row, the second on a smaller grid with fewer blobs, and a
description whose workspace exceeds the static array (rejected)."""
import sys

import numpy as np
import pytest

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


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def _both(torch, w, prec, nsteps, v0):
    """(mb_step on a grid, mb_step_noalloc) outputs for the same state."""
    from paper_1407_5600_amd import Grid, Springs
    from paper_1407_5600_amd.binding import step_noalloc
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    out = []
    for noalloc in (False, True):
        q = torch.from_numpy(w.q.copy()).cuda()
        fdt = torch.float64 if prec == "fp64" else torch.float32
        v = torch.from_numpy(v0).to(fdt).cuda()
        Fe = torch.from_numpy(w.Fext).cuda()
        u = torch.zeros_like(q)
        U0 = torch.zeros((w.P, 3), dtype=torch.float64, device="cuda")
        diag = torch.zeros(7, dtype=torch.float64, device="cuda")
        if noalloc:
            step_noalloc(sp, q, v, Fe, nsteps, u, U0, diag, L=w.L, rho=w.rho, eta=w.eta,
                         dt=w.dt, precision=prec)
        else:
            g = Grid(w.L, precision=prec, max_blobs=w.M, rho=w.rho, eta=w.eta, dt=w.dt)
            g.step(sp, q, v, Fe, nsteps, u, U0, diag)
        torch.cuda.synchronize()
        out.append({"q": q.cpu().numpy(), "v": v.double().cpu().numpy(),
                    "u": u.cpu().numpy(), "U0": U0.cpu().numpy(), "diag": diag.cpu().numpy()})
    return out


def test_noalloc_step_matches_grid_step(torch_cuda):
    torch = torch_cuda
    cases = [(48, 150, "mixed", 4), (32, 40, "fp64", 3)]  # the second one smaller
    for L, P, prec, n in cases:
        say("noalloc", L, P, prec, n)
        w = inputs.random_suspension(500 + L, L, P)
        v0 = 0.05 * np.random.default_rng(L).standard_normal((3, L, L, L))
        ref, got = _both(torch, w, prec, n, v0)
        for k in ("u", "U0", "v", "diag"):
            e = rel(got[k], ref[k])
            say(f"noalloc {prec} L={L} {k}: rel {e:.2e} (bitwise {np.array_equal(got[k], ref[k])})")
            assert e <= TOL[prec], k
        dq = ref["q"] - w.q
        assert np.abs(got["q"] - ref["q"]).max() <= TOL[prec] * np.abs(dq).max()


def test_noalloc_rejects_beyond_its_scratch(torch_cuda):
    torch = torch_cuda
    from paper_1407_5600_amd import MultiblobError, Springs, binding
    from paper_1407_5600_amd.binding import step_noalloc
    w = inputs.random_suspension(7, 128, 10)
    sp = Springs(w.nb, w.pa, w.pb, w.r0, w.k)
    q = torch.from_numpy(w.q.copy()).cuda()
    v = torch.zeros((3, 128, 128, 128), dtype=torch.float64, device="cuda")
    with pytest.raises(MultiblobError) as ex:
        step_noalloc(sp, q, v, torch.from_numpy(w.Fext).cuda(), 1, L=128)
    assert ex.value.status == binding.MB_ERR_UNSUPPORTED
