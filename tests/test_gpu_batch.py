"""Batches of independent boxes (the pair-mobility sweep set-up): a batch
grid advances nbox equal boxes in one launch per kernel and must give, box
by box, what the single-box path gives (which the parity suite holds to the
oracle); the graph-captured multi-grid step must equal eager steps on every
replay."""
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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def _springs():
    from paper_1407_5600_amd import Springs
    tmpl = inputs.icosahedron_template(1.0)
    pa, pb, r0 = inputs.pair_table(tmpl)
    return Springs(len(tmpl), pa, pb, r0, 100.0), {"nb": len(tmpl), "pa": pa, "pb": pb,
                                                   "r0": r0, "k": 100.0}


@pytest.mark.parametrize("prec,L,nbox", [("fp64", 24, 5), ("mixed", 32, 7), ("fp64", 48, 3)])
def test_batch_matches_single_boxes(torch_cuda, prec, L, nbox):
    """Spread, solve, interpolate and 6 steps of a batch against the same
    boxes one at a time."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid
    say("batch vs single", prec, L, nbox)
    boxes = [b for b in inputs.pair_sweep(seed=L + nbox, nbox=8 * nbox, sizes=(L,))][:nbox]
    sp, _ = _springs()
    Mb = boxes[0]["q"].shape[0]
    qb = np.concatenate([b["q"] for b in boxes])
    Fe = np.concatenate([b["Fext"] for b in boxes])
    F = np.random.default_rng(1).standard_normal(qb.shape)
    gb = Grid(L, precision=prec, max_blobs=nbox * Mb, nbox=nbox)
    fb = gb.spread(dev(torch, qb), dev(torch, F))
    vb = gb.fluid_solve(gb.field(), fb)
    ub = gb.interpolate(dev(torch, qb), vb)
    q_run = dev(torch, qb)
    v_run = gb.field()
    gb.step(sp, q_run, v_run, dev(torch, Fe), 6)
    torch.cuda.synchronize()
    for i, b in enumerate(boxes):
        g1 = Grid(L, precision=prec, max_blobs=Mb)
        sl = slice(i * Mb, (i + 1) * Mb)
        f1 = g1.spread(dev(torch, b["q"]), dev(torch, F[sl]))
        v1 = g1.fluid_solve(g1.field(), f1)
        u1 = g1.interpolate(dev(torch, b["q"]), v1)
        q1 = dev(torch, b["q"])
        w1 = g1.field()
        g1.step(sp, q1, w1, dev(torch, b["Fext"]), 6)
        torch.cuda.synchronize()
        assert torch.equal(fb[i], f1), f"spread box {i}"
        assert torch.equal(vb[i], v1), f"solve box {i}"
        assert torch.equal(ub[sl], u1), f"interp box {i}"
        assert rel(q_run[sl].cpu().numpy() - b["q"], q1.cpu().numpy() - b["q"]) < 1e-13
        assert rel(v_run[i].double().cpu().numpy(), w1.double().cpu().numpy()) < 1e-13


TOL = {"fp64": 1e-12, "mixed": 1e-5}


@pytest.mark.parametrize("prec,L", [("fp64", 24), ("fp64", 48), ("mixed", 24), ("mixed", 32),
                                    ("mixed", 48), ("mixed", 64)])
def test_batch_step_vs_oracle(torch_cuda, prec, L):
    """Four steps of a batch of three pair boxes (the edge sizes of the pair
    sweep) against the oracle stepping each box alone: particle velocities,
    fluid velocity and positions of every box."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid
    say("batch vs oracle", prec, L)
    nbox, n = 3, 4
    boxes = inputs.pair_sweep(seed=11 + L, nbox=12, sizes=(L,))[:nbox]
    sp, spd = _springs()
    Mb = boxes[0]["q"].shape[0]
    q = dev(torch, np.concatenate([b["q"] for b in boxes]))
    g = Grid(L, precision=prec, max_blobs=nbox * Mb, nbox=nbox)
    vv = g.field()
    U0 = torch.empty((2 * nbox, 3), dtype=torch.float64, device="cuda")
    g.step(sp, q, vv, dev(torch, np.concatenate([b["Fext"] for b in boxes])), n, U0_out=U0)
    torch.cuda.synchronize()
    tol = TOL[prec]
    for i, b in enumerate(boxes):
        ref = oracle.step(oracle.params(L), spd, b["q"], np.zeros((3, L, L, L)), b["Fext"], n)
        sl = slice(i * Mb, (i + 1) * Mb)
        eU = rel(U0[2 * i:2 * i + 2].cpu().numpy(), ref["U0"])
        ev = rel(vv[i].double().cpu().numpy(), ref["v"])
        # positions: q + dt u rounds to the ulp of |q| once per step on
        # each side (a fused multiply-add on the GPU, two roundings on the CPU)
        qg = q[sl].cpu().numpy()
        dq = ref["q"] - b["q"]
        bound = tol * np.abs(dq).max() + 2 * n * np.spacing(np.abs(ref["q"]).max())
        eq = np.abs(qg - ref["q"]).max()
        say(f"box {i}: U0 {eU:.2e} v {ev:.2e} dq max err {eq:.2e} (bound {bound:.2e})")
        assert eU < tol and ev < tol and eq <= bound


def test_graph_replays_match_eager_steps(torch_cuda):
    """Three grids (batches of different box sizes, one mixed) stepped by
    the captured graph and eagerly: equal after 5 replays, and again after
    eager work and synchronisations, replay by replay.  The eager steps of
    these grids scan the tile counts inside the springs kernel, the captured
    ones in the separate scan kernel: the two give the same offsets."""
    torch = torch_cuda
    from paper_1407_5600_amd import Grid
    from paper_1407_5600_amd.binding import step_graph
    say("graph replays")
    sp, _ = _springs()
    specs = [(24, 4, "fp64"), (32, 3, "mixed"), (48, 2, "fp64")]
    grids, eg, qs, qe, vs, ve, fe = [], [], [], [], [], [], []
    for L, nbox, prec in specs:
        boxes = inputs.pair_sweep(seed=L, nbox=10 * nbox, sizes=(L,))[:nbox]
        Mb = boxes[0]["q"].shape[0]
        q = np.concatenate([b["q"] for b in boxes])
        F = np.concatenate([b["Fext"] for b in boxes])
        for lst_g, lst_q, lst_v in ((grids, qs, vs), (eg, qe, ve)):
            g = Grid(L, precision=prec, max_blobs=nbox * Mb, nbox=nbox)
            lst_g.append(g)
            lst_q.append(dev(torch, q))
            lst_v.append(g.field())
        fe.append(dev(torch, F))
    spr = [sp] * len(specs)

    def eager(n):
        for g, q, v, F in zip(eg, qe, ve, fe):
            g.step(sp, q, v, F, n)

    def same():
        torch.cuda.synchronize()
        for a, b in zip(qs + vs, qe + ve):
            assert torch.equal(a, b)

    step_graph(grids, spr, qs, vs, fe, None, 5)
    eager(5)
    same()
    for _ in range(3):
        _ = (qs[0] * 2.0).sum().item()  # eager work and a synchronisation
        step_graph(grids, spr, qs, vs, fe, None, 1)
        eager(1)
        same()
    step_graph(grids, spr, qs, vs, fe, None, 4)
    eager(4)
    same()
