"""Seeded synthetic inputs shaped like the paper's colloid configurations.

This module builds inputs only: particle templates, pair tables, particle
placements, orientations and external forces.  It holds none of the step's
arithmetic (no kernel, spreading, interpolation, spring force or fluid solve)
and imports neither the GPU library nor the oracle, so both sides can be fed
identical arrays.

Particle model (Sec. "Multiblob particle model", Fig. 1): 12 blobs on the
vertices of an icosahedron of circumradius ``a`` plus one blob at its centre
(index 12), all pairs joined by harmonic springs whose rest lengths are the
template distances.  The circumradius relates to the vertex distance d as
a = sqrt(10 + 2 sqrt 5) / 4 * d = 0.95106 d (appendix, eq. jm2a context).

Workloads (all h = 1, periodic cubic boxes):
  single   one particle in a 32^3 box, centre uniform in the box, canonical
           orientation, Fext = (1, 0, 0).
  dense    128^3 box, 36,669 particles at volume fraction 0.3 for the
           effective radius 1.6 h, random sequential addition with centre
           distance >= 3.2 h, uniformly random orientations,
           Fext ~ N(0, 1) per component.
  large    256^3 box, 391,139 particles at volume fraction 0.4; random
           sequential addition cannot reach 0.4 (its jamming limit is about
           0.38), so centres start on a random subset of a 74^3 simple-cubic
           lattice (bounded random displacements keep every pair at least
           3.2 h apart) and are then moved by hard-sphere Monte Carlo sweeps,
           the paper's preparation of dense configurations for its
           viscosity runs.
  pair     two particles separated along x (pair-mobility set-up).
  diff     64^3 box with 16 particles by random sequential addition.
The seeded generator is numpy's PCG64 (``numpy.random.default_rng``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0
CIRCUMRADIUS_OVER_EDGE = math.sqrt(10.0 + 2.0 * math.sqrt(5.0)) / 4.0
EFFECTIVE_RADIUS = 1.6  # hard-sphere radius used to set volume fractions


def icosahedron_template(a: float = 1.0, centre: bool = True) -> np.ndarray:
    """Blob offsets s_i from the particle centre, shape (13, 3) (or (12, 3)).

    Vertices are the cyclic permutations of (0, +-1, +-golden), scaled to
    circumradius ``a``; the centre blob, if present, is last."""
    verts = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            base = (0.0, s1, s2 * GOLDEN)
            for rot in range(3):
                verts.append(base[-rot:] + base[:-rot] if rot else base)
    v = np.array(verts, dtype=np.float64)
    v *= a / np.linalg.norm(v[0])
    if centre:
        v = np.vstack([v, np.zeros((1, 3))])
    return v


def pair_table(template: np.ndarray):
    """All blob pairs (a < b) of the template with rest lengths |s_b - s_a|.

    Returns (pair_a int32, pair_b int32, rest_len float64); 78 pairs for 13
    blobs."""
    n = template.shape[0]
    pa, pb, r0 = [], [], []
    for i in range(n):
        for j in range(i + 1, n):
            pa.append(i)
            pb.append(j)
            r0.append(float(np.linalg.norm(template[j] - template[i])))
    return (np.array(pa, dtype=np.int32), np.array(pb, dtype=np.int32),
            np.array(r0, dtype=np.float64))


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly random rotation matrices (n, 3, 3) from normalised
    Gaussian quaternions."""
    qt = rng.standard_normal((n, 4))
    qt /= np.linalg.norm(qt, axis=1, keepdims=True)
    w, x, y, z = qt.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def particles_for_fraction(L: float, phi: float,
                           radius: float = EFFECTIVE_RADIUS) -> int:
    """Number of spheres of ``radius`` filling fraction phi of an L^3 box."""
    return int(round(phi * L ** 3 / (4.0 / 3.0 * math.pi * radius ** 3)))


def rsa_centres(rng: np.random.Generator, L: float, n: int,
                dmin: float = 2 * EFFECTIVE_RADIUS,
                max_attempts: int | None = None) -> np.ndarray:
    """Random sequential addition of n centres in a periodic box with
    minimum-image distance >= dmin.

    Candidates are drawn uniformly in batches; candidate i is accepted iff it
    keeps dmin from every centre accepted before it (earlier batches through
    a cell grid whose cells hold at most one centre, earlier members of its
    own batch through a pairwise check), which is exactly sequential
    addition over the candidate stream."""
    ncell = int(math.ceil(L * math.sqrt(3.0) / dmin))
    cs = L / ncell                       # cell diagonal < dmin
    reach = int(math.ceil(dmin / cs))
    rng_off = np.arange(-reach, reach + 1)
    offs = np.stack(np.meshgrid(rng_off, rng_off, rng_off, indexing="ij"),
                    axis=-1).reshape(-1, 3)
    occ = np.full((ncell, ncell, ncell), -1, dtype=np.int64)
    # Fine grid of cells lying wholly within dmin of an accepted centre: a
    # candidate in such a cell is rejected without the exact test.
    nfine = int(math.ceil(L / 0.5))
    g = L / nfine
    blocked = np.zeros((nfine, nfine, nfine), dtype=bool)
    rfine = int(math.ceil(dmin / g)) + 1
    f_off = np.arange(-rfine, rfine + 1)
    f_offs = np.stack(np.meshgrid(f_off, f_off, f_off, indexing="ij"),
                      axis=-1).reshape(-1, 3)
    r_block = dmin - 0.5 * g * math.sqrt(3.0) - 1e-9
    f_offs = f_offs[np.linalg.norm(f_offs, axis=1) * g
                    <= r_block + 2.0 * g * math.sqrt(3.0)]
    out = np.empty((n, 3))
    count = 0
    attempts = 0
    limit = max_attempts if max_attempts is not None else 400 * n + 10000
    d2min = dmin * dmin
    while count < n:
        if attempts > limit:
            raise RuntimeError(f"RSA stalled after {count} of {n} centres")
        B = int(min(2048, max(64, 4 * (n - count))))
        cand = rng.uniform(0.0, L, size=(B, 3))
        attempts += B
        fi = np.floor(cand / g).astype(np.int64) % nfine
        cand = cand[~blocked[fi[:, 0], fi[:, 1], fi[:, 2]]]
        if cand.shape[0] == 0:
            continue
        ci = np.floor(cand / cs).astype(np.int64) % ncell
        nbr = (ci[:, None, :] + offs[None, :, :]) % ncell
        occupant = occ[nbr[..., 0], nbr[..., 1], nbr[..., 2]]
        has = occupant >= 0
        d = out[np.where(has, occupant, 0)] - cand[:, None, :]
        d -= L * np.round(d / L)
        ok = ~(has & ((d * d).sum(-1) < d2min)).any(axis=1)
        idx = np.nonzero(ok)[0]
        if idx.size == 0:
            continue
        C = cand[idx]
        dd = C[:, None, :] - C[None, :, :]
        dd -= L * np.round(dd / L)
        ci_, cj_ = np.nonzero(np.triu((dd * dd).sum(-1) < d2min, 1))
        earlier = [[] for _ in range(idx.size)]
        for i_, j_ in zip(ci_.tolist(), cj_.tolist()):
            earlier[j_].append(i_)
        taken = [False] * idx.size
        accepted = []
        for j in range(idx.size):
            if count + len(accepted) >= n:
                break
            if not any(taken[i_] for i_ in earlier[j]):
                taken[j] = True
                accepted.append(j)
        acc = C[accepted]
        m = acc.shape[0]
        out[count:count + m] = acc
        aci = np.floor(acc / cs).astype(np.int64) % ncell
        occ[aci[:, 0], aci[:, 1], aci[:, 2]] = np.arange(count, count + m)
        base = np.floor(acc / g).astype(np.int64)
        cells = base[:, None, :] + f_offs[None, :, :]
        dc = (cells + 0.5) * g - acc[:, None, :]
        inside = (dc * dc).sum(-1) <= r_block * r_block
        cw = cells[inside] % nfine
        blocked[cw[:, 0], cw[:, 1], cw[:, 2]] = True
        count += m
    return out


def lattice_centres(rng: np.random.Generator, L: float, n: int,
                    dmin: float = 2 * EFFECTIVE_RADIUS) -> np.ndarray:
    """n centres on a random subset of the densest simple-cubic lattice whose
    spacing exceeds dmin, each displaced uniformly within +-(spacing-dmin)/2
    per axis, which keeps every pair at least dmin apart."""
    m = int(L // dmin)
    while m > 0 and L / m < dmin:
        m -= 1
    if m ** 3 < n:
        raise ValueError(f"{n} centres do not fit a {m}^3 lattice")
    spacing = L / m
    pick = rng.choice(m ** 3, size=n, replace=False)
    iz, rem = np.divmod(pick, m * m)
    iy, ix = np.divmod(rem, m)
    c = (np.stack([ix, iy, iz], axis=1) + 0.5) * spacing
    slack = 0.5 * (spacing - dmin) * (1.0 - 1e-9)
    c += rng.uniform(-slack, slack, size=c.shape)
    return c % L


def hard_sphere_centres(rng: np.random.Generator, L: float, n: int, radius: float,
                        sweeps: int = 20, step: float | None = None) -> np.ndarray:
    """Equilibrium hard-sphere configuration of n spheres of ``radius`` in a
    periodic box (the Monte Carlo preparation of the viscosity measurement,
    Sec. Stresslet and Viscosity): random sequential addition (or a lattice
    start when that is too dense for it), then ``sweeps`` Metropolis sweeps
    of single-sphere moves, uniform in +-step per axis, rejected on overlap.
    The step defaults to a fifth of the mean free spacing."""
    dmin = 2.0 * radius
    phi = n * 4.0 / 3.0 * math.pi * radius ** 3 / L ** 3
    c = (rsa_centres(rng, L, n, dmin=dmin) if phi < 0.3
         else lattice_centres(rng, L, n, dmin=dmin))
    if step is None:
        step = 0.2 * max((L ** 3 / max(n, 1)) ** (1.0 / 3.0) - dmin, 0.05 * dmin)
    d2min = dmin * dmin
    for _ in range(sweeps):
        for i in rng.permutation(n):
            trial = (c[i] + rng.uniform(-step, step, size=3)) % L
            d = c - trial
            d -= L * np.round(d / L)
            r2 = (d * d).sum(1)
            r2[i] = np.inf
            if r2.min() >= d2min:
                c[i] = trial
    return c


def place_particles(centres: np.ndarray, template: np.ndarray,
                    rotations: np.ndarray | None = None) -> np.ndarray:
    """Blob positions (P * nb, 3), blob nb*p + b of particle p."""
    s = template if rotations is None else np.einsum("pij,bj->pbi", rotations,
                                                     template)
    if s.ndim == 2:
        s = np.broadcast_to(s, (centres.shape[0],) + s.shape)
    q = centres[:, None, :] + s
    return np.ascontiguousarray(q.reshape(-1, 3))


@dataclass
class Workload:
    """One synthetic workload: grid/fluid parameters, springs and blobs."""
    name: str
    L: int
    h: float
    rho: float
    eta: float
    dt: float
    steps: int
    q: np.ndarray                      # (M, 3) blob positions
    Fext: np.ndarray                   # (P, 3) per-particle external force
    nb: int
    pa: np.ndarray
    pb: np.ndarray
    r0: np.ndarray
    k: float
    template: np.ndarray
    extra: dict = field(default_factory=dict)

    @property
    def P(self) -> int:
        return self.Fext.shape[0]

    @property
    def M(self) -> int:
        return self.q.shape[0]

    def springs(self) -> dict:
        return {"nb": self.nb, "pa": self.pa, "pb": self.pb, "r0": self.r0,
                "k": self.k}


def _make(name, L, centres, rng, rotate, Fext, steps, a=1.0, k=100.0,
          dt=0.01, rho=1.0, eta=1.0, h=1.0, extra=None):
    tmpl = icosahedron_template(a)
    pa, pb, r0 = pair_table(tmpl)
    R = random_rotations(rng, centres.shape[0]) if rotate else None
    q = place_particles(centres, tmpl, R)
    return Workload(name, L, h, rho, eta, dt, steps, q,
                    np.ascontiguousarray(Fext, dtype=np.float64), tmpl.shape[0],
                    pa, pb, r0, k, tmpl, extra or {})


def single(seed: int = 1) -> Workload:
    """One 13-blob particle in a periodic 32^3 box, Fext = (1, 0, 0),
    dt = 0.01, 200 steps."""
    rng = np.random.default_rng(seed)
    L = 32
    c = rng.uniform(0.0, L, size=(1, 3))
    return _make("single", L, c, rng, False, np.array([[1.0, 0.0, 0.0]]), 200)


def dense(seed: int = 2, L: int = 128, phi: float = 0.3,
          n: int | None = None) -> Workload:
    """Dense suspension: 36,669 particles in 128^3 at phi = 0.3 (RSA)."""
    rng = np.random.default_rng(seed)
    P = particles_for_fraction(L, phi) if n is None else n
    c = rsa_centres(rng, float(L), P)
    F = rng.standard_normal((P, 3))
    return _make("dense", L, c, rng, True, F, 1000,
                 extra={"phi": phi})


def large(seed: int = 5, L: int = 256, phi: float = 0.4,
          n: int | None = None, sweeps: int = 20) -> Workload:
    """Large suspension: 391,139 particles in 256^3 at phi = 0.4: a random
    subset of a simple-cubic lattice (random sequential addition jams below
    0.4), then `sweeps` hard-sphere Monte Carlo sweeps (hard_sphere_sweeps)
    with centre distance >= 3.2 h."""
    rng = np.random.default_rng(seed)
    P = particles_for_fraction(L, phi) if n is None else n
    c = lattice_centres(rng, float(L), P)
    start = c.copy()
    free = (L ** 3 / P) ** (1.0 / 3.0) - 2 * EFFECTIVE_RADIUS
    mc = hard_sphere_sweeps(rng, c, float(L), 2 * EFFECTIVE_RADIUS, sweeps, 0.5 * free)
    d = c - start
    d -= L * np.round(d / L)
    F = rng.standard_normal((P, 3))
    return _make("large", L, c, rng, True, F, 100,
                 extra={"phi": phi, "mc_sweeps": sweeps,
                        "mc_acceptance": float(np.mean(mc["acceptance"])),
                        "mc_rms_displacement": float(np.sqrt((d * d).sum(1).mean()))})


def pair(seed: int = 3, L: int = 32, sep: float | None = None) -> Workload:
    """Two particles separated along x, opposite forces +-(1, 0, 0)."""
    rng = np.random.default_rng(seed)
    if sep is None:
        sep = float(rng.uniform(2.0, 6.0))
    mid = np.full(3, L / 2.0)
    c = np.stack([mid - [sep / 2, 0, 0], mid + [sep / 2, 0, 0]])
    F = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    return _make("pair", L, c, rng, False, F, 500, extra={"sep": sep})


def diff(seed: int = 4) -> Workload:
    """Differentiation case: 64^3 box, 16 particles placed by random
    sequential addition, 100 steps of dt = 0.01; per-particle forces N(0, 1)
    (split over the blobs as the initial per-blob forces) and target
    velocities V ~ N(0, 0.1^2) per component (extra["V"]); the centres and
    rotations are in extra so the template can be rescaled."""
    rng = np.random.default_rng(seed)
    c = rsa_centres(rng, 64.0, 16)
    F = rng.standard_normal((16, 3))
    R = random_rotations(rng, 16)
    V = 0.1 * rng.standard_normal((16, 3))
    tmpl = icosahedron_template(1.0)
    pa, pb, r0 = pair_table(tmpl)
    q = place_particles(c, tmpl, R)
    return Workload("diff", 64, 1.0, 1.0, 1.0, 0.01, 100, q, F, tmpl.shape[0], pa, pb, r0,
                    100.0, tmpl, {"centres": c, "rotations": R, "V": V})


def pair_sweep(seed: int = 3, nbox: int = 512, sizes=(24, 32, 48, 64),
               sep_range=(2.0, 6.0), template=None, rotate=False) -> list:
    """Batched pair-mobility sweep: nbox independent periodic boxes with
    edges drawn uniformly from `sizes`, each with two particles separated
    along x by a distance uniform in sep_range, centred in the box, forces
    +-(1, 0, 0), dt = 0.01, 500 steps.  Returns one dict per box with L, q
    (26, 3), Fext (2, 3), sep and the two centres c (2, 3).  The particle is
    `template` (default: the filled icosahedron of circumradius 1), both
    particles of a box in the canonical orientation or, with rotate, in one
    random orientation per box (drawn after the boxes, which stay the
    same)."""
    rng = np.random.default_rng(seed)
    tmpl = icosahedron_template(1.0) if template is None else template
    Ls = rng.choice(np.asarray(sizes), size=nbox)
    seps = rng.uniform(sep_range[0], sep_range[1], size=nbox)
    F = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    boxes = []
    for L, sep in zip(Ls, seps):
        mid = np.full(3, L / 2.0) + rng.uniform(-0.5, 0.5, size=3)
        c = np.stack([mid - [sep / 2, 0, 0], mid + [sep / 2, 0, 0]])
        boxes.append({"L": int(L), "sep": float(sep), "q": place_particles(c, tmpl),
                      "Fext": F.copy(), "c": c})
    if rotate:
        R = random_rotations(rng, nbox)
        for b, Rb in zip(boxes, R):
            b["q"] = place_particles(b["c"], tmpl, np.stack([Rb, Rb]))
    return boxes


def random_suspension(seed: int, L: int, P: int, phi_cap: float = 0.3,
                      rotate: bool = True, spread_box: bool = True) -> Workload:
    """A smaller seeded suspension for parity cases: P particles by RSA."""
    rng = np.random.default_rng(seed)
    c = rsa_centres(rng, float(L), P)
    F = rng.standard_normal((P, 3))
    return _make(f"rsa{L}_{P}", L, c, rng, rotate, F, 1)


def random_blobs(seed: int, M: int, L: int, spread: float = 1.0,
                 offset: float = 0.0) -> np.ndarray:
    """M free blob positions, uniform in [offset, offset + spread * L)^3."""
    rng = np.random.default_rng(seed)
    return offset + rng.uniform(0.0, spread * L, size=(M, 3))


def random_forces(seed: int, M: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((M, 3))


def random_field(seed: int, L: int, scale: float = 1.0) -> np.ndarray:
    """A (3, L, L, L) Gaussian staggered field."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((3, L, L, L))


# Changes whenever a generator changes what it returns (the cache key
# includes it, so no stale file is loaded).
_GENERATOR_VERSION = 2

_GENERATORS = {"single": single, "dense": dense, "large": large, "pair": pair,
               "diff": diff}


def cached(name: str, **kw) -> Workload:
    """A named workload, generated once and kept as .npz under the directory
    in $MB_INPUT_CACHE (default: the system temporary directory).  The file
    holds exactly what the generator returned, so cached and fresh inputs
    are identical."""
    import hashlib
    import os
    import tempfile
    key = hashlib.sha1(repr((name, sorted(kw.items()), _GENERATOR_VERSION)).encode()
                       ).hexdigest()[:16]
    root = os.environ.get("MB_INPUT_CACHE",
                          os.path.join(tempfile.gettempdir(), "mb_input_cache"))
    path = os.path.join(root, f"{name}_{key}.npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        tmpl = z["template"]
        pa, pb, r0 = z["pa"], z["pb"], z["r0"]
        sc = z["scalars"]
        return Workload(name, int(sc[0]), float(sc[1]), float(sc[2]), float(sc[3]),
                        float(sc[4]), int(sc[5]), z["q"], z["Fext"], int(sc[6]),
                        pa, pb, r0, float(sc[7]), tmpl,
                        {k[6:]: (float(z[k]) if z[k].ndim == 0 else z[k])
                         for k in z.files if k.startswith("extra_")})
    w = _GENERATORS[name](**kw)
    os.makedirs(root, exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp.npz"
    np.savez(tmp, q=w.q, Fext=w.Fext, template=w.template, pa=w.pa, pb=w.pb, r0=w.r0,
             scalars=np.array([w.L, w.h, w.rho, w.eta, w.dt, w.steps, w.nb, w.k]),
             **{f"extra_{k}": v for k, v in w.extra.items()})
    os.replace(tmp, path)
    return w


def hard_sphere_sweeps(rng: np.random.Generator, c: np.ndarray, L: float, dmin: float,
                       sweeps: int, step: float, target_accept: float = 0.4) -> dict:
    """Hard-sphere Monte Carlo on the centres c (n, 3) in place: `sweeps`
    sweeps of single-sphere displacements, uniform in +-step per axis,
    rejected on overlap (minimum-image distance < dmin), as in the Monte
    Carlo preparation of Sec. Stresslet and Viscosity.  Vectorised by a
    checkerboard of cells of side >= dmin + 2 step (an even number per
    axis): in each sub-step one random sphere of every occupied cell of one
    of the 8 parity classes moves; spheres of same-class cells are at least
    dmin + 2 step apart along some axis, so their moves cannot conflict, and
    each trial position is checked against the current centres (a periodic
    k-d tree: only the mover itself may lie within dmin).  A sweep is as
    many attempts as spheres.  The step is scaled after each sweep towards
    `target_accept`.  Returns the acceptance per sweep and the final step."""
    from scipy.spatial import cKDTree
    n = c.shape[0]
    accept_hist = []
    for _ in range(sweeps):
        ncell = int(L // (dmin + 2.0 * step))
        ncell -= ncell % 2
        if ncell < 4:
            raise ValueError("box too small for the checkerboard")
        cs = L / ncell
        attempts = accepted = 0
        while attempts < n:
            for cls in rng.permutation(8):
                ci = np.floor(c / cs).astype(np.int64) % ncell
                par = (ci[:, 0] & 1) | ((ci[:, 1] & 1) << 1) | ((ci[:, 2] & 1) << 2)
                members = np.nonzero(par == cls)[0]
                if members.size == 0:
                    continue
                members = members[rng.permutation(members.size)]
                cid = (ci[members, 2] * ncell + ci[members, 1]) * ncell + ci[members, 0]
                _, first = np.unique(cid, return_index=True)
                mover = members[first]  # one random sphere per occupied cell
                trial = (c[mover] + rng.uniform(-step, step, size=(mover.size, 3))) % L
                tree = cKDTree(c % L, boxsize=L, balanced_tree=False, compact_nodes=False)
                near = tree.query_ball_point(trial, dmin * (1.0 - 1e-12), return_length=True)
                ok = near <= 1  # the mover itself (within sqrt(3) step < dmin)
                c[mover[ok]] = trial[ok]
                attempts += mover.size
                accepted += int(ok.sum())
                if attempts >= n:
                    break
        rate = accepted / max(attempts, 1)
        accept_hist.append(rate)
        step *= min(2.0, max(0.5, rate / target_accept))
    return {"acceptance": accept_hist, "step": step}
