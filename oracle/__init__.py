"""The oracle: a plain FP64 CPU implementation of the multiblob step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with the GPU library (``paper_1407_5600_amd``) and never imports it.

Thin numpy/ctypes wrappers around ``mbo.c``; each function's docstring names
the passage of Vazquez-Quesada, Balboa Usabiaga & Delgado-Buscalioni,
arXiv:1407.5600, that it follows.  Arrays are float64, C-contiguous:
positions/forces (M, 3), staggered fields (3, L, L, L) with x fastest.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


class Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int),
        ("h", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("steady", ctypes.c_int),
        ("zero_mean", ctypes.c_int),
    ]


def lib():
    """Load liboracle.so, building it first if it is absent."""
    global _lib
    if _lib is None:
        path = os.environ.get("MBO_ORACLE_LIB", _build.LIB)
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        _lib = ctypes.CDLL(path)
        d = ctypes.c_double
        _lib.mbo_phi.restype = d
        _lib.mbo_phi.argtypes = [d]
        _lib.mbo_phi_deriv.restype = d
        _lib.mbo_phi_deriv.argtypes = [d]
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def params(L, h=1.0, rho=1.0, eta=1.0, dt=0.01, steady=False, zero_mean=False):
    return Params(int(L), float(h), float(rho), float(eta), float(dt),
                  int(bool(steady)), int(bool(zero_mean)))


def phi(r):
    """3-point kernel Phi (eq. delta), r in units of h."""
    return lib().mbo_phi(float(r))


def spread(prm, q, F):
    """Force density f = sum_i S_i F_i on the staggered grid (S_i = J_i^*)."""
    q = _f64(q)
    F = _f64(F)
    M = q.shape[0]
    f = np.zeros((3, prm.L, prm.L, prm.L))
    lib().mbo_spread(ctypes.byref(prm), ctypes.c_long(M), _p(q), _p(F), _p(f))
    return f


def interpolate(prm, q, v):
    """Blob velocities u_i = J_i v (eq. ju, lattice sum)."""
    q = _f64(q)
    v = _f64(v)
    M = q.shape[0]
    u = np.zeros((M, 3))
    lib().mbo_interpolate(ctypes.byref(prm), ctypes.c_long(M), _p(q), _p(v),
                          _p(u))
    return u


def spring_forces(P, nb, pa, pb, r0, k, q, Fext):
    """Harmonic springs of each particle plus Fext/nb per blob (Fig. 1)."""
    pa = np.ascontiguousarray(pa, dtype=np.int32)
    pb = np.ascontiguousarray(pb, dtype=np.int32)
    r0 = _f64(r0)
    q = _f64(q)
    F = np.zeros((P * nb, 3))
    fe = None if Fext is None else _f64(Fext)
    lib().mbo_spring_forces(ctypes.c_long(P), ctypes.c_int(nb),
                            ctypes.c_int(len(pa)), _p(pa), _p(pb), _p(r0),
                            ctypes.c_double(k), _p(q),
                            None if fe is None else _p(fe), _p(F))
    return F


def fft(x, sign=-1):
    """1-D DFT by recursive mixed-radix Cooley-Tukey (complex128 in/out)."""
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    lib().mbo_fft(ctypes.c_int(a.shape[0]), _p(a), ctypes.c_long(1),
                  ctypes.c_int(sign))
    return a


def dft(x, sign=-1):
    """Direct O(n^2) DFT."""
    a = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.zeros_like(a)
    lib().mbo_dft(ctypes.c_int(a.shape[0]), _p(a), _p(out), ctypes.c_int(sign))
    return out


def fft3(x, sign=-1):
    """3-D DFT of an (L, L, L) complex array (axis 2 = x fastest)."""
    a = np.ascontiguousarray(x, dtype=np.complex128).copy()
    lib().mbo_fft3(ctypes.c_int(a.shape[0]), _p(a), ctypes.c_int(sign))
    return a


def divergence(prm, v):
    """Cell-centred discrete divergence of a staggered field."""
    v = _f64(v)
    out = np.zeros((prm.L, prm.L, prm.L))
    lib().mbo_divergence(ctypes.byref(prm), _p(v), _p(out))
    return out


def fluid_solve(prm, v, f):
    """One fluid solve of eq. vf (Crank-Nicolson or steady Stokes) with the
    solenoidal projection, exact in Fourier space on the MAC grid."""
    v = _f64(v)
    f = _f64(f)
    out = np.zeros((3, prm.L, prm.L, prm.L))
    lib().mbo_fluid_solve(ctypes.byref(prm), _p(v), _p(f), _p(out))
    return out


def step(prm, springs, q, v, Fext, nsteps=1, f_fluid=None, scheme="euler"):
    """Run ``nsteps`` time steps in place on copies of q and v.

    springs: dict with keys nb, pa, pb, r0, k.  f_fluid: optional force
    density (3, L, L, L) on the fluid added to the spread blob forces in
    every step (the periodic forcing of Sec. Stresslet and Viscosity).
    scheme: "euler" (first order: force and interpolation at q^n) or
    "midpoint" (the second-order predictor-corrector, mbo_step_midpoint).
    Returns a dict with the new q, v and the last step's u, U0 and
    diagnostics {Pi_x, Pi_y, Pi_z, sumF_x, sumF_y, sumF_z, max|Dv|}.
    """
    q = _f64(q).copy()
    v = _f64(v).copy()
    Fext = _f64(Fext)
    nb = int(springs["nb"])
    P = q.shape[0] // nb
    pa = np.ascontiguousarray(springs["pa"], dtype=np.int32)
    pb = np.ascontiguousarray(springs["pb"], dtype=np.int32)
    r0 = _f64(springs["r0"])
    u = np.zeros_like(q)
    U0 = np.zeros((P, 3))
    diag = np.zeros(7)
    ff = None if f_fluid is None else _f64(f_fluid, (3, prm.L, prm.L, prm.L))
    fn = {"euler": lib().mbo_step_forced, "midpoint": lib().mbo_step_midpoint}[scheme]
    fn(ctypes.byref(prm), ctypes.c_long(P), ctypes.c_int(nb), ctypes.c_int(len(pa)),
       _p(pa), _p(pb), _p(r0), ctypes.c_double(springs["k"]), _p(q), _p(v), _p(Fext),
       None if ff is None else _p(ff), _p(u), _p(U0), ctypes.c_int(nsteps), _p(diag))
    return {"q": q, "v": v, "u": u, "U0": U0, "diag": diag}


# ---- derivatives (reverse mode) -------------------------------------------

def phi_deriv(r):
    """Phi'(r) of the 3-point kernel (eq. delta is C^1)."""
    return lib().mbo_phi_deriv(float(r))


def interpolate_grad(prm, q, v, W):
    """sum_a W_{i,a} grad_{q_i} (J_i v)_a per blob (M, 3): the derivative of
    the interpolation of eq. ju with respect to the blob positions."""
    q = _f64(q)
    v = _f64(v)
    W = _f64(W)
    g = np.zeros_like(q)
    lib().mbo_interpolate_grad(ctypes.byref(prm), ctypes.c_long(q.shape[0]), _p(q),
                               _p(v), _p(W), _p(g))
    return g


def spring_adjoint(P, nb, pa, pb, r0, k, q, Fbar):
    """(dF/dq)^T Fbar, Fbar . dF/dk and Fbar . dF/dr0 of the spring forces
    (Fig. 1 springs, Fext excluded).  Returns (qbar (M, 3), kbar, r0bar)."""
    pa = np.ascontiguousarray(pa, dtype=np.int32)
    pb = np.ascontiguousarray(pb, dtype=np.int32)
    r0 = _f64(r0)
    q = _f64(q)
    Fbar = _f64(Fbar)
    qbar = np.zeros_like(q)
    kbar = ctypes.c_double(0.0)
    r0bar = np.zeros(len(pa))
    lib().mbo_spring_adjoint(ctypes.c_long(P), ctypes.c_int(nb), ctypes.c_int(len(pa)),
                             _p(pa), _p(pb), _p(r0), ctypes.c_double(k), _p(q),
                             _p(Fbar), _p(qbar), ctypes.byref(kbar), _p(r0bar))
    return qbar, kbar.value, r0bar


def loss_grad(prm, springs, q0, v0, G, V, nsteps):
    """Loss sum_p |U_p - V_p|^2 of an nsteps trajectory (per-blob external
    forces G (M, 3); U_p the mean blob velocity of particle p in the last
    step) and its gradients by the reverse sweep.  Returns (loss, dict with
    q0, v0, G, k, r0)."""
    q0 = _f64(q0)
    v0 = _f64(v0)
    G = _f64(G)
    V = _f64(V)
    nb = int(springs["nb"])
    P = q0.shape[0] // nb
    pa = np.ascontiguousarray(springs["pa"], dtype=np.int32)
    pb = np.ascontiguousarray(springs["pb"], dtype=np.int32)
    r0 = _f64(springs["r0"])
    loss = ctypes.c_double(0.0)
    kbar = ctypes.c_double(0.0)
    qbar = np.zeros_like(q0)
    vbar = np.zeros_like(v0)
    Gbar = np.zeros_like(G)
    r0bar = np.zeros(len(pa))
    lib().mbo_loss_grad(ctypes.byref(prm), ctypes.c_long(P), ctypes.c_int(nb),
                        ctypes.c_int(len(pa)), _p(pa), _p(pb), _p(r0),
                        ctypes.c_double(springs["k"]), _p(q0), _p(v0), _p(G), _p(V),
                        ctypes.c_int(nsteps), ctypes.byref(loss), _p(qbar), _p(vbar),
                        _p(Gbar), ctypes.byref(kbar), _p(r0bar))
    return loss.value, {"q0": qbar, "v0": vbar, "G": Gbar, "k": kbar.value, "r0": r0bar}

