"""ctypes binding of libmultiblob.so (the C ABI in include/multiblob.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Tensors are torch tensors on the library's device; the binding
checks dtype, device, shape and contiguity, then passes raw pointers and the
current HIP stream.  Loading fails loudly if the shared library is missing.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmultiblob.so")

MB_OK, MB_ERR_INVALID, MB_ERR_UNSUPPORTED, MB_ERR_NOMEM, MB_ERR_DEVICE = 0, -1, -2, -3, -4
MB_ERR_NONFINITE = -5
MB_FP64, MB_MIXED = 0, 1
MB_UNSTEADY_CN, MB_STEADY_STOKES = 0, 1
MB_SCHEME_EULER, MB_SCHEME_MIDPOINT = 0, 1
SCHEMES = {"euler": MB_SCHEME_EULER, "midpoint": MB_SCHEME_MIDPOINT}
NDIAG = 7


class MultiblobError(RuntimeError):
    def __init__(self, status: int, call: str):
        self.status = status
        super().__init__(f"{call}: {status_string(status)} ({status})")


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("zero_mean", ctypes.c_int32),
        ("h", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("max_blobs", ctypes.c_int64),
        ("deterministic", ctypes.c_int32),
        ("check_finite", ctypes.c_int32),
        ("external_workspace", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python paper_1407_5600_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "mb_grid_create": ([ctypes.POINTER(GridDesc), ctypes.POINTER(vp)], i32),
            "mb_grid_create_batch": ([ctypes.POINTER(GridDesc), i32, ctypes.POINTER(vp)], i32),
            "mb_step_graph": ([i32, vp, vp, vp, vp, vp, vp, vp, i32, vp], i32),
            "mb_grid_destroy": ([vp], i32),
            "mb_workspace_size": ([ctypes.POINTER(GridDesc), i32], ctypes.c_size_t),
            "mb_grid_set_workspace": ([vp, vp, ctypes.c_size_t], i32),
            "mb_springs_set_params": ([vp, vp, d, vp], i32),
            "mb_step_noalloc": ([ctypes.POINTER(GridDesc), vp, i64, vp, vp, vp, vp, vp, vp, i32,
                                 vp], i32),
            "mb_springs_create": ([i32, i32, vp, vp, vp, d, ctypes.POINTER(vp)], i32),
            "mb_springs_destroy": ([vp], i32),
            "mb_spread": ([vp, i64, vp, vp, vp, vp], i32),
            "mb_interpolate": ([vp, i64, vp, vp, vp, vp], i32),
            "mb_fluid_solve": ([vp, vp, vp, vp, vp], i32),
            "mb_spring_forces": ([vp, i64, vp, vp, vp, vp], i32),
            "mb_step": ([vp, vp, i64, vp, vp, vp, vp, vp, vp, i32, vp], i32),
            "mb_step_ext": ([vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, i32, vp], i32),
            "mb_step_forced": ([vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp], i32),
            "mb_spring_forces_ext": ([vp, i64, vp, vp, vp, vp, vp], i32),
            "mb_interpolate_grad": ([vp, i64, vp, vp, vp, vp, vp], i32),
            "mb_spring_adjoint": ([vp, i64, vp, vp, vp, vp, vp, vp], i32),
            "mb_step_adjoint": ([vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
                                i32),
            "mb_status_string": ([i32], ctypes.c_char_p),
            "mb_grid_set_timing": ([vp, ctypes.c_uint32], i32),
            "mb_grid_set_scheme": ([vp, i32], i32),
            "mb_grid_set_tiles": ([vp, i32, i32, i32], i32),
            "mb_grid_get_tiles": ([vp, vp], i32),
            "mb_grid_autotune": ([vp, vp, i64, vp, vp, vp, i32, vp, vp], i32),
            "mb_grid_kernel_times": ([vp, vp, vp, vp, i32, ctypes.POINTER(i32)], i32),
            "mb_kernel_name": ([i32], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


EXPORTED = ("mb_grid_create", "mb_grid_destroy", "mb_springs_create",
            "mb_springs_destroy", "mb_spread", "mb_interpolate", "mb_fluid_solve",
            "mb_spring_forces", "mb_step", "mb_status_string", "mb_grid_set_timing",
            "mb_grid_kernel_times", "mb_kernel_name", "mb_step_ext", "mb_spring_forces_ext",
            "mb_interpolate_grad", "mb_spring_adjoint", "mb_step_adjoint",
            "mb_grid_create_batch", "mb_step_graph", "mb_step_forced",
            "mb_grid_set_scheme", "mb_grid_set_tiles", "mb_grid_get_tiles",
            "mb_grid_autotune", "mb_workspace_size", "mb_grid_set_workspace",
            "mb_springs_set_params", "mb_step_noalloc")


def status_string(st: int) -> str:
    return lib().mb_status_string(int(st)).decode()


def _check(st: int, call: str):
    if st != MB_OK:
        raise MultiblobError(st, call)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, shape=None, name="tensor", device=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on {t.device}, the grid on cuda:{device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Springs:
    """Spring table of one particle template (mb_springs_create)."""

    def __init__(self, nb, pair_a, pair_b, rest_len, k):
        import numpy as np
        pa = np.ascontiguousarray(pair_a, dtype=np.int32)
        pb = np.ascontiguousarray(pair_b, dtype=np.int32)
        r0 = np.ascontiguousarray(rest_len, dtype=np.float64)
        if not (len(pa) == len(pb) == len(r0)):
            raise ValueError("pair arrays differ in length")
        h = ctypes.c_void_p()
        _check(lib().mb_springs_create(int(nb), len(pa), pa.ctypes.data_as(ctypes.c_void_p),
                                       pb.ctypes.data_as(ctypes.c_void_p),
                                       r0.ctypes.data_as(ctypes.c_void_p), float(k),
                                       ctypes.byref(h)), "mb_springs_create")
        self.handle = h
        self.nb = int(nb)
        self.npairs = len(pa)
        self.k = float(k)

    def set_params(self, rest_len, k, stream=None):
        """mb_springs_set_params: new rest lengths (host values, copied in
        stream order) and stiffness for the later calls."""
        import numpy as np
        r0 = np.ascontiguousarray(rest_len, dtype=np.float64)
        if r0.shape != (self.npairs,):
            raise ValueError(f"rest_len must have shape ({self.npairs},)")
        _check(lib().mb_springs_set_params(self.handle, r0.ctypes.data_as(ctypes.c_void_p),
                                           float(k), _stream(stream)),
               "mb_springs_set_params")
        self._r0_keep = r0  # the copy may still read it
        self.k = float(k)

    def close(self):
        if self.handle:
            lib().mb_springs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Grid:
    """A periodic MAC grid with its FFT tables and scratch (mb_grid_create)."""

    def __init__(self, L, h=1.0, rho=1.0, eta=1.0, dt=0.01, precision="fp64",
                 mode="unsteady", zero_mean=False, max_blobs=0, nbox=1, scheme="euler",
                 deterministic=False, check_finite=False, workspace=None):
        """workspace: None (the library allocates the grid's scratch),
        "torch" (a torch uint8 tensor of mb_workspace_size bytes, allocated
        here and kept by this object), or such a tensor of the caller's."""
        import torch
        prec = {"fp64": MB_FP64, "mixed": MB_MIXED}[precision]
        md = {"unsteady": MB_UNSTEADY_CN, "steady": MB_STEADY_STOKES}[mode]
        self.desc = GridDesc(int(L), prec, md, int(bool(zero_mean)), float(h), float(rho),
                             float(eta), float(dt), int(max_blobs), int(bool(deterministic)),
                             int(bool(check_finite)), int(workspace is not None), 0)
        h_ = ctypes.c_void_p()
        if nbox == 1:
            _check(lib().mb_grid_create(ctypes.byref(self.desc), ctypes.byref(h_)),
                   "mb_grid_create")
        else:
            _check(lib().mb_grid_create_batch(ctypes.byref(self.desc), int(nbox),
                                              ctypes.byref(h_)), "mb_grid_create_batch")
        self.handle = h_
        self.nbox = int(nbox)
        self.L = int(L)
        self.precision = precision
        self.field_dtype = torch.float64 if prec == MB_FP64 else torch.float32
        self.device = torch.cuda.current_device()
        self.scheme = "euler"
        self.workspace = None
        if workspace is not None:
            self.set_workspace(None if isinstance(workspace, str) else workspace)
        if scheme != "euler":
            self.set_scheme(scheme)

    def workspace_size(self):
        """mb_workspace_size of this grid's description and box count."""
        return int(lib().mb_workspace_size(ctypes.byref(self.desc), self.nbox))

    def set_workspace(self, buf=None):
        """mb_grid_set_workspace: the grid's scratch in a torch uint8 tensor
        (allocated here when buf is None), kept alive by this object."""
        import torch
        n = self.workspace_size()
        if buf is None:
            buf = torch.empty(n, dtype=torch.uint8, device=torch.device("cuda", self.device))
        if not (isinstance(buf, torch.Tensor) and buf.is_cuda and buf.is_contiguous()):
            raise ValueError("workspace must be a contiguous GPU tensor")
        nbytes = buf.numel() * buf.element_size()
        _check(lib().mb_grid_set_workspace(self.handle, ctypes.c_void_p(buf.data_ptr()), nbytes),
               "mb_grid_set_workspace")
        self.workspace = buf

    @property
    def tiles(self):
        """Tile shape (tx, ty, tz) of the binning, spreading and interpolation."""
        out = (ctypes.c_int32 * 3)()
        _check(lib().mb_grid_get_tiles(self.handle, out), "mb_grid_get_tiles")
        return tuple(out)

    def set_tiles(self, tx, ty, tz):
        """mb_grid_set_tiles."""
        _check(lib().mb_grid_set_tiles(self.handle, int(tx), int(ty), int(tz)),
               "mb_grid_set_tiles")

    def autotune(self, springs, q, v, Fext=None, nsteps=10, stream=None):
        """mb_grid_autotune: time every tile shape on copies of (q, v), keep
        the fastest; returns it."""
        import torch
        M = q.shape[0]
        P = M // springs.nb
        out = (ctypes.c_int32 * 3)()
        _check(lib().mb_grid_autotune(
            self.handle, springs.handle, P, _ptr(q, torch.float64, (M, 3), "q", self.device),
            self._fptr(v, "v"), _ptr(Fext, torch.float64, (P, 3), "Fext", self.device),
            int(nsteps), _stream(stream), out), "mb_grid_autotune")
        return tuple(out)

    def set_scheme(self, scheme):
        """mb_grid_set_scheme: "euler" (first order) or "midpoint" (second)."""
        _check(lib().mb_grid_set_scheme(self.handle, SCHEMES[scheme]), "mb_grid_set_scheme")
        self.scheme = scheme

    def close(self):
        if self.handle:
            lib().mb_grid_destroy(self.handle)
            self.handle = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers --------------------------------------------------------
    @property
    def field_shape(self):
        """(3, L, L, L), or (nbox, 3, L, L, L) for a batch of boxes."""
        s = (3, self.L, self.L, self.L)
        return s if self.nbox == 1 else (self.nbox,) + s

    def field(self, zero=True):
        import torch
        dev = torch.device("cuda", self.device)
        return (torch.zeros if zero else torch.empty)(self.field_shape, dtype=self.field_dtype,
                                                      device=dev)

    def _fptr(self, t, name):
        return _ptr(t, self.field_dtype, self.field_shape, name, self.device)

    # -- calls ----------------------------------------------------------
    def spread(self, q, F, f_out=None, stream=None):
        import torch
        M = q.shape[0]
        f_out = self.field(zero=False) if f_out is None else f_out
        _check(lib().mb_spread(self.handle, M, _ptr(q, torch.float64, (M, 3), "q", self.device),
                               _ptr(F, torch.float64, (M, 3), "F", self.device),
                               self._fptr(f_out, "f_out"), _stream(stream)), "mb_spread")
        return f_out

    def interpolate(self, q, v, u_out=None, stream=None):
        import torch
        M = q.shape[0]
        if u_out is None:
            u_out = torch.empty((M, 3), dtype=torch.float64, device=q.device)
        _check(lib().mb_interpolate(self.handle, M, _ptr(q, torch.float64, (M, 3), "q", self.device),
                                    self._fptr(v, "v"),
                                    _ptr(u_out, torch.float64, (M, 3), "u_out", self.device),
                                    _stream(stream)), "mb_interpolate")
        return u_out

    def fluid_solve(self, v_in, f, v_out=None, stream=None):
        v_out = self.field(zero=False) if v_out is None else v_out
        vin = None if v_in is None else self._fptr(v_in, "v_in")
        _check(lib().mb_fluid_solve(self.handle, vin, self._fptr(f, "f"),
                                    self._fptr(v_out, "v_out"), _stream(stream)),
               "mb_fluid_solve")
        return v_out

    def step(self, springs, q, v, Fext, nsteps=1, u_out=None, U0_out=None,
             diag_out=None, stream=None):
        import torch
        M = q.shape[0]
        P = M // springs.nb
        if P * springs.nb != M:
            raise ValueError("blob count is not a multiple of blobs per particle")
        _check(lib().mb_step(
            self.handle, springs.handle, P,
            _ptr(q, torch.float64, (M, 3), "q", self.device), self._fptr(v, "v"),
            _ptr(Fext, torch.float64, (P, 3), "Fext", self.device),
            _ptr(u_out, torch.float64, (M, 3), "u_out", self.device),
            _ptr(U0_out, torch.float64, (P, 3), "U0_out", self.device),
            _ptr(diag_out, torch.float64, (NDIAG,), "diag_out", self.device),
            int(nsteps), _stream(stream)), "mb_step")

    def step_ext(self, springs, q, v, Fext=None, F_blob=None, nsteps=1, u_out=None,
                 U0_out=None, diag_out=None, stream=None):
        """mb_step_ext: mb_step with optional per-blob external forces."""
        import torch
        M = q.shape[0]
        P = M // springs.nb
        if P * springs.nb != M:
            raise ValueError("blob count is not a multiple of blobs per particle")
        _check(lib().mb_step_ext(
            self.handle, springs.handle, P,
            _ptr(q, torch.float64, (M, 3), "q", self.device), self._fptr(v, "v"),
            _ptr(Fext, torch.float64, (P, 3), "Fext", self.device),
            _ptr(F_blob, torch.float64, (M, 3), "F_blob", self.device),
            _ptr(u_out, torch.float64, (M, 3), "u_out", self.device),
            _ptr(U0_out, torch.float64, (P, 3), "U0_out", self.device),
            _ptr(diag_out, torch.float64, (NDIAG,), "diag_out", self.device),
            int(nsteps), _stream(stream)), "mb_step_ext")

    def step_forced(self, springs, q, v, f_fluid, Fext=None, F_blob=None, nsteps=1,
                    u_out=None, U0_out=None, diag_out=None, stream=None):
        """mb_step_forced: mb_step_ext with a force density f_fluid on the fluid."""
        import torch
        M = q.shape[0]
        P = M // springs.nb
        if P * springs.nb != M:
            raise ValueError("blob count is not a multiple of blobs per particle")
        if f_fluid is None:
            raise ValueError("f_fluid is required")
        _check(lib().mb_step_forced(
            self.handle, springs.handle, P,
            _ptr(q, torch.float64, (M, 3), "q", self.device), self._fptr(v, "v"),
            _ptr(Fext, torch.float64, (P, 3), "Fext", self.device),
            _ptr(F_blob, torch.float64, (M, 3), "F_blob", self.device),
            self._fptr(f_fluid, "f_fluid"),
            _ptr(u_out, torch.float64, (M, 3), "u_out", self.device),
            _ptr(U0_out, torch.float64, (P, 3), "U0_out", self.device),
            _ptr(diag_out, torch.float64, (NDIAG,), "diag_out", self.device),
            int(nsteps), _stream(stream)), "mb_step_forced")

    def interpolate_grad(self, q, v, W, g_inout=None, stream=None):
        """mb_interpolate_grad: g += sum_a W_a grad_q (J v)_a (accumulates)."""
        import torch
        M = q.shape[0]
        if g_inout is None:
            g_inout = torch.zeros((M, 3), dtype=torch.float64, device=q.device)
        _check(lib().mb_interpolate_grad(
            self.handle, M, _ptr(q, torch.float64, (M, 3), "q", self.device),
            self._fptr(v, "v"), _ptr(W, torch.float64, (M, 3), "W", self.device),
            _ptr(g_inout, torch.float64, (M, 3), "g", self.device), _stream(stream)),
            "mb_interpolate_grad")
        return g_inout

    def step_adjoint(self, springs, q_n, v_np1, qbar, vbar, Fext=None, F_blob=None,
                     ubar_loss=None, Fblob_bar=None, kbar=None, r0bar=None, stream=None):
        """mb_step_adjoint: reverse one step (qbar, vbar updated in place;
        Fblob_bar, kbar, r0bar accumulated)."""
        import torch
        M = q_n.shape[0]
        P = M // springs.nb
        f64 = torch.float64
        _check(lib().mb_step_adjoint(
            self.handle, springs.handle, P, _ptr(q_n, f64, (M, 3), "q_n", self.device),
            self._fptr(v_np1, "v_np1"), _ptr(Fext, f64, (P, 3), "Fext", self.device),
            _ptr(F_blob, f64, (M, 3), "F_blob", self.device),
            _ptr(ubar_loss, f64, (M, 3), "ubar_loss", self.device),
            _ptr(qbar, f64, (M, 3), "qbar", self.device), self._fptr(vbar, "vbar"),
            _ptr(Fblob_bar, f64, (M, 3), "Fblob_bar", self.device),
            _ptr(kbar, f64, (1,), "kbar", self.device),
            _ptr(r0bar, f64, (springs.npairs,), "r0bar", self.device),
            _stream(stream)), "mb_step_adjoint")

    # -- timing ---------------------------------------------------------
    def set_timing(self, kernels=None):
        """Time the named kernels (None: none, "all": every kernel)."""
        if kernels is None:
            mask = 0
        elif kernels == "all":
            mask = 0xFFFFFFFF
        else:
            names = kernel_names()
            mask = 0
            for k in kernels:
                mask |= 1 << names.index(k)
        _check(lib().mb_grid_set_timing(self.handle, mask), "mb_grid_set_timing")

    def kernel_times(self, stream=None):
        """{kernel name: (total ms, launches)} since timing was enabled."""
        cap = 64
        ms = (ctypes.c_double * cap)()
        n = (ctypes.c_int64 * cap)()
        cnt = ctypes.c_int32()
        _check(lib().mb_grid_kernel_times(self.handle, _stream(stream), ms, n, cap,
                                          ctypes.byref(cnt)), "mb_grid_kernel_times")
        out = {}
        for i in range(cnt.value):
            if n[i]:
                out[lib().mb_kernel_name(i).decode()] = (ms[i], n[i])
        return out


def spring_forces(springs, q, Fext, F_out=None, stream=None, F_blob=None):
    """mb_spring_forces (mb_spring_forces_ext with F_blob): spring forces
    plus Fext/nb (plus F_blob) per blob."""
    import torch
    M = q.shape[0]
    P = M // springs.nb
    if F_out is None:
        F_out = torch.empty((M, 3), dtype=torch.float64, device=q.device)
    if F_blob is None:
        _check(lib().mb_spring_forces(springs.handle, P, _ptr(q, torch.float64, (M, 3), "q"),
                                      _ptr(Fext, torch.float64, (P, 3), "Fext"),
                                      _ptr(F_out, torch.float64, (M, 3), "F_out"),
                                      _stream(stream)), "mb_spring_forces")
    else:
        _check(lib().mb_spring_forces_ext(springs.handle, P,
                                          _ptr(q, torch.float64, (M, 3), "q"),
                                          _ptr(Fext, torch.float64, (P, 3), "Fext"),
                                          _ptr(F_blob, torch.float64, (M, 3), "F_blob"),
                                          _ptr(F_out, torch.float64, (M, 3), "F_out"),
                                          _stream(stream)), "mb_spring_forces_ext")
    return F_out


def spring_adjoint(springs, q, Fbar, qbar, kbar=None, r0bar=None, stream=None):
    """mb_spring_adjoint: qbar += (dF/dq)^T Fbar; kbar (1,), r0bar (npairs,)
    accumulate the stiffness and rest-length parts (may be None)."""
    import torch
    M = q.shape[0]
    P = M // springs.nb
    f64 = torch.float64
    _check(lib().mb_spring_adjoint(springs.handle, P, _ptr(q, f64, (M, 3), "q"),
                                   _ptr(Fbar, f64, (M, 3), "Fbar"),
                                   _ptr(qbar, f64, (M, 3), "qbar"),
                                   _ptr(kbar, f64, (1,), "kbar"),
                                   _ptr(r0bar, f64, (springs.npairs,), "r0bar"),
                                   _stream(stream)), "mb_spring_adjoint")
    return qbar


def step_graph(grids, springs, qs, vs, Fexts=None, F_blobs=None, nsteps=1, stream=None):
    """mb_step_graph: nsteps steps of several grids, one step of each captured
    into a HIP graph and replayed (returns when done)."""
    import torch
    n = len(grids)
    G = (ctypes.c_void_p * n)(*[g.handle.value for g in grids])
    S = (ctypes.c_void_p * n)(*[sp.handle.value for sp in springs])
    P = (ctypes.c_int64 * n)(*[q.shape[0] // sp.nb for q, sp in zip(qs, springs)])
    f64 = torch.float64
    Q = (ctypes.c_void_p * n)(*[_ptr(q, f64, (q.shape[0], 3), "q", g.device).value
                                for q, g in zip(qs, grids)])
    V = (ctypes.c_void_p * n)(*[g._fptr(v, "v").value for v, g in zip(vs, grids)])

    def opt(ts, shape_of, name):
        if ts is None:
            return None
        return (ctypes.c_void_p * n)(*[None if t is None else
                                       _ptr(t, f64, shape_of(i), name, grids[i].device).value
                                       for i, t in enumerate(ts)])
    FE = opt(Fexts, lambda i: (P[i], 3), "Fext")
    FB = opt(F_blobs, lambda i: (qs[i].shape[0], 3), "F_blob")
    _check(lib().mb_step_graph(n, G, S, P, Q, V, FE, FB, int(nsteps), _stream(stream)),
           "mb_step_graph")


NOALLOC_SCRATCH_BYTES = 32 << 20  # MB_NOALLOC_SCRATCH_BYTES


def step_noalloc(springs, q, v, Fext, nsteps=1, u_out=None, U0_out=None, diag_out=None,
                 stream=None, L=None, h=1.0, rho=1.0, eta=1.0, dt=0.01, precision="fp64",
                 mode="unsteady", zero_mean=False, deterministic=False, check_finite=False):
    """mb_step_noalloc: nsteps first-order steps of a grid of these
    parameters (max_blobs = the blob count) whose workspace is the library's
    static device array: the call allocates nothing."""
    import torch
    M = q.shape[0]
    P = M // springs.nb
    if P * springs.nb != M:
        raise ValueError("blob count is not a multiple of blobs per particle")
    prec = {"fp64": MB_FP64, "mixed": MB_MIXED}[precision]
    md = {"unsteady": MB_UNSTEADY_CN, "steady": MB_STEADY_STOKES}[mode]
    desc = GridDesc(int(L), prec, md, int(bool(zero_mean)), float(h), float(rho), float(eta),
                    float(dt), int(M), int(bool(deterministic)), int(bool(check_finite)), 0, 0)
    fdt = torch.float64 if prec == MB_FP64 else torch.float32
    f64 = torch.float64
    _check(lib().mb_step_noalloc(
        ctypes.byref(desc), springs.handle, P, _ptr(q, f64, (M, 3), "q"),
        _ptr(v, fdt, (3, L, L, L), "v"), _ptr(Fext, f64, (P, 3), "Fext"),
        _ptr(u_out, f64, (M, 3), "u_out"), _ptr(U0_out, f64, (P, 3), "U0_out"),
        _ptr(diag_out, f64, (NDIAG,), "diag_out"), int(nsteps), _stream(stream)),
        "mb_step_noalloc")


def kernel_names():
    out = []
    i = 0
    while True:
        n = lib().mb_kernel_name(i)
        if n is None:
            return out
        out.append(n.decode())
        i += 1


# C-ABI names, for callers that prefer them.
def mb_spread(grid, q, F, f_out=None, stream=None):
    return grid.spread(q, F, f_out, stream)


def mb_interpolate(grid, q, v, u_out=None, stream=None):
    return grid.interpolate(q, v, u_out, stream)


def mb_fluid_solve(grid, v_in, f, v_out=None, stream=None):
    return grid.fluid_solve(v_in, f, v_out, stream)


def mb_spring_forces(springs, q, Fext, F_out=None, stream=None):
    return spring_forces(springs, q, Fext, F_out, stream)


def mb_step(grid, springs, q, v, Fext, nsteps=1, u_out=None, U0_out=None,
            diag_out=None, stream=None):
    return grid.step(springs, q, v, Fext, nsteps, u_out, U0_out, diag_out, stream)


def mb_step_ext(grid, springs, q, v, Fext=None, F_blob=None, nsteps=1, u_out=None,
                U0_out=None, diag_out=None, stream=None):
    return grid.step_ext(springs, q, v, Fext, F_blob, nsteps, u_out, U0_out, diag_out,
                         stream)


def mb_step_forced(grid, springs, q, v, f_fluid, Fext=None, F_blob=None, nsteps=1,
                   u_out=None, U0_out=None, diag_out=None, stream=None):
    return grid.step_forced(springs, q, v, f_fluid, Fext, F_blob, nsteps, u_out, U0_out,
                            diag_out, stream)


def mb_spring_forces_ext(springs, q, Fext, F_blob, F_out=None, stream=None):
    return spring_forces(springs, q, Fext, F_out, stream, F_blob)


def mb_interpolate_grad(grid, q, v, W, g_inout=None, stream=None):
    return grid.interpolate_grad(q, v, W, g_inout, stream)


def mb_spring_adjoint(springs, q, Fbar, qbar, kbar=None, r0bar=None, stream=None):
    return spring_adjoint(springs, q, Fbar, qbar, kbar, r0bar, stream)


def mb_step_adjoint(grid, springs, q_n, v_np1, qbar, vbar, Fext=None, F_blob=None,
                    ubar_loss=None, Fblob_bar=None, kbar=None, r0bar=None, stream=None):
    return grid.step_adjoint(springs, q_n, v_np1, qbar, vbar, Fext, F_blob, ubar_loss,
                             Fblob_bar, kbar, r0bar, stream)


def mb_step_graph(grids, springs, qs, vs, Fexts=None, F_blobs=None, nsteps=1, stream=None):
    return step_graph(grids, springs, qs, vs, Fexts, F_blobs, nsteps, stream)

