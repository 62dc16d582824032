"""C-ABI contract on the CPU host: the library loads, exports every function
the header declares, and rejects invalid arguments before touching the
device (no compute call runs here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1407_5600_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "multiblob.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_step_calls():
    names = _declared()
    for n in ("mb_grid_create", "mb_spread", "mb_interpolate", "mb_fluid_solve",
              "mb_spring_forces", "mb_step"):
        assert n in names


def test_every_declared_symbol_is_exported():
    L = b.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) == set(b.EXPORTED)


def test_status_strings():
    for st in (0, -1, -2, -3, -4, -5):
        assert b.status_string(st)
    assert "invalid" in b.status_string(-1)
    assert "non-finite" in b.status_string(b.MB_ERR_NONFINITE)


def _desc(**kw):
    d = dict(L=32, precision=0, mode=0, zero_mean=0, h=1.0, rho=1.0, eta=1.0,
             dt=0.01, max_blobs=100, deterministic=0, check_finite=0,
             external_workspace=0, reserved=0)
    d.update(kw)
    return b.GridDesc(d["L"], d["precision"], d["mode"], d["zero_mean"], d["h"],
                      d["rho"], d["eta"], d["dt"], d["max_blobs"], d["deterministic"],
                      d["check_finite"], d["external_workspace"], d["reserved"])


def _create(**kw):
    desc = _desc(**kw)
    h = ctypes.c_void_p(123)
    st = b.lib().mb_grid_create(ctypes.byref(desc), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kw", [
    dict(L=20), dict(L=7), dict(L=1024), dict(L=40), dict(L=0),
    dict(precision=2), dict(mode=5), dict(zero_mean=3),
    dict(h=0.0), dict(h=-1.0), dict(h=float("nan")), dict(dt=0.0),
    dict(rho=0.0), dict(eta=-1.0), dict(mode=1, eta=0.0), dict(max_blobs=-1),
    dict(L=648), dict(deterministic=2), dict(check_finite=-1), dict(external_workspace=2),
    dict(reserved=1),
])
def test_grid_create_rejects_invalid(kw):
    st, h = _create(**kw)
    assert st == b.MB_ERR_INVALID
    assert h.value is None
    assert b.lib().mb_workspace_size(ctypes.byref(_desc(**kw)), 1) == 0


@pytest.mark.parametrize("L", [12, 18, 27, 36, 54, 81, 108, 162, 324, 486])
def test_grid_create_unsupported_sizes(L):
    """2^a 3^b sizes that are not multiples of 8 have no tile kernels."""
    st, h = _create(L=L)
    assert st == b.MB_ERR_UNSUPPORTED
    assert h.value is None


@pytest.mark.parametrize("kw", [dict(), dict(L=24), dict(L=512), dict(precision=1),
                                dict(mode=1, rho=0.0), dict(eta=0.0), dict(deterministic=1),
                                dict(check_finite=1), dict(external_workspace=1)])
def test_grid_create_valid_needs_device(kw):
    """Valid descriptions pass validation and then report the missing GPU."""
    st, h = _create(**kw)
    assert st == b.MB_ERR_DEVICE
    assert h.value is None


def test_workspace_size():
    """mb_workspace_size is host arithmetic: it covers the spectrum, the spread
    boxes and the per-blob scratch, grows with max_blobs, the precision and
    the box count, and is a multiple of 256 bytes."""
    ws = lambda nbox=1, **kw: b.lib().mb_workspace_size(ctypes.byref(_desc(**kw)), nbox)
    for L in (8, 24, 32, 128, 144, 512):
        for prec, s in ((0, 8), (1, 4)):
            n = ws(L=L, precision=prec, max_blobs=1000)
            spectrum = 3 * L * L * (L // 2 + 1) * 2 * s
            boxes = 3 * L ** 3 * s  # at least one entry per node
            assert n % 256 == 0 and n > spectrum + boxes + 1000 * 48
    assert ws(L=64, precision=0) > ws(L=64, precision=1)
    assert ws(L=64, max_blobs=10 ** 6) - ws(L=64, max_blobs=1000) >= 999000 * 48
    assert ws(nbox=4, L=32) > 3 * ws(nbox=1, L=32)
    assert ws(nbox=0) == 0 and ws(nbox=70000) == 0
    assert b.lib().mb_workspace_size(None, 1) == 0
    # the description flags do not change the size
    assert ws(L=48, deterministic=1, check_finite=1, external_workspace=1) == ws(L=48)


def test_null_arguments():
    L = b.lib()
    assert L.mb_grid_create(None, None) == b.MB_ERR_INVALID
    h = ctypes.c_void_p()
    assert L.mb_grid_create(None, ctypes.byref(h)) == b.MB_ERR_INVALID
    assert L.mb_spread(None, 0, None, None, None, None) == b.MB_ERR_INVALID
    assert L.mb_interpolate(None, 0, None, None, None, None) == b.MB_ERR_INVALID
    assert L.mb_fluid_solve(None, None, None, None, None) == b.MB_ERR_INVALID
    assert L.mb_spring_forces(None, 0, None, None, None, None) == b.MB_ERR_INVALID
    assert L.mb_step(None, None, 0, None, None, None, None, None, None, 1, None) == b.MB_ERR_INVALID
    assert L.mb_grid_destroy(None) == b.MB_OK
    assert L.mb_grid_set_workspace(None, None, 0) == b.MB_ERR_INVALID
    assert L.mb_springs_set_params(None, None, 1.0, None) == b.MB_ERR_INVALID
    assert L.mb_springs_destroy(None) == b.MB_OK
    assert L.mb_grid_set_timing(None, 1) == b.MB_ERR_INVALID
    assert L.mb_kernel_name(0) == b"bin_count"
    assert L.mb_kernel_name(-1) is None


@pytest.mark.parametrize("case", ["self_pair", "out_of_range", "bad_rest", "neg_k", "nb0"])
def test_springs_create_rejects_invalid(case):
    pa = np.array([0, 1], np.int32)
    pb = np.array([1, 2], np.int32)
    r0 = np.array([1.0, 1.0])
    nb, k = 3, 1.0
    if case == "self_pair":
        pb[0] = 0
    elif case == "out_of_range":
        pb[1] = 3
    elif case == "bad_rest":
        r0[0] = 0.0
    elif case == "neg_k":
        k = -1.0
    elif case == "nb0":
        nb = 0
    h = ctypes.c_void_p()
    st = b.lib().mb_springs_create(nb, 2, pa.ctypes.data_as(ctypes.c_void_p),
                                   pb.ctypes.data_as(ctypes.c_void_p),
                                   r0.ctypes.data_as(ctypes.c_void_p), k, ctypes.byref(h))
    assert st == b.MB_ERR_INVALID


def test_springs_create_valid_needs_device():
    from paper_1407_5600_amd import inputs
    pa, pb, r0 = inputs.pair_table(inputs.icosahedron_template())
    h = ctypes.c_void_p()
    st = b.lib().mb_springs_create(13, len(pa), pa.ctypes.data_as(ctypes.c_void_p),
                                   pb.ctypes.data_as(ctypes.c_void_p),
                                   r0.ctypes.data_as(ctypes.c_void_p), 100.0, ctypes.byref(h))
    assert st == b.MB_ERR_DEVICE


def test_product_path_does_not_touch_the_oracle():
    """The GPU package neither imports nor loads anything under oracle/."""
    pkg = os.path.join(ROOT, "paper_1407_5600_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "liboracle" not in text and "mbo_" not in text, fn
