"""The C ABI library loads without a GPU, exports every declared entry point, and
rejects bad arguments before touching the device."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from paper_2509_06971_amd import _lib as L

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="libpetto.so not built")


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_phase_count_matches_header():
    import re
    txt = open(L.HEADER).read()
    assert int(re.search(r"#define PETTO_MAX_PHASES (\d+)", txt).group(1)) == L.MAX_PHASES


def test_exports_every_declared_symbol(lib):
    declared = L.declared_functions()
    assert len(declared) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for name in declared:
        assert name in exported, name
        assert hasattr(lib, name)
    assert lib.petto_version().decode().startswith("petto")


def _struct(prob, keep):
    from paper_2509_06971_amd.api import _problem_struct
    return _problem_struct(prob, keep)


def _create(lib, probs, prec=L.FP64):
    keep = []
    arr = (L.Problem * len(probs))()
    for i, p in enumerate(probs):
        arr[i] = _struct(p, keep)
    h = C.c_void_p()
    st = lib.petto_create(arr, len(probs), prec, C.byref(h))
    return st, h


def _expect_invalid(lib, probs, needle, prec=L.FP64, status=L.ERR_INVALID):
    st, h = _create(lib, probs, prec)
    assert st == status, (st, lib.petto_last_error())
    assert not h.value
    assert needle in lib.petto_last_error().decode()


def test_null_and_count_arguments(lib):
    h = C.c_void_p()
    assert lib.petto_create(None, 1, 0, C.byref(h)) == L.ERR_INVALID
    assert b"probs" in lib.petto_last_error()
    arr = (L.Problem * 1)()
    assert lib.petto_create(arr, 0, 0, C.byref(h)) == L.ERR_INVALID
    assert lib.petto_create(arr, 1, 7, C.byref(h)) == L.ERR_INVALID
    assert lib.petto_create(arr, 1, 0, None) == L.ERR_INVALID
    assert lib.petto_destroy(None) == L.OK
    assert lib.petto_field_offset(None, 0, 0) == C.c_size_t(-1).value
    info = (L.SolveInfo * 1)()
    assert lib.petto_apt_solve(None, None, None, None, None, None, info) == L.ERR_INVALID
    assert lib.petto_residual(None, None, None, None, None) == L.ERR_INVALID
    assert lib.petto_adjoint(None, None, None, None, 0, None, None, None) == L.ERR_INVALID
    assert lib.petto_adjoint_noalloc(None, None, None, None, 0, None, None, None) == L.ERR_INVALID
    assert lib.petto_phase_update(None, None, None, None, None, None) == L.ERR_INVALID
    assert lib.petto_step(None, None, None, None, None, None, None, None, None, None, None) == L.ERR_INVALID
    assert lib.petto_set_timing(None, 1) == L.ERR_INVALID


def test_problem_validation(lib):
    good = W.cantilever2d(8, 4)
    import copy

    def mod(**kw):
        p = copy.deepcopy(good)
        for k, v in kw.items():
            setattr(p, k, v)
        return p

    _expect_invalid(lib, [mod(physics=5)], "physics")
    _expect_invalid(lib, [mod(ndim=4)], "ndim")
    _expect_invalid(lib, [mod(n=(1, 4))], "n[0]")
    _expect_invalid(lib, [mod(h=0.0)], "h must be positive")
    _expect_invalid(lib, [mod(nu=0.5)], "nu")
    _expect_invalid(lib, [mod(emin=2.0)], "emin")
    _expect_invalid(lib, [mod(p=0.5)], "penalty")
    _expect_invalid(lib, [mod(side=(7, 0, 0, 0, 0, 0))], "side[0]")
    _expect_invalid(lib, [mod(load=None)], "needs a load")
    _expect_invalid(lib, [mod(load=np.zeros_like(good.load))], "load is zero")
    bad = good.load.copy()
    bad[1, 2, 3] = np.nan
    _expect_invalid(lib, [mod(load=bad)], "not finite")
    # the mask must hold the clamped side's normal unknowns
    fx = good.fixed.copy()
    fx[0, 1, 0] = 0
    _expect_invalid(lib, [mod(fixed=fx)], "misses the normal unknown")
    fx = good.fixed.copy()
    fx[0, 4, 3] = 1        # padding slot of u_x (row j = ny)
    _expect_invalid(lib, [mod(fixed=fx)], "padding")
    # all sides free and no pins: rigid modes
    _expect_invalid(lib, [mod(side=(0,) * 6, fixed=np.zeros_like(good.fixed))], "no Dirichlet")
    _expect_invalid(lib, [good, good], "one design", status=L.ERR_UNSUPPORTED)


def test_heat_validation(lib):
    import copy
    probs, _, _ = W.heat_batch(2, 8, 12, seed=1)
    p = copy.deepcopy(probs[0])
    p.fixed = np.zeros_like(p.fixed)
    _expect_invalid(lib, [p], "no Dirichlet face")
    p = copy.deepcopy(probs[0])
    p.fixed = p.fixed.copy()
    p.fixed[3, 3] |= 1
    _expect_invalid(lib, [p], "interior cell")
    p = copy.deepcopy(probs[0])
    p.fixed = None
    _expect_invalid(lib, [p], "Dirichlet faces")
    q3, _ = W.heat_slab((4, 4, 4))
    _expect_invalid(lib, [q3], "2D", status=L.ERR_UNSUPPORTED)
    _expect_invalid(lib, [probs[0], W.cantilever2d(8, 4)], "same physics")


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        L._lib_saved = L._lib
        try:
            L._lib = None
            L.load(str(tmp_path / "nope.so"))
        finally:
            L._lib = L._lib_saved


def test_3d_layer_size_limit(lib):
    """The 3D sweep addresses an xy layer by 32-bit byte offsets: larger layers are
    refused before anything is allocated (the load is never read)."""
    arr = (L.Problem * 1)()
    p = arr[0]
    p.physics, p.ndim = L.ELASTIC, 3
    p.n[0], p.n[1], p.n[2] = 30000, 30000, 2
    p.h, p.e0, p.emin, p.nu, p.p, p.nphase = 1.0, 1.0, 1e-9, 0.3, 3.0, 1
    dummy = (C.c_double * 1)()
    p.load = C.cast(dummy, C.POINTER(C.c_double))
    h = C.c_void_p()
    assert lib.petto_create(arr, 1, L.FP32, C.byref(h)) == L.ERR_UNSUPPORTED
    assert not h.value
    assert b"too large for the 3D sweep" in lib.petto_last_error()
