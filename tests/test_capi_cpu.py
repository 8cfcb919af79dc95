"""The C-ABI library loads, exports every entry point its header declares,
and rejects bad arguments on the host before touching a device."""
import ctypes as C
import os
import re

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbremd.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_five_calls():
    names = _declared()
    for fn in ("gb_born_radii", "gb_energy_forces", "titration_delta_e", "md_step", "remd_exchange"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    from paper_1809_07726_amd import _capi
    lib = C.CDLL(_capi.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_capi.EXPORTED)


def test_host_side_argument_checks():
    from paper_1809_07726_amd import _capi as A
    L = A.lib
    h = C.c_void_p()
    off = (C.c_int32 * 3)(0, 5, 9)
    p = A.obc2()
    assert L.gbr_ctx_create(None, C.byref(p), 2, off) == A.GBR_E_INVAL
    assert L.gbr_ctx_create(C.byref(h), None, 2, off) == A.GBR_E_INVAL
    assert L.gbr_ctx_create(C.byref(h), C.byref(p), 0, off) == A.GBR_E_INVAL
    bad = (C.c_int32 * 3)(0, 5, 5)          # empty replica
    assert L.gbr_ctx_create(C.byref(h), C.byref(p), 2, bad) == A.GBR_E_INVAL
    assert b"atoms" in L.gbr_last_error()
    bad0 = (C.c_int32 * 3)(1, 5, 9)
    assert L.gbr_ctx_create(C.byref(h), C.byref(p), 2, bad0) == A.GBR_E_INVAL
    neg = A.obc2(); neg.eps_out = -1.0
    assert L.gbr_ctx_create(C.byref(h), C.byref(neg), 2, off) == A.GBR_E_INVAL
    # offsets whose difference overflows 32 bits, and a batch over GBR_MAX_ATOMS
    wide = (C.c_int32 * 3)(0, 5, -2 ** 31)
    assert L.gbr_ctx_create(C.byref(h), C.byref(p), 2, wide) == A.GBR_E_INVAL
    nb = A.MAX_ATOMS // 2 ** 20 + 1
    many = (C.c_int32 * (nb + 1))(*[r << 20 for r in range(nb + 1)])
    assert L.gbr_ctx_create(C.byref(h), C.byref(p), nb, many) == A.GBR_E_INVAL
    assert b"at most" in L.gbr_last_error()
    assert L.gbr_ctx_destroy(None) == A.GBR_OK             # a null context is a no-op
    # every call rejects a null context
    assert L.gb_born_radii(None, None, None, None, None, None, None, None) == A.GBR_E_INVAL
    assert L.gbr_set_launch(None, 4, 8) == A.GBR_E_INVAL
    assert L.gbr_set_timing(None, 1) == A.GBR_E_INVAL
    assert L.md_step(None, None, None, 0, 0, 1, 0, None) == A.GBR_E_INVAL
    assert L.remd_exchange(None, None, 0, None, None, None, None, None, None, None, None, 0, None) == A.GBR_E_INVAL
    assert L.titration_delta_e(None, None, None, None, None, None, 0, None, None) == A.GBR_E_INVAL
    assert L.gb_energy_forces(None, *([None] * 11), 0, None, None, None) == A.GBR_E_INVAL


@pytest.mark.skipif(torch.cuda.is_available(), reason="only meaningful without a device")
def test_context_without_device_reports_nodevice():
    from paper_1809_07726_amd import _capi as A
    h = C.c_void_p()
    off = (C.c_int32 * 2)(0, 8)
    p = A.obc2()
    assert A.lib.gbr_ctx_create(C.byref(h), C.byref(p), 1, off) == A.GBR_E_NODEVICE
