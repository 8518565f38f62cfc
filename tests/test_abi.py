"""The C ABI library loads and exports every function include/sgad.h declares
(CPU only: no compute call is made without a GPU)."""
import ctypes
import os
import re

from paper_2603_21055_amd import sgad

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = sgad.load()
    names = sgad.declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_binding_declares_every_header_function():
    assert set(sgad.declared_symbols()) <= set(sgad._SIGS)


def test_struct_layouts_match_header():
    # sizes of the POD structs the header defines, computed from their fields
    assert ctypes.sizeof(sgad.Cam) == 24
    assert ctypes.sizeof(sgad.Pose) == 48
    assert ctypes.sizeof(sgad.Job) == 12
    assert ctypes.sizeof(sgad.KfGrads) == 32
    assert ctypes.sizeof(sgad.AdamGroup) == 56
    assert ctypes.sizeof(sgad.Keyframe) == 24 + 48 + 6 * 8


def test_status_codes_match_header():
    txt = open(os.path.join(ROOT, "include", "sgad.h")).read()
    codes = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"(SGAD_\w+)\s*=\s*(\d+)", txt))
    assert codes["SGAD_OK"] == sgad.OK and codes["SGAD_EINVAL"] == sgad.EINVAL
    assert codes["SGAD_ERANGE"] == sgad.ERANGE and codes["SGAD_EHIP"] == sgad.EHIP
    assert codes["SGAD_ENOMEM"] == sgad.ENOMEM and codes["SGAD_EDATA"] == sgad.EDATA


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        return
    lib = sgad.load()
    h = ctypes.c_void_p()
    assert lib.sgad_create(0, ctypes.byref(h)) != sgad.OK
    assert not h.value
