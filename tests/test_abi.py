"""C-ABI checks that need no GPU: the library loads and exports every symbol the
public header declares; the header's enums match the binding's constants."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1105_2791_amd", "libmodal.so")
HEADER = os.path.join(ROOT, "include", "modal.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmodal.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_function(lib):
    from paper_1105_2791_amd._lib import header_functions
    names = header_functions(HEADER)
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1105_2791_amd import _lib
    assert set(_lib.header_functions(HEADER)) == set(_lib._SIGS)


def test_enums_match_binding():
    from paper_1105_2791_amd import _lib
    txt = open(HEADER).read()

    def val(name):
        m = re.search(rf"\b{name}\s*=\s*(\d+)", txt)
        return int(m.group(1)) if m else None
    assert val("MODAL_OK") == _lib.OK and val("MODAL_ENOSPACE") == _lib.ENOSPACE
    assert val("MODAL_F64") == _lib.F64 and val("MODAL_BF16X3") == _lib.BF16X3
    assert val("MODAL_OP_FNL") == _lib.OP_FNL and val("MODAL_LIN_APPLY") == _lib.LIN_APPLY
    assert val("MODAL_COV_FISHER") == _lib.COV_FISHER
    assert val("MODAL_OP_LINEAR_FINALIZE") == _lib.OP_LINEAR_FINALIZE
    assert val("MODAL_F16X3") == _lib.F16X3
    assert _lib.STAGES[val("MODAL_STAGE_LINEAR")] == "linear" and len(_lib.STAGES) == val("MODAL_NSTAGES")


def test_version_without_gpu(lib):
    lib.modal_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.modal_version()


def test_create_rejects_bad_arguments_before_touching_the_device(lib):
    """Argument validation happens before any HIP call, so it runs on the CPU."""
    import numpy as np
    lib.modal_create.restype = ctypes.c_int
    h = ctypes.c_void_p()
    q = np.ones((2, 9))
    cl = np.ones(9)
    # null q -> EINVAL; ntheta <= lmax -> ESHAPE; odd nphi -> ESHAPE; P < 1 -> EINVAL
    assert lib.modal_create(ctypes.byref(h), 8, 12, 24, 2, 0, None, cl.ctypes.data_as(ctypes.c_void_p), None) == 1
    assert lib.modal_create(ctypes.byref(h), 8, 8, 24, 2, 0, q.ctypes.data_as(ctypes.c_void_p),
                            cl.ctypes.data_as(ctypes.c_void_p), None) == 2
    assert lib.modal_create(ctypes.byref(h), 8, 12, 25, 2, 0, q.ctypes.data_as(ctypes.c_void_p),
                            cl.ctypes.data_as(ctypes.c_void_p), None) == 2
    assert lib.modal_create(ctypes.byref(h), 8, 12, 16, 2, 0, q.ctypes.data_as(ctypes.c_void_p),
                            cl.ctypes.data_as(ctypes.c_void_p), None) == 2
    assert lib.modal_create(ctypes.byref(h), 8, 12, 24, 0, 0, q.ctypes.data_as(ctypes.c_void_p),
                            cl.ctypes.data_as(ctypes.c_void_p), None) == 1
    assert h.value is None
