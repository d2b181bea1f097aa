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
    """Argument validation, the table-size check included, happens before any HIP call, so
    it runs on the CPU."""
    import numpy as np
    from paper_1105_2791_amd import _lib as L
    L.lib()   # signatures
    h = ctypes.c_void_p()
    q = np.ones((2, 9))
    cl = np.ones(9)
    qp, cp = q.ctypes.data_as(ctypes.c_void_p), cl.ctypes.data_as(ctypes.c_void_p)
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: every call below fails first
    need = L.lib().modal_ctx_bytes(8, 12, 24, 2, L.F64, 0)

    def create(lmax, nt, nphi, P, prec, flags, q_, tables, nbytes):
        return L.lib().modal_create(ctypes.byref(h), lmax, nt, nphi, P, prec, flags, q_, cp, None, tables, nbytes)
    # null q or null tables -> EINVAL; ntheta <= lmax -> ESHAPE; odd nphi -> ESHAPE;
    # nphi <= 2 lmax -> ESHAPE; P < 1 -> EINVAL; unknown flag -> EINVAL
    assert create(8, 12, 24, 2, L.F64, 0, None, fake, need) == L.EINVAL
    assert create(8, 12, 24, 2, L.F64, 0, qp, None, need) == L.EINVAL
    assert create(8, 8, 24, 2, L.F64, 0, qp, fake, need) == L.ESHAPE
    assert create(8, 12, 25, 2, L.F64, 0, qp, fake, need) == L.ESHAPE
    assert create(8, 12, 16, 2, L.F64, 0, qp, fake, need) == L.ESHAPE
    assert create(8, 12, 24, 0, L.F64, 0, qp, fake, need) == L.EINVAL
    assert create(8, 12, 24, 2, L.F64, 4, qp, fake, need) == L.EINVAL
    # a buffer one byte short of the size query -> ENOSPACE
    assert create(8, 12, 24, 2, L.F64, 0, qp, fake, need - 1) == L.ENOSPACE
    assert h.value is None


def test_ctx_bytes_size_query(lib):
    """modal_ctx_bytes: host only, 256-byte granular, 0 for rejected arguments, and it grows
    by the lambda table (split precisions only) and with the grid."""
    from paper_1105_2791_amd import _lib as L
    f = L.lib().modal_ctx_bytes
    assert f(8, 8, 24, 2, L.F64, 0) == 0 and f(8, 12, 24, 0, L.F64, 0) == 0 and f(8, 12, 25, 2, L.F64, 0) == 0
    small = f(32, 48, 96, 8, L.BF16X3, 0)
    big = f(32, 48, 96, 8, L.BF16X3, L.CTX_LAMBDA_TABLE)
    assert small > 0 and small % 256 == 0 and big % 256 == 0
    assert big - small >= 33 * 16384   # at least one 16 KB record per m
    assert f(32, 48, 96, 8, L.F64, L.CTX_LAMBDA_TABLE) == f(32, 48, 96, 8, L.F64, 0)   # ignored for FP64
    # the pixel weights alone: FP64 and FP32 planes of npix values
    assert f(1000, 1536, 3072, 40, L.BF16X3, 0) > 12 * 1536 * 3072
    assert f(150, 199, 400, 13, L.F32, 0) < f(150, 399, 800, 13, L.F32, 0)
