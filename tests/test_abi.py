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


def _plan(lib, P):
    """The split contraction's plan for P modes, through the C ABI (host only)."""
    nmax = P * (P + 1) * (P + 2) // 6
    max_items = 64
    items = (ctypes.c_int * (2 * max_items))()
    slots = (ctypes.c_int * (4 * 32 * max_items))()
    cell = (ctypes.c_int * nmax)()
    mult = ctypes.c_int(0)
    n = lib.modal_cubic_plan(P, max_items, items, slots, cell, ctypes.byref(mult))
    assert n > 0, (P, n)
    return n, list(items)[:2 * n], list(slots)[:4 * 32 * n], list(cell), mult.value


@pytest.mark.parametrize("P", list(range(1, 65)))
def test_cubic_plan_writes_every_triple_once(lib, P):
    """The cells the split contraction writes, emulated from the plan as the kernel's
    write-out reads it, cover every triple p <= r <= s exactly through the cell the
    reduction reads; no cell is written by two items (Sec. II, eq. (bbispect): the
    triple product is symmetric, so beta_prs is any pairing of the three maps)."""
    n, items, slots, cell, mult = _plan(lib, P)
    pair = {}
    for a in range(P):
        for b in range(a, P):
            pair[(a, b)] = len(pair)
    written = {}
    for i in range(n):
        first, s0 = items[2 * i], items[2 * i + 1]
        assert first == 32 * i
        assert P - 64 <= s0 <= max(0, P - 32)   # the window lies in the staged B rows
        for k in range(32):
            a0, b0, zlo, zhi = slots[4 * (first + k): 4 * (first + k) + 4]
            for j in range(4):
                a, b = a0 + j // 2, b0 + j % 2
                if a >= P or b >= P or a > b:
                    continue
                for t in range(max(s0, zlo, 0), min(s0 + 32, zhi, P)):
                    key = pair[(a, b)] * P + t
                    assert key not in written, (P, a, b, t)
                    written[key] = i
    tris = [(p, r, s) for p in range(P) for r in range(p, P) for s in range(r, P)]
    assert len(cell) == len(tris)
    inv = {v: k for k, v in pair.items()}
    for (p, r, s), c in zip(tris, cell):
        assert c in written, (P, p, r, s)
        a, b = inv[c // P]
        assert sorted((a, b, c % P)) == [p, r, s]
    assert mult in (1, 2, 4, 8)
    assert n * mult == 8 if mult > 1 else n >= 5


@pytest.mark.parametrize("P,items,mult", [(8, 1, 8), (30, 2, 4), (40, 4, 2), (50, 8, 1)])
def test_cubic_plan_item_counts(lib, P, items, mult):
    """Work of the split contraction at the configured mode counts: for P 40 the two
    classes take 61 blocks per window (4 items; 8 with pairs a <= b against modes t >= b)."""
    n, _, _, _, m = _plan(lib, P)
    assert (n, m) == (items, mult)


def test_cubic_plan_rejects_bad_P(lib):
    assert lib.modal_cubic_plan(0, 64, None, None, None, None) < 0
    assert lib.modal_cubic_plan(65, 64, None, None, None, None) < 0
    assert lib.modal_cubic_plan(40, 1, None, None, None, None) < 0
