"""Host-side checks of the C-ABI library (no GPU compute): it loads, exports
every function include/lpb.h declares, fills default options, reports errors
without aborting, and tabulates the Gaunt integrals it builds its translation
operators from (checked against sympy's exact values)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lpb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lpb_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lpb():
    from paper_2002_01334_amd import lpb as m

    if not os.path.exists(m.LIB_PATH):
        pytest.skip("liblpbfmm.so not built (run __graft_entry__.build())")
    m.load()
    return m


def test_exports_every_declared_symbol(lpb):
    names = _declared()
    assert "lpb_evaluate" in names and len(names) >= 13
    lib = ctypes.CDLL(lpb.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lpb.EXPORTS)


def test_default_options(lpb):
    o = lpb.Options()
    lpb.load().lpb_default_options(ctypes.byref(o))
    assert (o.p, o.leaf_cap, o.precision, o.device, o.stages, o.timing) == (10, 50, 0, 0, 3, 0)
    assert o.quad_tol == 1e-16 and o.iface_tol == 1e-9


def test_create_rejects_bad_options_without_touching_the_gpu(lpb):
    L = lpb.load()
    for field, val in (("p", 0), ("p", 21), ("leaf_cap", 0)):
        o = lpb.Options()
        L.lpb_default_options(ctypes.byref(o))
        setattr(o, field, val)
        h = ctypes.c_void_p()
        rc = L.lpb_create(ctypes.byref(o), ctypes.byref(h))
        assert rc == lpb.LPB_ERANGE and not h.value
        assert L.lpb_last_error(None)
    # FP64 stops at LPB_MAX_P_FP64 = 15
    o = lpb.Options()
    L.lpb_default_options(ctypes.byref(o))
    o.p, o.precision = 16, lpb.LPB_FP64
    h = ctypes.c_void_p()
    assert L.lpb_create(ctypes.byref(o), ctypes.byref(h)) == lpb.LPB_ERANGE and not h.value
    # an allocator hook needs both functions
    o = lpb.Options()
    L.lpb_default_options(ctypes.byref(o))
    o.alloc = lpb.ALLOC_FN(lambda n, user: None)
    h = ctypes.c_void_p()
    assert L.lpb_create(ctypes.byref(o), ctypes.byref(h)) == lpb.LPB_EINVAL and not h.value
    # autotune is 0, 1 or 2; batch schedule codes stop at 7
    for field, val in (("autotune", 3), ("autotune", -1), ("schedule", 8 << 4), ("schedule", -1)):
        o = lpb.Options()
        L.lpb_default_options(ctypes.byref(o))
        setattr(o, field, val)
        h = ctypes.c_void_p()
        assert L.lpb_create(ctypes.byref(o), ctypes.byref(h)) == lpb.LPB_EINVAL and not h.value, (field, val)
    assert L.lpb_create(None, None) == lpb.LPB_EINVAL


def test_null_context_is_rejected(lpb):
    L = lpb.load()
    assert L.lpb_evaluate(None, None, None, 0) == lpb.LPB_EINVAL
    assert L.lpb_get_stats(None, None) == lpb.LPB_EINVAL
    assert L.lpb_evaluate_noalloc(None, None, None) == lpb.LPB_EINVAL
    L.lpb_destroy(None)


def test_library_gaunt_matches_sympy(lpb):
    from sympy.physics.wigner import gaunt

    cases = [(0, 0, 0, 0, 0, 0), (2, 1, 3, -1, 3, 0), (5, -3, 4, 2, 5, 1), (10, 4, 10, -7, 14, 3),
             (15, 15, 15, -14, 20, -1), (20, -5, 18, 9, 30, -4)]
    for n1, m1, n2, m2, n3, m3 in cases:
        ref = float(gaunt(n1, n2, n3, m1, m2, m3)) * (-1) ** (m1 + m2 + m3)
        assert lpb.host_gaunt(n1, m1, n2, m2, n3, m3) == pytest.approx(ref, abs=1e-15, rel=1e-12)
