"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid descriptors before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2306_00271_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol():
    lib = _lib()
    so = lib.load()
    header = open(os.path.join(ROOT, "include", "rheed.h")).read()
    names = set(re.findall(r"\b(rheed_[a-z0-9_]+)\s*\(", header))
    assert names, "no declarations found"
    for n in sorted(names):
        assert hasattr(so, n), n
    assert names == set(lib.SYMBOLS), "binding and header disagree"


def test_binding_constants_match_header():
    """Every RHEED_* constant the binding defines has the header's value."""
    lib = _lib()
    header = open(os.path.join(ROOT, "include", "rheed.h")).read()
    values = {m.group(1): int(m.group(2))
              for m in re.finditer(r"\b(RHEED_[A-Z0-9_]+)\s*=\s*(-?\d+)", header)}
    values.update({m.group(1): int(m.group(2))
                   for m in re.finditer(r"#define\s+(RHEED_[A-Z0-9_]+)\s+(-?\d+)", header)})
    ours = {k: v for k, v in vars(lib).items() if k.startswith("RHEED_") and isinstance(v, int)}
    assert len(ours) >= 15
    for k, v in sorted(ours.items()):
        assert k in values, f"{k} is not in the header"
        assert values[k] == v, f"{k}: binding {v}, header {values[k]}"


def test_beam_constants_and_errors():
    lib = _lib()
    so = lib.load()
    g, k = C.c_double(), C.c_double()
    assert so.rheed_beam_constants(15000.0, C.byref(g), C.byref(k)) == 0
    assert g.value == pytest.approx(63.2045, rel=1e-5) and k.value == pytest.approx(0.270173, rel=1e-5)
    assert so.rheed_beam_constants(-1.0, C.byref(g), C.byref(k)) == lib.RHEED_E_INVALID
    assert b"energy" in so.rheed_last_error()
    assert so.rheed_status_string(lib.RHEED_E_UNSUPPORTED) == b"unsupported"


def _structure(lib, beams, **kw):
    st = lib.Structure()
    arr = np.ascontiguousarray(np.asarray(beams, dtype=np.int32))
    st.n_beams = arr.shape[0]
    st.beam_hk = arr.ctypes.data_as(C.POINTER(C.c_int32))
    st.recip = (C.c_double * 4)(1.0, 0.0, 0.0, 1.0)
    st.n_slices = kw.get("n_slices", 10)
    st.thickness = kw.get("thickness", 5.0)
    st.wavenumber = 50.0
    st.n_atoms = 0
    return st, arr


@pytest.mark.parametrize("case,code", [
    ("beam0", -1), ("dup", -1), ("slices", -1), ("toomany", -4), ("box", -4), ("thr", -1)])
def test_plan_create_rejects_bad_descriptors(case, code):
    lib = _lib()
    so = lib.load()
    beams = [[0, 0], [1, 0], [0, 1]]
    kw = {}
    if case == "beam0":
        beams = [[1, 0], [0, 0]]
    elif case == "dup":
        beams = [[0, 0], [1, 0], [1, 0]]
    elif case == "slices":
        kw["n_slices"] = 0
    elif case == "toomany":
        beams = [[0, 0]] + [[h, 0] for h in range(1, 577)]   # N = 577 > RHEED_MAX_BEAMS
    elif case == "box":
        beams = [[0, 0], [9, 0], [0, 9], [-9, 0], [0, -9]]
    st, keep = _structure(lib, beams, **kw)
    arr = (lib.Structure * 1)(st)
    opts = lib.Opts(lib.RHEED_RK4, 0.5 if case == "thr" else 1000.0, 20, 0)
    aps = (C.c_int32 * 1)(3)
    h = C.c_void_p()
    assert so.rheed_plan_create(C.byref(h), C.byref(opts), 1, arr, aps) == code
    assert not h.value
    assert so.rheed_forward(None, None, None, None, None, None, None, None, 0, None) == lib.RHEED_E_INVALID
