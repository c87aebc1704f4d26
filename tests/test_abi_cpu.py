"""Host-side checks of the C ABI (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgm.h")
LIB = os.path.join(ROOT, "paper_1809_07986_amd", "libsgm.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("sgm_create", "sgm_full_frame", "sgm_reduced_frame", "sgm_get_disparity", "sgm_get_variance",
                 "sgm_get_motion_mask", "sgm_destroy"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_1809_07986_amd import _native
    assert sorted(_native.EXPORTS) == _declared()


def test_product_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1809_07986_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "sgm_oracle" not in text, f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsgm.so not built")
def test_paper_preset_is_table_1():
    # Table 1, "proposed": P1 6, P2 65, census window 5x5, max disparity 128;
    # host-only calls (they fill a struct)
    from paper_1809_07986_amd import _native as N
    lib = N.load()
    p, d = N.SgmParams(), N.SgmParams()
    assert lib.sgm_paper_params(ctypes.byref(p), 1242, 375, 128) == 0
    assert lib.sgm_default_params(ctypes.byref(d), 1242, 375, 128) == 0
    assert (p.census_w, p.census_h, p.p1, p.p2, p.max_disp, p.path_mask) == (5, 5, 6, 65, 128, 0xFF)
    for name, _ in N.SgmParams._fields_:
        if name not in ("census_w", "census_h", "p1", "p2"):
            assert getattr(p, name) == getattr(d, name), name
