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
