"""The C ABI library loads and exports every symbol include/speedygs.h declares
(no compute call: this runs without a GPU), and the Python binding's struct
layouts match the header."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "speedygs.h")
LIB = os.path.join(ROOT, "paper_2607_12656_amd", "libspeedygs.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sgs_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_2607_12656_amd import build
        build.build()
    return LIB


def test_library_exports_every_declared_symbol(built):
    L = C.CDLL(built)
    names = declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


def test_binding_covers_the_header(built):
    from paper_2607_12656_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()
    _lib.lib()


def test_struct_layouts():
    from paper_2607_12656_amd import _lib
    assert C.sizeof(_lib.sgs_camera) == 19 * 4
    assert C.sizeof(_lib.sgs_options) == 8 * 4
    # 64 floats, 3 int32, padding to 8, int64
    assert C.sizeof(_lib.sgs_adam_options) == 280
    assert _lib.sgs_adam_options.step.offset == 272
    src = open(HEADER).read()
    assert "#define SGS_STATS_WORDS 128" in src and _lib.STATS_WORDS == 128
    assert "#define SGS_RATE_GRAD_FLOATS 256" in src and _lib.RATE_GRAD_FLOATS == 256


def test_missing_library_fails_loudly(tmp_path):
    from paper_2607_12656_amd import _lib
    with pytest.raises(RuntimeError):
        _lib.lib(str(tmp_path / "nope.so"))


def test_null_context_arguments_are_rejected(built):
    """Calls that fail argument checks return EINVAL before touching a device."""
    L = C.CDLL(built)
    L.sgs_set_scene.restype = C.c_int
    assert L.sgs_set_scene(None, 1, 64, 1, None, 1, 8, 8, None) == -1
    L.sgs_render_fwd.restype = C.c_int
    assert L.sgs_render_fwd(None, None, None, None, None, None, None) == -1
    L.sgs_last_error.restype = C.c_char_p
    assert L.sgs_last_error(None) == b"null context"
