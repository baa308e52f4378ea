"""The C-ABI library loads without a GPU and exports every function that
include/rtq.h declares (no compute calls here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rtq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rtq_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("rtq_scene_build", "rtq_scene_destroy", "rtq_trace_closest", "rtq_trace_occluded", "rtq_render",
                 "rtq_render_backward", "rtq_scene_set_albedo", "rtq_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2001_02620_amd as rtq
    L = rtq.load_library()
    for name in _declared():
        assert hasattr(L, name), name
    assert rtq.version().startswith("rtq")
    assert set(rtq.EXPORTS) <= set(_declared())


def test_error_message_is_available_without_gpu():
    import paper_2001_02620_amd as rtq
    L = rtq.load_library()
    assert isinstance(L.rtq_last_error(), bytes)


def test_null_arguments_are_rejected_on_the_host():
    """Argument checks that run before any device call (no GPU needed)."""
    import paper_2001_02620_amd as rtq
    L = rtq.load_library()
    assert L.rtq_scene_set_textures(None, None, 4, 1, None) == -1
    assert b"NULL" in L.rtq_last_error()
    assert L.rtq_scene_set_albedo(None, None, 0, None) == -1
