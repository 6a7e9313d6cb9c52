"""The C-ABI library loads without a GPU and exports every symbol include/vplg.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vplg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vplg_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("vplg_context_create", "vplg_scene_upload", "vplg_vpls_generate", "vplg_gbuffer_render",
                 "vplg_gather", "vplg_gather_visibility_dump", "vplg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2203_11484_amd import vplg
    lib = vplg.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    # the binding covers the same set of entry points
    assert sorted(vplg.exported_symbols()) == _declared()


def test_calls_without_a_context_fail_cleanly():
    from paper_2203_11484_amd import vplg
    L = vplg.lib()
    assert L.vplg_version() >= 10000
    assert L.vplg_context_destroy(None) == vplg.EINVAL
    assert L.vplg_context_usage(None, None, None) == vplg.EINVAL
    assert b"context" in L.vplg_last_error()
    out = ctypes.c_void_p()
    rc = L.vplg_context_create(-1, 0, ctypes.byref(out))
    assert rc in (vplg.EINVAL, vplg.EHIP)
    assert not out.value
