"""The C-ABI library loads and exports every entry point include/gsr.h
declares; host-side argument validation (no GPU call is made)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gsr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2411_17660_amd import native
    return native.load()


def test_header_declares_entry_points():
    names = _declared()
    for n in ("gsr_create", "gsr_forward", "gsr_backward", "gsr_step_l1", "gsr_loss_l1",
              "gsr_loss_render", "gsr_step_render"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2411_17660_amd import native
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in native.EXPORTS, name


def test_struct_layouts_match_header(lib):
    from paper_2411_17660_amd import native
    assert C.sizeof(native.Camera) == 28
    assert C.sizeof(native.Settings) == 48
    assert native.Settings.key_capacity.offset == 32
    assert C.sizeof(native.Stats) == 64


def test_null_context_is_rejected_without_touching_the_gpu(lib):
    from paper_2411_17660_amd import native
    s = native.make_settings(3)
    cams = native.make_cameras([(16, 16, 10, 10, 8, 8)])
    rc = lib.gsr_forward(None, C.byref(s), 0, None, None, None, None, None, 1, cams, None, None,
                         None, None, None)
    assert rc == 1
    assert lib.gsr_backward(None, *([None] * 10)) == 1
    assert lib.gsr_loss_render(None, *([None] * 4), 0.9, 0.2, *([None] * 6)) == 1
    assert lib.gsr_last_error(None) == b""
    assert lib.gsr_create(None, 0) == 1
