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


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of the header's struct, from a C compiler."""
    import subprocess
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src.write_text(f"""#include <stddef.h>
#include <stdio.h>
#include "gsr.h"
int main(void) {{
  printf("%zu\\n", sizeof({struct}));
{body}  return 0;
}}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    vals = [int(v) for v in out.split()]
    return vals[0], vals[1:]


@pytest.mark.parametrize("cname,pyname", [("gsr_camera", "Camera"), ("gsr_settings", "Settings"),
                                          ("gsr_stats", "Stats")])
def test_struct_layouts_match_header(lib, cname, pyname, tmp_path):
    from paper_2411_17660_amd import native
    cls = getattr(native, pyname)
    fields = [f for f, _ in cls._fields_]
    size, offs = _c_layout(cname, fields, tmp_path)
    assert C.sizeof(cls) == size
    assert [getattr(cls, f).offset for f in fields] == offs


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
