"""The C ABI without a GPU: the library loads, exports what the header
declares, the header compiles as C and C++, struct layouts agree with the
binding, and argument errors are reported without touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2405_13364_amd import lucidraster as lr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lucidraster.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lr_\w+)\s*\(", src, re.M)))


def test_header_declares_the_binding_exports():
    assert declared() == sorted(lr.EXPORTS)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lr.LIB_PATH):
        pytest.skip("library not built")
    return lr.load_library()


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.check_output(["nm", "-D", "--defined-only", lr.LIB_PATH], text=True)
    syms = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(declared()) <= syms


@pytest.mark.parametrize("lang,compiler", [("c", "gcc"), ("c++", "g++")])
def test_header_compiles(lang, compiler, tmp_path):
    src = tmp_path / ("t.c" if lang == "c" else "t.cpp")
    src.write_text('#include "lucidraster.h"\nint main(void){lr_quad q; (void)q; return (int)sizeof(lr_stats);}\n')
    subprocess.check_call([compiler, "-Wall", "-Werror", "-I", os.path.dirname(HEADER), "-c", str(src),
                           "-o", str(tmp_path / "t.o")])


def test_struct_layouts(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lucidraster.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lr_quad), sizeof(lr_camera),'
                   ' sizeof(lr_config), sizeof(lr_stats), sizeof(lr_request), offsetof(lr_request, out_rgba8),'
                   ' offsetof(lr_request, block_h), sizeof(lr_tune_rule), offsetof(lr_request, status));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)], text=True).split()]
    want = [52, ctypes.sizeof(lr.Camera), ctypes.sizeof(lr.Config), ctypes.sizeof(lr.Stats),
            ctypes.sizeof(lr.Request), lr.Request.out_rgba8.offset, lr.Request.block_h.offset,
            ctypes.sizeof(lr.TuneRule), lr.Request.status.offset]
    assert got == want


def test_status_strings(lib):
    for code, name in [(0, "LR_OK"), (-1, "LR_ERR_INVALID_ARG"), (-4, "LR_ERR_CAPACITY"),
                       (-6, "LR_ERR_BUSY"), (-99, "LR_ERR_UNKNOWN")]:
        assert lib.lr_status_string(code).decode() == name


def test_argument_errors_need_no_device(lib):
    h = ctypes.c_void_p()
    assert lib.lr_create(None, ctypes.byref(h)) == lr.LR_ERR_INVALID_ARG
    # the caller owns device memory: no arena is an error, not an allocation
    cfg = lr.Config(device=0, bin_size=32, sorter_depth=8, block_h=8, arena=None, arena_bytes=1 << 30)
    assert lib.lr_create(ctypes.byref(cfg), ctypes.byref(h)) == lr.LR_ERR_INVALID_ARG
    assert b"arena" in lib.lr_last_error(None)
    for field, bad in [("bin_size", 24), ("sorter_depth", 5), ("block_h", 3), ("batch_slots", 9),
                       ("arena_bytes", 4096)]:
        cfg = lr.Config(device=0, bin_size=32, sorter_depth=8, block_h=8, arena=0x10000, arena_bytes=1 << 20)
        setattr(cfg, field, bad)
        assert lib.lr_create(ctypes.byref(cfg), ctypes.byref(h)) == lr.LR_ERR_INVALID_ARG, field
        assert lib.lr_last_error(None)
    cam = lr.Camera()
    assert lib.lr_render(None, 1, ctypes.byref(cam), 8, 8, None, None) == lr.LR_ERR_INVALID_ARG
    assert lib.lr_render_noalloc(None, 1, ctypes.byref(cam), 8, 8, None, None) == lr.LR_ERR_INVALID_ARG
    assert lib.lr_sync(None) == lr.LR_ERR_INVALID_ARG
    assert lib.lr_destroy(None) == lr.LR_ERR_INVALID_ARG
    assert lib.lr_upload_scene(None, None, 0, 0, None) == lr.LR_ERR_INVALID_ARG
    assert lib.lr_render_batch(None, None, 0, None) == lr.LR_ERR_INVALID_ARG
    assert lib.lr_set_tuning(None, None, 0) == lr.LR_ERR_INVALID_ARG
    assert lib.lr_request_bytes(None, None, None) == lr.LR_ERR_INVALID_ARG


def test_context_without_device_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    # a non-null arena address: the call gets as far as looking for a device
    cfg = lr.Config(device=0, bin_size=32, sorter_depth=8, block_h=8, arena=0x10000, arena_bytes=1 << 20)
    h = ctypes.c_void_p()
    assert lib.lr_create(ctypes.byref(cfg), ctypes.byref(h)) == lr.LR_ERR_DEVICE


def test_binding_fails_loudly_when_library_missing(tmp_path):
    with pytest.raises(ImportError):
        lr.load_library(str(tmp_path / "missing.so"))
