"""Host-only checks of the C ABI: libws.so loads, exports every symbol that
include/ws.h declares, and rejects bad arguments before touching a device."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2410_08946_amd as ws
    from paper_2410_08946_amd import _build
    if not os.path.exists(ws.lib_path()):
        _build.build()
    return ws.load_library()


def _declared():
    src = open(os.path.join(ROOT, "include", "ws.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ws_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    import paper_2410_08946_amd as ws
    lib = _lib()
    names = _declared()
    assert "ws_watershed" in names and "ws_waterfall" in names and "ws_gradient" in names
    for n in names:
        assert hasattr(lib, n), n
        assert n in ws.binding.SIGNATURES, n


def test_footprint_is_host_arithmetic():
    lib = _lib()
    n = 4096 * 4096
    fp = lib.ws_footprint_bytes(4096, 4096, 1, 8, 2, 6)
    assert fp >= n * (2 + 4 * 6)
    # the edge slabs grow with the neighbourhood; a single layer needs no waterfall tables
    assert lib.ws_footprint_bytes(4096, 4096, 1, 4, 2, 6) < fp
    assert lib.ws_footprint_bytes(4096, 4096, 1, 8, 2, 1) < lib.ws_footprint_bytes(4096, 4096, 1, 8, 2, 2)
    assert lib.ws_footprint_bytes(64, 64, 64, 26, 1, 3) > lib.ws_footprint_bytes(64, 64, 64, 6, 1, 3)
    assert lib.ws_footprint_bytes(0, 4, 1, 8, 1, 3) == 0
    assert lib.ws_footprint_bytes(4, 4, 1, 8, 3, 3) == 0
    assert lib.ws_footprint_bytes(4, 4, 1, 8, 1, 0) == 0
    assert lib.ws_footprint_bytes(4, 4, 1, 6, 1, 3) == 0   # 3D connectivity on a 2D image
    assert lib.ws_footprint_bytes(4, 4, 4, 8, 1, 3) == 0   # 2D connectivity on a 3D image
    assert lib.ws_footprint_bytes(1 << 16, 1 << 16, 1, 8, 1, 1) == 0


def test_null_context_is_rejected_without_device():
    lib = _lib()
    buf = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert lib.ws_watershed(None, buf, 1, 8, 8, 1, 4, buf, None) == -1
    assert b"ctx" in lib.ws_last_error(None)
    assert lib.ws_waterfall(None, buf, buf, 1, 8, 8, 1, 4, 3, buf, None, None) == -1
    assert lib.ws_gradient(None, buf, 8, 8, 1, 1.0, 1, buf, None, None) == -1
    assert lib.ws_watershed_stages(None, buf, 1, 8, 8, 1, 4, buf, buf, None) == -1
    assert lib.ws_set_option(None, b"rr", 2) == -1
    assert lib.ws_sync(None, None) == -1
    assert lib.ws_create(None, 0, 0) == -1
    lib.ws_destroy(None)


def test_product_path_has_no_oracle_dependency():
    """The package never imports the oracle and the HIP sources never include it."""
    pkg = os.path.join(ROOT, "paper_2410_08946_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("the oracle", ""), f
                assert "ws_oracle" not in txt, f


def test_item_layout_matches_header(tmp_path):
    """The binding's ws_item has the header's size and field offsets (a small
    C program compiled against include/ws.h prints them)."""
    import shutil
    import subprocess

    from paper_2410_08946_amd.binding import WsItem
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text(
        "#include <stddef.h>\n#include <stdio.h>\n#include \"ws.h\"\n"
        "int main(void) { printf(\"%zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(ws_item), "
        "offsetof(ws_item, grad), offsetof(ws_item, nx), offsetof(ws_item, ny), offsetof(ws_item, nz), "
        "offsetof(ws_item, conn), offsetof(ws_item, out), offsetof(ws_item, nregions)); return 0; }\n")
    exe = tmp_path / "layout"
    subprocess.check_call([gcc, "-I" + os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(WsItem)] + [getattr(WsItem, f).offset
                                       for f in ("grad", "nx", "ny", "nz", "conn", "out", "nregions")]
    assert got == want
