"""The C-ABI library loads and exports every entry point its header declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

import paper_1003_4548_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pdf_[a-z_0-9]+)\s*\(", txt))
    return names


def test_header_declares_the_binding_entry_points():
    assert _declared() == set(P.ENTRY_POINTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(P.library_path()):
        pytest.skip("library not built")
    lib = ctypes.CDLL(P.library_path())
    for name in sorted(_declared()):
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    # pdf_params: 8 int32 + 13 doubles; pdf_mesh: 2 int32 + 5 pointers; pdf_sizes: 4 int32 + 3 int64
    assert ctypes.sizeof(P.PdfParams) == 8 * 4 + 13 * 8
    assert ctypes.sizeof(P.PdfMesh) == 8 + 5 * 8
    assert ctypes.sizeof(P.PdfSizes) == 16 + 3 * 8
