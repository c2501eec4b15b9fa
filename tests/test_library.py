"""The C-ABI library loads and exports every entry point its header declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re
import shutil
import subprocess

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


def test_struct_layouts_match_header(tmp_path):
    # pdf_params: 10 int32 + 17 doubles; pdf_mesh: 2 int32 + 5 pointers; pdf_sizes: 4 int32 + 3 int64
    assert ctypes.sizeof(P.PdfParams) == 10 * 4 + 17 * 8
    assert ctypes.sizeof(P.PdfMesh) == 8 + 5 * 8
    assert ctypes.sizeof(P.PdfSizes) == 16 + 3 * 8
    # every field offset as the C compiler lays out the header's struct
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    names = [f[0] for f in P.PdfParams._fields_]
    src = tmp_path / "offsets.c"
    body = "".join(f'  printf("%s %zu\\n", "{n}", offsetof(pdf_params, {n}));\n' for n in names)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "pdfpic.h"\nint main(void) {\n'
                   + body + '  printf("size %zu\\n", sizeof(pdf_params));\n  return 0;\n}\n')
    exe = tmp_path / "offsets"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for n in names:
        assert int(out[n]) == getattr(P.PdfParams, n).offset, n
    assert int(out["size"]) == ctypes.sizeof(P.PdfParams)


def test_create_rejects_bad_frequency_constants():
    """Argument checks of pdf_create run before any device call."""
    if not os.path.exists(P.library_path()):
        pytest.skip("library not built")
    L = P.load_library()

    def create(**kw):
        base = dict(f32_state=1, model=0, moments=2, hist_bins=0, mix=1, psi_init=0, flags=15, omega=1, vbins=2,
                    dt=1e-3, nu=1e-4, C0=3.5, CT=6.0, Cs=0.02, Ct=0.7, Cmu=0.09, kappa=0.41, Ewall=8.5,
                    yp=0.05, Lx=1.0, Ly=1.0, slack=2.0, C3=5.0, C4=0.25, Cw1=0.5, Cw2=0.73)
        base.update(kw)
        p = P.PdfParams(**base)
        ctx = ctypes.c_void_p()
        return L.pdf_create(ctypes.byref(p), None, ctypes.byref(ctx))

    assert create(omega=2) == -1
    assert create(C3=0.0) == -1
    assert create(C4=-0.25) == -1
    assert create(Cw1=50.0) == -1          # 1/2 + 3/4 C0 + C3 + Cw2 - Cw1 <= 0: no finite beta
    assert create(vbins=3) == -1
    assert create(vbins=5) == -1           # fine bins run without the turbulent frequency
    assert create(vbins=5, omega=0, f32_state=0) == -1
