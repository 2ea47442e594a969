"""The C-ABI library loads on a machine without a GPU and exports every
function include/m1.h declares; the Python binding names the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "m1.h")
LIB = os.path.join(ROOT, "paper_2606_26268_amd", "libm1.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(m1_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("m1_create", "m1_set_opacity_table", "m1_step_explicit", "m1_step_implicit"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2606_26268_amd import m1
    assert sorted(m1.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_params_layout_matches_the_header():
    """m1_params_default (host code, no GPU) fills the binding's structure
    with the documented defaults: the field offsets agree with m1.h."""
    from paper_2606_26268_amd import m1
    p = m1.m1_params_default(2.5)
    assert (p.c, p.a_rad, p.gamma, p.e_floor) == (2.5, 1.0, 5.0 / 3.0, 1e-30)
    assert (p.precision, p.recon, p.riemann, p.absorb_only, p.second_order) == (m1.M1_P64, 0, 0, 0, 0)


def test_struct_layouts_match_the_header(tmp_path):
    """Every structure of the binding has the size and field offsets that a
    C compiler gives the header's declaration (gcc on the host; no GPU)."""
    import ctypes as C
    import shutil
    import subprocess
    from paper_2606_26268_amd import m1
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    structs = [getattr(m1, n) for n in ("m1_grid", "m1_params", "m1_fields", "m1_diag", "m1_mlp", "m1_train_cfg",
                                        "m1_train_report")]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "m1.h"', "int main(void) {"]
    expect = []
    for s in structs:
        lines.append(f'    printf("%zu\\n", sizeof({s.__name__}));')
        expect.append(C.sizeof(s))
        for f in s._fields_:
            lines.append(f'    printf("%zu\\n", offsetof({s.__name__}, {f[0]}));')
            expect.append(getattr(s, f[0]).offset)
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    r = subprocess.run([gcc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == expect
