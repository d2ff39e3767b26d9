"""The ctypes binding and include/dmrg.h agree on every struct's size and
field offsets (a C program built with the host compiler prints them), and the
host-only entry points behave as documented (no GPU needed)."""

import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")
LIB = os.path.join(ROOT, "paper_2311_02854_amd", "lib", "libdmrg.so")

STRUCTS = {
    "dmrg_integrals": "Integrals",
    "dmrg_mps": "Mps",
    "dmrg_build_opts": "BuildOpts",
    "dmrg_stats": "Stats",
    "dmrg_davidson_opts": "DavidsonOpts",
    "dmrg_davidson_stats": "DavidsonStats",
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    from paper_2311_02854_amd import binding as B
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dmrg.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in getattr(B, pyname)._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c99", "-I", HEADER_DIR, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    vals = {}
    for ln in out.splitlines():
        s, f, v = ln.split()
        vals[(s, f)] = int(v)
    return vals


@pytest.mark.parametrize("cname", sorted(STRUCTS))
def test_struct_layout_matches_header(c_layout, cname):
    from paper_2311_02854_amd import binding as B
    cls = getattr(B, STRUCTS[cname])
    assert ctypes.sizeof(cls) == c_layout[(cname, "size")], cname
    for field, _ in cls._fields_:
        assert getattr(cls, field).offset == c_layout[(cname, field)], (cname, field)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_davidson_default_options():
    from paper_2311_02854_amd import binding as B
    lib = B.load()
    o = B.DavidsonOpts()
    lib.dmrg_davidson_default_opts(ctypes.byref(o))
    assert o.tol_residual == 1e-6 and o.max_iter == 200 and o.m_max == 24
    assert o.precision == 0 and o.precond == 0 and o.stagnation == 4
    assert o.precond_shift == 1.0          # shifted diagonal preconditioner by default
    assert o.switch_residual == 1e-4 and o.e_tol == 1e-6 and o.e_ref != o.e_ref   # NaN: no reference
    assert not o.trace and o.trace_cap == 0 and not o.mlp_weights


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_launch_shape_rejects_bad_values():
    from paper_2311_02854_amd import binding as B
    lib = B.load()
    # null ops, unknown precision / tile, grid below -1 (dynamic units)
    assert lib.dmrg_launch_shape(None, 0, 0, 0) == -1
    assert lib.dmrg_autotune(None, None, 0, None, None) == -1
