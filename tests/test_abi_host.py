"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/pmx.h declares, and reports errors as status codes (no GPU needed)."""
import ctypes
import os
import re
import subprocess
from pathlib import Path

import pytest

from paper_2401_12501_amd import pmx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            names.update(re.findall(r"^PMX_API\s+[\w\s\*]+?\b(pmx_\w+)\s*\(", txt, flags=re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 14
    L = ctypes.CDLL(pmx.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps every declared call under the same name
    assert set(names) <= set(pmx._SIGS)


def test_default_options():
    o = pmx.pmx_default_options()
    assert o.eta_near == 1.5 and o.n_gl == 16 and o.fmm_order == 6 and o.overlap == 1
    assert o.gmres_tol == 1e-10 and o.ir_tol == 1e-8 and o.inner_tol == 1e-4
    assert o.precision == pmx.PMX_PREC_FP64_DIRECT


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and struct size of the binding equals what the C compiler lays out
    from include/pmx.h (a small program built with gcc prints them)."""
    structs = {"pmx_options": pmx.pmx_options, "pmx_info": pmx.pmx_info,
               "pmx_operator_stats": pmx.pmx_operator_stats}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "pmx.h"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = Path(__file__).resolve().parents[1] / "include"
    subprocess.run(["gcc", "-std=c11", f"-I{inc}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "sizeof")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def test_null_arguments_are_errors():
    L = pmx.lib()
    assert L.pmx_apply(None, 0, 1, None, None, 0, None) == pmx.PMX_ERR_INVALID
    assert "null" in pmx.pmx_last_error()
    assert L.pmx_operator_get_stats(None, None) == pmx.PMX_ERR_INVALID
    L.pmx_operator_destroy(None)     # NULL-safe
    L.pmx_surface_destroy(None)
    L.pmx_ctx_destroy(None)
    assert L.pmx_edge_create(None, 1, None, None, None, None, None, None, 1, 0, None, None) == pmx.PMX_ERR_INVALID
    assert L.pmx_edge_apply(None, None, 0, 1, None, None, 0, None) == pmx.PMX_ERR_INVALID
    assert L.pmx_edge_size(None, None, None) == pmx.PMX_ERR_INVALID
    assert L.pmx_edge_export_points(None, None, None, None, None, None) == pmx.PMX_ERR_INVALID
    L.pmx_edge_destroy(None)
    assert L.pmx_edge_apply_kprime(None, 1, None, None, 0, None) == pmx.PMX_ERR_INVALID
    assert L.pmx_edge_apply_dlayer(None, 1, None, None, 0, None) == pmx.PMX_ERR_INVALID
