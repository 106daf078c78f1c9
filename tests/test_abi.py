"""The C-ABI library loads on the CPU and exports every function include/bloch.h declares;
the Python binding declares exactly that set.  No compute call is made (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bloch.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bl_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("bl_create", "bl_destroy", "bl_solve_k", "bl_solve_path", "bl_footprint_bytes",
                 "bl_apply", "bl_set_k", "bl_gram", "bl_ritz_small"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2304_00337_amd import native
    if not os.path.exists(native.LIB_PATH):
        pytest.fail("libbloch.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(native.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(native.EXPORTED) == _declared()


def test_host_only_calls():
    """Calls that touch no device: defaults, footprint, error strings, argument checks."""
    from paper_2304_00337_amd import native
    lib = native.load()
    o = native.BlOpts()
    lib.bl_default_opts(ctypes.byref(o), 16)
    assert (o.nev, o.nthrow, o.nodal_cycles, o.extrap_depth) == (16, 8, 2, 3)
    g = native.BlGrid(256, 256, 1.0, 1.0)
    fp = lib.bl_footprint_bytes(ctypes.byref(g), ctypes.byref(o))
    assert 100e6 < fp < 20e9
    assert lib.bl_strerror(-4) == b"not converged"
    h = ctypes.c_void_p()
    bad = native.BlGrid(1, 4, 1.0, 1.0)
    eps = (ctypes.c_double * 4)(1, 1, 1, 1)
    assert lib.bl_create(ctypes.byref(bad), eps, ctypes.byref(o), None, ctypes.byref(h)) == native.BL_EINVAL
    assert b"n and m" in lib.bl_last_error()
    g2 = native.BlGrid(2, 2, 1.0, 1.0)
    neg = (ctypes.c_double * 4)(1, -1, 1, 1)
    assert lib.bl_create(ctypes.byref(g2), neg, ctypes.byref(o), None, ctypes.byref(h)) == native.BL_EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and every field offset of the public structs, compiled from bloch.h with the
    host C compiler, equal the ctypes declarations of the binding."""
    import shutil
    import subprocess
    from paper_2304_00337_amd import native
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"bl_grid": native.BlGrid, "bl_opts": native.BlOpts, "bl_info": native.BlInfo,
               "bl_problem": native.BlProblem, "bl_request": native.BlRequest,
               "bl_request_info": native.BlRequestInfo, "bl_server_counters": native.BlServerCounters}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bloch.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def test_raster_sources_match_the_oracle():
    """Host logic of the Section 6 raster: the library's sources of every grid point equal
    the oracle's, bit for bit; invalid arguments are rejected."""
    from oracle.extrapolation import raster_sources as ref
    from paper_2304_00337_amd import native
    from paper_2304_00337_amd.api import raster_sources
    for kappa in (2, 3, 4, 5, 7, 30):
        for j in range(kappa):
            for i in range(kappa):
                assert raster_sources(kappa, i, j) == ref(kappa, i, j), (kappa, i, j)
    lib = native.load()
    buf = (ctypes.c_int32 * 6)()
    assert lib.bl_raster_sources(1, 0, 0, buf) == native.BL_EINVAL
    assert lib.bl_raster_sources(4, 4, 0, buf) == native.BL_EINVAL
    assert lib.bl_raster_sources(4, 0, -1, buf) == native.BL_EINVAL
    assert lib.bl_raster_sources(4, 1, 1, None) == native.BL_EINVAL
