"""The C ABI without a GPU: the shared library loads, exports every entry
point that include/pbicgstab.h declares, the ctypes binding agrees with the
header (names, enum values, struct layouts as the C compiler lays them out),
and the host-side argument checks reject malformed input before any device
call is made."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pbicgstab.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1809_01948_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1809_01948_amd import build
        build.build()
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^[A-Za-z_][\w \*]*?\b((?:pbicgstab|classic_bicgstab)_\w+)\s*\(",
                          text, flags=re.M))


def declared_enums():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for body in re.findall(r"enum\s*\{(.*?)\}", text, flags=re.S):
        for name, val in re.findall(r"(PBCG_\w+)\s*=\s*(-?\d+)", body):
            out[name] = int(val)
    return out


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ("pbicgstab_create_csr", "pbicgstab_create_stencil", "pbicgstab_solve",
              "classic_bicgstab_solve", "pbicgstab_destroy", "pbicgstab_last_error",
              "pbicgstab_grad_values", "pbicgstab_update_values"):
        assert f in fns, f


def test_library_exports_every_declared_symbol(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    for name in sorted(declared_functions()):
        assert hasattr(so, name), name
    nm = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    exported = {line.split()[-1] for line in nm.splitlines() if " T " in line}
    assert declared_functions() <= exported


def test_binding_matches_header(lib):
    assert set(lib.SIGNATURES) == declared_functions()
    enums = declared_enums()
    assert (enums["PBCG_FP64"], enums["PBCG_MIXED"]) == (lib.FP64, lib.MIXED)
    assert (enums["PBCG_PC_NONE"], enums["PBCG_PC_JACOBI"]) == (lib.PC_NONE, lib.PC_JACOBI)
    assert (enums["PBCG_ST_2D5"], enums["PBCG_ST_3D7"], enums["PBCG_ST_DIA5"]) == \
        (lib.ST_2D5, lib.ST_3D7, lib.ST_DIA5)
    for name, code in enums.items():
        if name in ("PBCG_OK",) or not (name.startswith("PBCG_ERR") or name in (
                "PBCG_CONVERGED", "PBCG_MAXIT", "PBCG_BREAKDOWN_RHO", "PBCG_BREAKDOWN_OMEGA",
                "PBCG_NONFINITE", "PBCG_TRUE_RES_NOT_MET")):
            continue
        assert lib.STATUS_NAMES[code] == name[len("PBCG_"):], name


def test_struct_layout_matches_c_compiler(lib, tmp_path):
    """sizeof/offsetof of pbcg_opts and pbcg_stats from gcc against ctypes."""
    fields = {"pbcg_opts": [f for f, _ in lib.Opts._fields_],
              "pbcg_stats": [f for f, _ in lib.Stats._fields_]}
    src = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for st, fl in fields.items():
        src.append(f'  printf("{st} size %zu\\n", sizeof({st}));')
        for f in fl:
            src.append(f'  printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    src += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-o", str(exe), str(c)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True,
                               check=True).stdout.splitlines():
        st, f, v = line.split()
        got[(st, f)] = int(v)
    for st, cls in (("pbcg_opts", lib.Opts), ("pbcg_stats", lib.Stats)):
        assert got[(st, "size")] == ctypes.sizeof(cls), st
        for f in fields[st]:
            assert got[(st, f)] == getattr(cls, f).offset, (st, f)


def test_default_opts(lib):
    L = lib.load()
    o = lib.Opts()
    o.tol = -1.0
    L.pbicgstab_default_opts(ctypes.byref(o))
    assert o.tol == 1e-10 and o.maxit == 10000 and o.rr_period == 0 and o.rr_tau == 0.0
    assert o.rr_auto == 0 and o.rr_eps == 0.0 and o.use_graph == 0 and not o.history
    L.pbicgstab_default_opts(None)   # tolerated


def _create(L, n, rowptr, col, val):
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    va = np.ascontiguousarray(val, dtype=np.float64)
    rc = L.pbicgstab_create_csr(ctypes.byref(h), n, len(ci), rp.ctypes.data, ci.ctypes.data,
                                va.ctypes.data, 0, 0, None)
    return rc, h, L.pbicgstab_last_error().decode()


@pytest.mark.parametrize("case,msg", [
    ("n0", "n must be"),
    ("rowptr0", "rowptr[0]"),
    ("decreasing", "nondecreasing"),
    ("col", "column index"),
])
def test_create_rejects_malformed_csr_on_host(lib, case, msg):
    L = lib.load()
    rowptr, col, val, n = [0, 1, 2], [0, 1], [1.0, 2.0], 2
    if case == "n0":
        n = 0
    elif case == "rowptr0":
        rowptr = [1, 1, 2]
    elif case == "decreasing":
        rowptr, n = [0, 2, 1, 2], 3
    elif case == "col":
        col = [0, 5]
    rc, h, err = _create(L, n, rowptr, col, val)
    assert rc == -1 and not h.value
    assert msg in err


def test_null_handle_is_rejected(lib):
    L = lib.load()
    o = lib.Opts()
    L.pbicgstab_default_opts(ctypes.byref(o))
    st = lib.Stats()
    rc = L.pbicgstab_solve(None, None, None, ctypes.byref(o), ctypes.byref(st))
    assert rc == -1
    assert L.pbicgstab_last_error()
    L.pbicgstab_destroy(None)       # no-op
