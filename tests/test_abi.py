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
    assert (enums["PBCG_PC_NONE"], enums["PBCG_PC_JACOBI"],
            enums["PBCG_PC_BLOCK_JACOBI_BASE"]) == (lib.PC_NONE, lib.PC_JACOBI,
                                                    lib.PC_BLOCK_JACOBI_BASE)
    assert (enums["PBCG_ST_2D5"], enums["PBCG_ST_3D7"], enums["PBCG_ST_DIA5"],
            enums["PBCG_CSR"]) == (lib.ST_2D5, lib.ST_3D7, lib.ST_DIA5, lib.CSR)
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


def test_create_rejects_bad_arguments_before_any_device_call(lib):
    """n < 1, null CSR arrays and an unknown stencil kind are caught on the
    host (the CSR structure itself is read from the device and checked
    there: GPU tests)."""
    L = lib.load()
    h = ctypes.c_void_p()
    ws = ctypes.c_void_p(256)
    rc = L.pbicgstab_create_csr(ctypes.byref(h), 0, 0, ws, ws, ws, 0, 0, ws, 1 << 20, None)
    assert rc == -1 and not h.value and "n must be" in L.pbicgstab_last_error().decode()
    rc = L.pbicgstab_create_csr(ctypes.byref(h), 4, 4, None, None, None, 0, 0, ws, 1 << 20, None)
    assert rc == -1 and not h.value and "null CSR" in L.pbicgstab_last_error().decode()
    dims = (ctypes.c_int64 * 2)(4, 4)
    rc = L.pbicgstab_create_stencil(ctypes.byref(h), 7, dims, ws, 0, 0, ws, 1 << 20, None)
    assert rc == -1 and "kind" in L.pbicgstab_last_error().decode()


def _ws(L, fmt, n, nnz=0, width=0, prec=0, pc=0, tr=0):
    return L.pbicgstab_workspace_bytes(fmt, n, nnz, width, prec, pc, tr)


def test_workspace_bytes(lib):
    """Host arithmetic of the workspace size: 256-byte granularity, no matrix
    bytes for constant stencils, the documented increments for a Jacobi
    vector, a transposed layout and one more slot of slice width, and 0 for
    invalid arguments."""
    L = lib.load()
    CSR, S2, S3, D5 = lib.CSR, lib.ST_2D5, lib.ST_3D7, lib.ST_DIA5
    n = 5000
    npad = (n + 2047) // 2048 * 2048
    r256 = lambda b: (b + 255) // 256 * 256
    base = _ws(L, S2, n)
    assert base > 0 and base % 256 == 0
    assert _ws(L, S3, n) == base == _ws(L, S2, n, tr=1) == _ws(L, S2, n, pc=1)
    assert _ws(L, S2, n, prec=1) < base
    for prec, ts in ((0, 8), (1, 4)):
        d = _ws(L, D5, n, prec=prec)
        assert d == _ws(L, S2, n, prec=prec) + r256(5 * npad * ts)
        assert _ws(L, D5, n, prec=prec, pc=1) == d + r256(npad * ts)
        assert _ws(L, D5, n, prec=prec, tr=1) == d + r256(5 * npad * ts)
        c = _ws(L, CSR, n, 7 * n, 7, prec=prec)
        ns = (n + 63) // 64
        assert _ws(L, CSR, n, 7 * n, 8, prec=prec) == c + r256(ns * 64 * 8 * 4) - r256(
            ns * 64 * 7 * 4) + r256(ns * 64 * 8 * ts) - r256(ns * 64 * 7 * ts)
        assert _ws(L, CSR, n, 7 * n, 7, prec=prec, tr=1) > c
    # block-Jacobi (CSR only): A M^-1 bounded by width * b entries per row, M and
    # M^-1 in FP64 with b entries per row, one FP64 scratch vector; no transpose
    blk = lib.PC_BLOCK_JACOBI_BASE | 4
    cb = _ws(L, CSR, n, 5 * n, 5, pc=blk)
    ns = (n + 63) // 64
    assert cb == _ws(L, CSR, n, 5 * n, 5, pc=blk, tr=1)
    assert cb > _ws(L, CSR, n, 5 * n, 5) and cb % 256 == 0
    assert _ws(L, CSR, n, 5 * n, 6, pc=blk) - cb == r256(ns * 64 * 24 * 4) - r256(
        ns * 64 * 20 * 4) + r256(ns * 64 * 24 * 8) - r256(ns * 64 * 20 * 8)
    for bad in ((9, n, 0, 0, 0, 0, 0), (CSR, 0, 0, 0, 0, 0, 0), (CSR, n, -1, 0, 0, 0, 0),
                (S2, n, 0, 0, 2, 0, 0), (S2, n, 0, 0, 0, 3, 0), (S2, n, 0, 0, 0, blk, 0),
                (CSR, n, 5 * n, 5, 0, lib.PC_BLOCK_JACOBI_BASE | 1, 0),
                (CSR, n, 5 * n, 5, 0, lib.PC_BLOCK_JACOBI_BASE | 65, 0)):
        assert L.pbicgstab_workspace_bytes(*bad) == 0
        assert L.pbicgstab_last_error()


def test_null_handle_is_rejected(lib):
    L = lib.load()
    o = lib.Opts()
    L.pbicgstab_default_opts(ctypes.byref(o))
    st = lib.Stats()
    rc = L.pbicgstab_solve(None, None, None, ctypes.byref(o), ctypes.byref(st))
    assert rc == -1
    assert L.pbicgstab_last_error()
    L.pbicgstab_destroy(None)       # no-op
