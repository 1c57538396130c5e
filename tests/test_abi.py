"""The C-ABI library loads and exports every entry point the header declares.

Runs without a GPU: only host-side calls (workspace sizing, argument checks
that fail before any device work) are made.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfg.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(sfg_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_2008_07633_amd import sfg

    return sfg.lib()


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ["sfg_laplacian_csr", "sfg_smooth", "sfg_edge_scores", "sfg_coarsen", "sfg_sparsify"]:
        assert required in names


def test_library_exports_every_declared_symbol(L):
    from paper_2008_07633_amd import sfg

    for name in declared_symbols():
        assert hasattr(L, name), name
    assert sorted(sfg.EXPORTED) == declared_symbols()


def test_workspace_sizes_are_host_only(L):
    from paper_2008_07633_amd import sfg

    a = sfg.sfg_workspace_bytes(sfg.OP_SMOOTH, 1000, 0, 16, sfg.F64)
    b = sfg.sfg_workspace_bytes(sfg.OP_SMOOTH, 1000, 0, 16, sfg.F32)
    assert a >= 2 * 1000 * 16 * 8 and b >= 2 * 1000 * 16 * 4 and a > b
    assert sfg.sfg_workspace_bytes(sfg.OP_LAPLACIAN_CSR, 100, 300, 0, sfg.F64) > 5 * 101 * 4
    assert sfg.sfg_workspace_bytes(sfg.OP_SELECT_TOPK, 0, 10000, 0, sfg.F64) > 2 * 10000 * 4
    assert sfg.sfg_workspace_bytes(99, 1, 1, 1, sfg.F64) == 0


def test_argument_errors_before_device_work(L):
    from paper_2008_07633_amd import sfg

    H = sfg.CsrStruct(0, 0, None, None, None, None, None, sfg.F64)
    st = L.sfg_smooth(ctypes.byref(H), 4, 1, 0.5, None, sfg.F64, 0, None, None, 0, None)
    assert sfg.STATUS[st] == "SFG_EINVAL"
    assert b"null pointer" in L.sfg_last_error()
    st = L.sfg_csr_select(ctypes.byref(H), None, None, None, None, None, None, None, None, 0, None)
    assert sfg.STATUS[st] == "SFG_EINVAL"
    assert b"csr_select" in L.sfg_last_error()
    p = sfg.make_params(k=100)
    st = L.sfg_sparsify(10, 0, None, None, None, sfg.F64, ctypes.byref(p), None, None, None, None)
    assert sfg.STATUS[st] == "SFG_EUNSUPPORTED"
    p = sfg.make_params(omega=1.5)
    st = L.sfg_sparsify(10, 0, None, None, None, sfg.F64, ctypes.byref(p), None, None, None, None)
    assert sfg.STATUS[st] == "SFG_EINVAL"
    st = L.sfg_select_topk(None, sfg.F64, 10, 11, None, None, None, None, 0, None)
    assert sfg.STATUS[st] == "SFG_EINVAL"
    st = L.sfg_edge_scores(None, sfg.F64, 10, 65, 1, None, None, None, None, sfg.F64, None, sfg.F64, None)
    assert sfg.STATUS[st] == "SFG_EUNSUPPORTED"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2008_07633_amd import sfg

    monkeypatch.setattr(sfg, "_lib", None)
    monkeypatch.setattr(sfg, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        sfg.lib()


def test_every_entry_point_has_a_signature(L):
    # without argtypes ctypes passes Python ints as 32-bit C ints, and a size_t
    # passed on the stack arrives with undefined upper bits
    from paper_2008_07633_amd import sfg

    for name in sfg.EXPORTED:
        assert getattr(L, name).argtypes is not None, name


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes mirrors of the header's structs: same size and field offsets as the C compiler gives
    import shutil
    import subprocess

    from paper_2008_07633_amd import sfg

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    mirrors = {"sfg_csr": sfg.CsrStruct, "sfg_kappa_params": sfg.KappaParams, "sfg_kappa_report": sfg.KappaReport,
               "sfg_tree": sfg.TreeStruct, "sfg_surrogate": sfg.SurrogateStruct, "sfg_params": sfg.Params,
               "sfg_level_report": sfg.LevelReport, "sfg_report": sfg.Report,
               "sfg_pcg_report": sfg.PcgReport}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sfg.h"', "int main(void) {"]
    for c, py in mirrors.items():
        lines.append(f'printf("{c} (sizeof) %zu\\n", sizeof({c}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{c} {f} %zu\\n", offsetof({c}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        c, f, val = line.split()
        got[(c, f)] = int(val)
    for c, py in mirrors.items():
        assert got[(c, "(sizeof)")] == ctypes.sizeof(py), c
        for f, _ in py._fields_:
            assert got[(c, f)] == getattr(py, f).offset, (c, f)


def test_size_limits_before_device_work(L):
    # 32-bit row pointers and edge ids: 2m and n must stay below 2^31, rejected
    # as unsupported before any pointer is looked at or any device work is queued
    from paper_2008_07633_amd import sfg

    big_m, big_n = 1 << 30, (1 << 31) - 1
    cases = [
        (lambda: L.sfg_laplacian_csr(10, big_m, *[None] * 3, sfg.F64, *[None] * 8, 0, None), b"2*m"),
        (lambda: L.sfg_laplacian_csr(big_n, 0, *[None] * 3, sfg.F64, *[None] * 8, 0, None), b"n must"),
        (lambda: L.sfg_tree_order(10, big_m, *[None] * 3, sfg.F64, *[None] * 8, 0, None), b"2*m"),
        (lambda: L.sfg_pcg(10, big_m, *[None] * 3, sfg.F64, None, None, None, 1e-6, 10, None, None), b"2*m"),
        (lambda: L.sfg_kappa_estimate(10, big_m, *[None] * 3, sfg.F64, *[None] * 6), b"2*m"),
        (lambda: L.sfg_select_topk(None, sfg.F64, 1 << 31, 1, None, None, None, None, 0, None), b"ne must"),
    ]
    for call, msg in cases:
        st = call()
        assert sfg.STATUS[st] == "SFG_EUNSUPPORTED", L.sfg_last_error()
        assert msg in L.sfg_last_error()
    # one below the limit passes the size check and fails on the next argument
    st = L.sfg_laplacian_csr(10, (1 << 30) - 1, *[None] * 3, sfg.F64, *[None] * 8, 0, None)
    assert sfg.STATUS[st] == "SFG_EWORKSPACE"


def test_header_declares_every_export(L):
    # the reverse of the export check: no sfg_ entry point exists that the header does not document
    import shutil
    import subprocess

    from paper_2008_07633_amd import sfg

    if shutil.which("nm") is None:
        pytest.skip("no nm")
    out = subprocess.run(["nm", "-D", "--defined-only", sfg.LIB_PATH], check=True, capture_output=True,
                         text=True).stdout
    exported = sorted({f[2] for f in (line.split() for line in out.splitlines())
                       if len(f) == 3 and f[1] == "T" and f[2].startswith("sfg_")})
    assert exported == declared_symbols()


def test_header_compiles_as_c_and_cpp(tmp_path):
    import shutil
    import subprocess

    src_c = tmp_path / "h.c"
    src_c.write_text('#include "sfg.h"\nint main(void) { return (int)sizeof(sfg_params) == 0; }\n')
    src_cc = tmp_path / "h.cc"
    src_cc.write_text('#include "sfg.h"\nint main() { sfg_status s = SFG_OK; return (int)s; }\n')
    inc = os.path.join(ROOT, "include")
    for cc, src, std in (("gcc", src_c, "-std=c99"), ("g++", src_cc, "-std=c++17")):
        if shutil.which(cc) is None:
            pytest.skip(f"no {cc}")
        subprocess.run([cc, std, "-Wall", "-Werror", "-pedantic", "-fsyntax-only", "-I", inc, str(src)], check=True)
