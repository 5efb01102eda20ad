"""The C-ABI library loads and exports every entry point of include/pbh.h, and
argument checks that happen before any device work return PBH_EINVAL (CPU)."""
import ctypes as C
import os
import re

import pytest

import paper_1908_09378_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pbh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_named_contract():
    names = declared_functions()
    for f in ["pbh_create", "pbh_bulk_update", "pbh_extract_min", "pbh_destroy", "sssp", "pbh_last_error"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    L = pkg.lib()
    for f in declared_functions():
        assert hasattr(L, f), f


def test_null_arguments_are_rejected():
    L = pkg.lib()
    assert L.pbh_create(None, 10, 2) == pkg.PBH_EINVAL
    assert L.pbh_destroy(None) == pkg.PBH_OK
    assert L.pbh_bulk_update(None, None, None, 1) == pkg.PBH_EINVAL
    assert L.pbh_delete(None, None, 1) == pkg.PBH_EINVAL
    n = C.c_uint64(0)
    assert L.pbh_extract_min(None, 1, None, None, C.byref(n)) == pkg.PBH_EINVAL
    assert L.sssp(None, None, None, 4, 3, 0, None) == pkg.PBH_EINVAL
    assert b"NULL" in L.pbh_last_error()
    h = C.c_void_p()
    assert L.pbh_create(C.byref(h), 0, 2) == pkg.PBH_EINVAL
    assert L.pbh_create(C.byref(h), 10, 0) == pkg.PBH_EINVAL
    for bad in (pkg.PbhOpts(3, 0), pkg.PbhOpts(0, 2), pkg.PbhOpts(0, 0, (C.c_uint32 * 6)(1, 0, 0, 0, 0, 0))):
        assert L.pbh_create_ex(C.byref(h), 10, 2, C.byref(bad)) == pkg.PBH_EINVAL
    assert b"pbh_create_ex" in L.pbh_last_error()
    t = C.c_double(0.0)
    assert L.pbh_set_profiling(None, 1) == pkg.PBH_EINVAL
    assert L.pbh_merge_profile(None, C.byref(n), C.byref(n), C.byref(t)) == pkg.PBH_EINVAL
    assert L.pbh_traffic(None, C.byref(n)) == pkg.PBH_EINVAL


def test_sssp_rejects_bad_sizes_before_device_work():
    L = pkg.lib()
    dummy = C.c_void_p(0x1000)  # never dereferenced: the checks fail first
    assert L.sssp(dummy, dummy, dummy, 0, 0, 0, dummy) == pkg.PBH_EINVAL
    assert L.sssp(dummy, dummy, dummy, 5, 0, 5, dummy) == pkg.PBH_EINVAL
    assert b"source" in L.pbh_last_error()


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C layout: size and
    every field offset, as a C compiler lays them out from include/pbh.h."""
    import subprocess
    mirrors = {"pbh_opts": pkg.PbhOpts, "sssp_opts": pkg.SsspOpts, "sssp_stats": pkg.SsspStats,
               "sssp_query": pkg.SsspQuery, "sssp_nearfar_stats": pkg.NearFarStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pbh.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
