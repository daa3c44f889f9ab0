"""The binding's ctypes structures against the C structures of include/scc.h:
every size and member offset as the host C compiler lays them out (a C program
built from the header prints them), so that a member added on one side only
fails here rather than shifting the fields that follow it."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

import paper_2009_03052_amd as scc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [
    (scc._Allocator, "scc_allocator"),
    (scc._Csr, "scc_csr"),
    (scc._BuildOpts, "scc_build_opts"),
    (scc._Instance, "scc_instance"),
    (scc._BatchOpts, "scc_batch_opts"),
    (scc.BatchReport, "scc_batch_report"),
    (scc.TableInfo, "scc_table_info"),
    (scc._Build16Opts, "scc16_build_opts"),
    (scc.Table16Info, "scc16_table_info"),
    (scc._ServerOpts, "scc_server_opts"),
    (scc._Request, "scc_request"),
    (scc._Result, "scc_result"),
    (scc.ServerStats, "scc_server_stats"),
]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "scc.h"', "int main(void) {"]
    for cls, cname in PAIRS:
        lines.append(f'    printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'    printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["    return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {a: int(b) for a, b in (ln.split() for ln in out.splitlines())}


@pytest.mark.parametrize("cls,cname", PAIRS, ids=[c for _, c in PAIRS])
def test_struct_layout_matches_header(c_layout, cls, cname):
    assert C.sizeof(cls) == c_layout[cname], cname
    for f, _ in cls._fields_:
        assert getattr(cls, f).offset == c_layout[f"{cname}.{f}"], f"{cname}.{f}"
