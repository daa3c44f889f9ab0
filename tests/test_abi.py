"""The C-ABI library loads and exports every symbol declared in include/scc.h (CPU only)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "scc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(scc_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["scc_build_table", "scc_sample", "scc_classify", "scc_occ", "scc_export_level",
                 "scc_catalog", "scc_ags", "scc_table_destroy", "scc_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2009_03052_amd", "libscc.so"))
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    import paper_2009_03052_amd as scc
    assert set(declared_functions()) <= set(scc.exported_symbols())
    assert "gfx950" in scc.version()
    assert scc._lib.scc_num_unrooted(8) == 23
    assert scc._lib.scc_num_unrooted(9) == -1


def test_probe_rejects_bad_arguments():
    # argument checks only: every case returns before any device work
    import paper_2009_03052_amd as scc
    buf = (ctypes.c_uint64 * 64)()
    sink = (ctypes.c_uint64 * 1)()
    ms = ctypes.c_float(0)
    f = scc._lib.scc_probe_random_reads
    for nbytes, rb, n in [(512, 12, 4), (512, 0, 4), (512, 264, 4), (512, 64, -1), (512, 64, 1 << 30), (4, 64, 4)]:
        assert f(buf, nbytes, rb, n, 0, sink, None, ctypes.byref(ms)) == scc.EINVAL, (nbytes, rb, n)
    assert f(None, 512, 64, 4, 0, sink, None, ctypes.byref(ms)) == scc.EINVAL
