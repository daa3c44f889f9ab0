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
