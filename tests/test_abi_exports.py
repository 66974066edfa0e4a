"""The C-ABI library loads without a GPU and exports every declared symbol."""
import ctypes
import glob
import os
import re

from helpers import ROOT

LIB = os.path.join(ROOT, "paper_2411_10143_amd", "libcaskrylov.so")


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\**\s+\**(\w+)\s*\(", text,
                             flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def ensure_built():
    if not os.path.exists(LIB):
        from paper_2411_10143_amd import build
        build.build()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["spmv_create", "spmv_features", "spmv_select", "spmv_convert", "spmv_apply",
              "cg_solve", "gmres_solve", "spmv_destroy", "ck_last_error"]:
        assert n in names, n


def test_library_exports_every_declared_symbol():
    ensure_built()
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_calls_work_without_gpu():
    ensure_built()
    import paper_2411_10143_amd as ck
    for i in range(ck.NUM_CONFIGS):
        c = ck.config_from_id(i)
        assert ck.config_id(c) == i
        assert ck.kernel_name(c).startswith("spmv_")
    try:
        ck.config_from_id(ck.NUM_CONFIGS)
        raise AssertionError("expected an error")
    except ck.CkError as e:
        assert e.status == ck.CK_E_INVALID
    f = ck.Features()
    f.nrows, f.ncols, f.nnz = 100, 100, 500
    c = ck.spmv_select(f)
    assert c.format in (0, 1, 2) and 1 <= c.stages_done <= 3
