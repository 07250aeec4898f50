"""CPU-only checks of the C-ABI library: it loads and exports every entry point include/chfsi.h
declares (no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chfsi.h")
LIB = os.path.join(ROOT, "paper_1206_3768_amd", "libchfsi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chfsi_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["chfsi_create", "chfsi_destroy", "chfsi_solve", "chfsi_solve_batched", "chfsi_filter",
                     "chfsi_set_degree_model", "chfsi_get_trace", "chfsi_status_string"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libchfsi.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libchfsi.so not built")
def test_binding_lists_every_declared_symbol():
    from paper_1206_3768_amd import chfsi
    assert sorted(chfsi.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libchfsi.so not built")
def test_default_params_follow_table3():
    # Table 3 (parameter settings of ChFSI): degree 25, TOL 1e-10, blk = nev + 40
    import json
    from paper_1206_3768_amd import chfsi
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "table3_chfsi_parameters.json")))
    p = chfsi.default_params()
    assert p.deg == gold["deg"]
    assert p.tol == gold["tol"]
    assert p.nex == gold["blk_minus_nev"]
    assert gold["lanczos_iter_min"] <= p.lanczos_steps
    lib = chfsi.load()
    assert lib.chfsi_status_string(2) == b"S is not Hermitian positive definite"
