"""The C-ABI library loads on a machine without a GPU and exports every
function include/rif.h declares; the Python binding declares the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rif.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:unsigned\s+)?(?:long\s+)*[A-Za-z_][A-Za-z0-9_]*(?:\s+|\s*\*+\s*)([a-z_0-9]+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_four_hot_path_calls():
    names = declared_functions()
    for n in ("rif_transform", "rif_jk_mo", "rif_jk_ao_per_mo", "pnof7_energy_grad"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2012_15662_amd as rif
    if not os.path.exists(rif.LIB_PATH):
        pytest.fail("librif.so is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(rif.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_binding_covers_header():
    import paper_2012_15662_amd as rif
    assert sorted(rif.EXPORTS) == declared_functions()


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_2012_15662_amd as rif
    with pytest.raises(ValueError):
        rif._ptr(torch.zeros(4, dtype=torch.float64), "x", torch.float64)
