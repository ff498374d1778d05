"""The C-ABI library loads and exports every entry point include/dsmc.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(dsmc_\w+|dig_\w+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2607_08195_amd import dsmc
    lib = ctypes.CDLL(dsmc.LIB_PATH)
    declared = _declared()
    assert "dsmc_init" in declared and "dsmc_step" in declared and "dsmc_sample" in declared
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_refuses_without_device():
    import pytest
    import torch
    from paper_2607_08195_amd import dsmc, workloads as W
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(RuntimeError):
        dsmc.Simulation(W.cavity(n_hex=2, ppc=2))
