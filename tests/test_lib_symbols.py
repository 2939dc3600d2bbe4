"""The C-ABI library loads and exports every entry point include/sgp.h declares
(no compute: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgp.h")
LIB = os.path.join(ROOT, "paper_2410_04512_amd", "libsgp.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sgp_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_chain():
    names = declared()
    for f in ("sgp_collide", "sgp_assemble_gamma", "sgp_build_tree", "sgp_factor_tree", "sgp_pcg_solve"):
        assert f in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_2410_04512_amd import build
        build.build()
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_gpu():
    import torch
    import paper_2410_04512_amd as P
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        P.Context()
