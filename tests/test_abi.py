"""The C ABI: the library builds, loads and exports every declared symbol (CPU-only checks)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlmc.h")
LIB = os.path.join(ROOT, "paper_2503_05533_amd", "libmlmc.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mlmc_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_binding_exports():
    from paper_2503_05533_amd import EXPORTS
    assert sorted(EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libmlmc.so missing: run __graft_entry__.build()")
    import torch  # noqa: F401  (same HIP runtime as the binding)
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


def test_header_is_plain_c():
    txt = open(HEADER).read()
    assert 'extern "C"' in txt
    assert "torch" not in txt.lower().replace("pytorch", "")
    assert "hip_runtime" not in txt


def test_binding_refuses_without_gpu():
    import torch
    from paper_2503_05533_amd import MLMC, Config, MLMCError
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(MLMCError):
        MLMC(Config())
