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


STRUCTS = [("_Config", "mlmc_config"), ("_LevelOpts", "mlmc_level_opts"), ("_LevelStats", "mlmc_level_stats"),
           ("_Result", "mlmc_result"), ("_MCMCConfig", "mlmc_mcmc_config"), ("_MCMCResult", "mlmc_mcmc_result"),
           ("_MIMCConfig", "mlmc_mimc_config"), ("_MIMCResult", "mlmc_mimc_result"),
           ("_EstimateState", "mlmc_estimate_state")]


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes mirror has the size and field offsets the C compiler gives
    the header's struct (a field added, dropped or reordered on one side only
    fails here)."""
    import shutil
    import subprocess
    from paper_2503_05533_amd import mlmc as M
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mlmc.h"', "int main(void) {"]
    for py, c in STRUCTS:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (c, c))
        for name, _ in getattr(M, py)._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (c, name, c, name))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for py, c in STRUCTS:
        cls = getattr(M, py)
        assert int(got["%s size" % c]) == ctypes.sizeof(cls), c
        for name, _ in cls._fields_:
            assert int(got["%s %s" % (c, name)]) == getattr(cls, name).offset, (c, name)
