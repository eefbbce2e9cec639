"""CPU-side checks of the C ABI: the library loads and exports every declared symbol.

No compute call is made here (there is no GPU on the build host).
"""

from __future__ import annotations

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols() -> list[str]:
    src = open(os.path.join(ROOT, "include", "cstm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cstm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_api():
    names = declared_symbols()
    for must in ("cstm_graph_load", "cstm_cst_build", "cstm_cst_partition", "cstm_enumerate", "cstm_batch_enumerate"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2102_10768_amd import cstm

    lib = cstm.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(cstm.EXPORTS) == set(declared_symbols())
    assert b"gfx950" in lib.cstm_version()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2102_10768_amd import cstm

    monkeypatch.setattr(cstm, "_lib", None)
    monkeypatch.setattr(cstm, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        cstm.load_library()


def test_library_is_built_for_gfx950_only():
    lib = os.path.join(ROOT, "paper_2102_10768_amd", "libcstm.so")
    data = open(lib, "rb").read()
    assert b"gfx950" in data
    for other in (b"gfx90a", b"gfx942", b"gfx1100"):
        assert b"amdgcn-amd-amdhsa--" + other not in data


def test_context_creation_without_gpu_reports_an_error():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2102_10768_amd import cstm

    with pytest.raises(cstm.CstmError):
        cstm.Context(0)


def test_one_hip_runtime_per_process():
    from paper_2102_10768_amd import cstm

    cstm.load_library()
    maps = open("/proc/self/maps").read().splitlines()
    hip = {line.split()[-1] for line in maps if "libamdhip64" in line}
    assert len(hip) == 1, hip
