"""CPU-side checks of the C ABI: the library loads, exports every declared symbol
and refuses NULL handles.

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


# Every entry point that takes a handle, called with NULL ones: each must
# refuse with CSTM_EINVAL and a message, before any device work (so this runs
# without a GPU), and the void ones must ignore NULL.
_NULL_CALLS = {
    "cstm_ctx_get_tune": (None, None),
    "cstm_ctx_set_tune": (None, None),
    "cstm_ctx_lds_bytes": (None, None),
    "cstm_ctx_last_enum_stats": (None, None),
    "cstm_graph_load": (None, 0, 0, None, None, None, 0, None, None),
    "cstm_graph_info": (None, None, None, None, None),
    "cstm_graph_label_edges": (None, None, 0, None),
    "cstm_cst_build": (None, None, 1, None, 0, None, None, None),
    "cstm_cst_build_ordered": (None, None, 1, None, 0, None, None, None, None),
    "cstm_cst_estimate": (None, 1, None, 0, None, None),
    "cstm_cst_partition": (None, 0, 0, 0, None),
    "cstm_cst_workload": (None, None),
    "cstm_cst_info_get": (None, None),
    "cstm_cst_candidates": (None, 0, None, 0, None),
    "cstm_cst_times": (None, None, None, None),
    "cstm_enumerate": (None, 0, 0, None, 0, None, None, 0.0, None),
    "cstm_batch_enumerate": (None, 0, None, None, None, None),
    "cstm_enumerate_noalloc": (None, 0, None, 0.0, None),
    "cstm_enumerate_shared": (None, 0.0, 0, 0, None, None, None),
    "cstm_server_create": (None, None, 1, 0, 0, 0, 0, None),
    "cstm_server_submit": (None, 1, None, 0, None, 0, None),
    "cstm_server_poll": (None, 1, None),
    "cstm_server_wait": (None, 1, 0.0, None),
    "cstm_server_get_stats": (None, None),
}


def test_null_handles_are_refused_before_any_device_work():
    from paper_2102_10768_amd import cstm

    lib = cstm.load_library()
    for name, args in _NULL_CALLS.items():
        assert getattr(lib, name)(*args) == cstm.EINVAL, name
        assert lib.cstm_last_error(), name
    for name in ("cstm_ctx_destroy", "cstm_graph_free", "cstm_cst_free", "cstm_server_destroy"):
        getattr(lib, name)(None)
    # every status-returning entry point that takes a handle is covered
    takes_handle = {n for n in declared_symbols()
                    if n not in ("cstm_ctx_create", "cstm_last_error", "cstm_version")
                    and not n.endswith(("_destroy", "_free"))}
    assert takes_handle == set(_NULL_CALLS)
