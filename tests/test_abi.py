"""The C-ABI library loads and exports every function include/bdfx.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bdfx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bdfx_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("bdfx_create", "bdfx_mech_create", "bdfx_plan", "bdfx_bind", "bdfx_integrate",
              "bdfx_stats_summary", "bdfx_adjoint", "bdfx_perturb"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2405_01713_amd import bdfx
    if not os.path.exists(bdfx.LIB_PATH):
        pytest.skip("libbdfx.so not built")
    lib = ctypes.CDLL(bdfx.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(bdfx.EXPORTED) == set(_declared())
    assert bdfx.bdfx_version().startswith("bdfx")


def test_errors_without_device_are_loud():
    from paper_2405_01713_amd import bdfx
    if not os.path.exists(bdfx.LIB_PATH):
        pytest.skip("libbdfx.so not built")
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except Exception:
        pass
    with pytest.raises(bdfx.BdfxError):
        bdfx.bdfx_create(0, 0)
