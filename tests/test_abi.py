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
    return sorted(set(re.findall(r"\b(bdfx_[A-Za-z0-9_]+)\s*\(", src)))


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


def _struct_fields(name):
    """Field names of `typedef struct { ... } name;` in include/bdfx.h, in order
    (arrays by their name)."""
    src = open(os.path.join(ROOT, "include", "bdfx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    end = re.search(r"\}\s*" + name + r"\s*;", src)
    assert end, name
    start = src.rfind("typedef struct {", 0, end.start())
    body = src[start + len("typedef struct {"):end.start()]
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        # "int64_t nst, nfe" / "const double *atol" / "int64_t status_count[11]"
        names = decl.split(",")
        first = re.findall(r"\**\s*([A-Za-z_]\w*)\s*(?:\[\d+\])?\s*$", names[0])
        fields.append(first[0])
        for n in names[1:]:
            fields.append(re.findall(r"([A-Za-z_]\w*)", n)[0])
    return fields


@pytest.mark.parametrize("cname,pyname", [("bdfx_options", "Options"), ("bdfx_mech_desc", "MechDesc"),
                                          ("bdfx_summary", "Summary"), ("bdfx_tuning", "Tuning")])
def test_binding_structs_follow_the_header(cname, pyname):
    """The ctypes structures of the binding list the header's fields, by name,
    in the header's order."""
    from paper_2405_01713_amd import bdfx
    assert [n for n, _ in getattr(bdfx, pyname)._fields_] == _struct_fields(cname)


def test_cell_stats_dtype_follows_the_header():
    from paper_2405_01713_amd import bdfx
    assert list(bdfx.STATS_DTYPE.names) == _struct_fields("bdfx_cell_stats")
    assert bdfx.STATS_DTYPE.itemsize == 56


@pytest.mark.parametrize("cname,pyname", [("orc_opts", "Opts"), ("orc_stats", "Stats"),
                                          ("orc_mech", "Mech"), ("orc_record", "Record")])
def test_oracle_binding_structs_follow_its_source(cname, pyname):
    """Same check for the oracle's structures (test infrastructure)."""
    from oracle import oracle as O
    src = open(os.path.join(ROOT, "oracle", "bdf_oracle.c")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    end = re.search(r"\}\s*" + cname + r"\s*;", src)
    start = src.rfind("typedef struct {", 0, end.start())
    fields = []
    for decl in src[start + len("typedef struct {"):end.start()].split(";"):
        decl = decl.strip()
        if decl:
            parts = decl.split(",")
            fields.append(re.findall(r"([A-Za-z_]\w*)\s*(?:\[\d+\])?\s*$", parts[0])[0])
            fields += [re.findall(r"([A-Za-z_]\w*)", p)[0] for p in parts[1:]]
    assert [n for n, _ in getattr(O, pyname)._fields_] == fields
