"""The C-ABI library loads on a machine without a GPU and exports every entry
point that include/labfm.h declares (no compute calls are made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "labfm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(labfm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2102_02019_amd import labfm

    if not os.path.exists(labfm.LIB_PATH):
        pytest.fail("liblabfm.so is not built; run __graft_entry__.build()")
    return labfm.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("labfm_build_neighbours", "labfm_build_weights", "labfm_apply_operators",
                     "labfm_rk_step"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2102_02019_amd import labfm

    names = _declared()
    for name in names:
        assert hasattr(lib, name), name
    # the binding covers exactly the header's functions
    assert sorted(labfm.exported_symbols()) == names


def test_version_and_error_string(lib):
    assert b"gfx950" in lib.labfm_version()
    assert lib.labfm_last_error() is not None


def test_argument_errors_return_codes_without_gpu(lib):
    """Argument checks run on the host before any HIP call."""
    from paper_2102_02019_amd import labfm

    nnz = ctypes.c_int64(-1)
    box = labfm._Box(1.0, 1.0, 1, 1)
    code = lib.labfm_build_neighbours(None, None, None, 0, box, None, None, 0,
                                      ctypes.byref(nnz), None)
    assert code == labfm.ERR_ARG
    assert b"n must be positive" in lib.labfm_last_error()
    code = lib.labfm_apply_operators(None, 1, None, None, 0, None)
    assert code == labfm.ERR_ARG
    assert lib.labfm_rk_workspace_bytes(0) == 0
    assert lib.labfm_rk_workspace_bytes(1000) >= 6 * 1000 * 8


def test_oracle_and_product_are_separate():
    """The oracle imports nothing from the product package, and the product
    package (Python binding and sources) neither imports nor loads anything
    under oracle/."""
    odir = os.path.join(ROOT, "oracle")
    for f in os.listdir(odir):
        if f.endswith(".py"):
            text = open(os.path.join(odir, f)).read()
            assert "paper_2102_02019_amd" not in text, f
    pdir = os.path.join(ROOT, "paper_2102_02019_amd")
    for base, _, files in os.walk(pdir):
        if "_build" in base or "__pycache__" in base:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".c", ".h")):
                text = open(os.path.join(base, f)).read()
                assert not re.search(r"(import\s+oracle|from\s+oracle|oracle/|oracle\.)", text), \
                    os.path.join(base, f)
