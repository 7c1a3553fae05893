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
                                      ctypes.byref(nnz), None, 0, None)
    assert code == labfm.ERR_ARG
    assert b"n must be positive" in lib.labfm_last_error()
    code = lib.labfm_apply_operators(None, 1, None, None, 0, None)
    assert code == labfm.ERR_ARG
    assert lib.labfm_rk_workspace_bytes(0) == 0
    assert lib.labfm_rk_workspace_bytes(1000) >= 6 * 1000 * 8
    # the LU on given systems: order, count and buffers (count 0 does nothing)
    for m, count in ((0, 1), (11, 1), (4, -1), (4, 1)):
        assert lib.labfm_solve_systems(m, None, count, None, None, None, None) == labfm.ERR_ARG
    assert lib.labfm_solve_systems(4, None, 0, None, None, None, None) == labfm.OK


def test_calls_refuse_a_missing_or_short_workspace(lib):
    """Every call that needs temporary device memory takes it from the
    caller: a NULL or short workspace is an argument error, reported on the
    host before any device work (the other pointers here are never
    dereferenced)."""
    from paper_2102_02019_amd import labfm

    fake = ctypes.c_void_p(4096)  # stands in for device pointers
    box = labfm._Box(1.0, 1.0, 1, 1)
    n = 1000
    nnz = ctypes.c_int64(0)
    hmax = ctypes.c_int32(0)
    dt = ctypes.c_double(0.0)
    calls = {
        "morton_order": lambda ws, b: lib.labfm_morton_order(
            fake, fake, n, box, 0.1, fake, ws, b, None),
        "build_neighbours": lambda ws, b: lib.labfm_build_neighbours(
            fake, fake, fake, n, box, fake, fake, 10, ctypes.byref(nnz), ws, b, None),
        "build_weights": lambda ws, b: lib.labfm_build_weights(
            fake, fake, fake, fake, fake, n, box, fake, fake, 10, 0x3F, fake, None, None, fake,
            None, fake, ws, b, None),
        "optimise_stencils": lambda ws, b: lib.labfm_optimise_stencils(
            fake, fake, fake, fake, fake, n, box, fake, fake, 10, None, fake, None, ws, b, None),
        "build_tiles": lambda ws, b: lib.labfm_build_tiles(
            fake, fake, n, 10, fake, fake, fake, ctypes.byref(hmax), ws, b, None),
        "time_step": lambda ws, b: lib.labfm_time_step(
            fake, fake, n, 1.0, 1.0, 1.0, 0.4, ctypes.byref(dt), ws, b, None),
    }
    sizes = {"morton_order": lib.labfm_morton_workspace_bytes(n),
             "build_neighbours": lib.labfm_neighbours_workspace_bytes(n),
             "build_weights": lib.labfm_build_workspace_bytes(n),
             "optimise_stencils": lib.labfm_optimise_workspace_bytes(n, 10),
             "build_tiles": lib.labfm_tiles_workspace_bytes(),
             "time_step": lib.labfm_time_step_workspace_bytes()}
    for name, call in calls.items():
        need = sizes[name]
        assert need > 0, name
        for ws, b in ((None, need), (fake, need - 1)):
            assert call(ws, b) == labfm.ERR_ARG, name
            assert b"workspace" in lib.labfm_last_error(), name
    assert lib.labfm_build_workspace_bytes(n) >= 4 * n
    assert lib.labfm_transpose_workspace_bytes(n, 5000) >= 4 * (2 * (n + 1) + 5000)
    assert lib.labfm_boundary_workspace_bytes(n) >= 5 * n


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
