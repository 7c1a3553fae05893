"""labfm_build_weights_noalloc (the weight build with its work list in the
library's static device scratch) against labfm_build_weights, through the
C ABI: identical outputs on two calls in a row, the second on a smaller node
set, and a clear error above the scratch's node limit."""
import ctypes

import numpy as np
import pytest

from paper_2102_02019_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_02019_amd import labfm

    labfm.lib()
    return torch.device("cuda:0")


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _outputs(n, nnz, dev):
    from paper_2102_02019_amd import labfm

    return {"w": torch.full((6, nnz), np.nan, dtype=torch.float64, device=dev),
            "w32": torch.full((6, labfm.w32_stride(nnz)), np.nan, dtype=torch.float32,
                              device=dev),
            "mom32": torch.full((6, n), np.nan, dtype=torch.float32, device=dev),
            "kappa": torch.full((n,), np.nan, dtype=torch.float64, device=dev),
            "rowsum": torch.full((6, n), np.nan, dtype=torch.float64, device=dev),
            "status": torch.full((n,), -1, dtype=torch.int8, device=dev)}


def _call(name, nodes, arr, rp, col, out):
    from paper_2102_02019_amd import labfm

    P = labfm._ptr
    fn = getattr(labfm.lib(), name)
    args = [P(arr["x"]), P(arr["y"]), P(arr["h"]), P(arr["s"]), P(arr["m"]), nodes.n,
            labfm._box(nodes.box), P(rp), P(col), col.numel(), 0x3F, P(out["w"]), P(out["w32"]),
            P(out["mom32"]), P(out["kappa"]), P(out["rowsum"]), P(out["status"])]
    if name == "labfm_build_weights":  # the allocating entry point takes a workspace
        ws = torch.empty(labfm.lib().labfm_build_workspace_bytes(nodes.n), dtype=torch.uint8,
                         device=rp.device)
        args += [P(ws), ws.numel()]
    return fn(*args, labfm._stream())


def _case(nodes, dev):
    from paper_2102_02019_amd import labfm

    arr = {k: T(getattr(nodes, k), dev) for k in ("x", "y", "h", "s", "m")}
    rp, col = labfm.build_neighbours(arr["x"], arr["y"], arr["h"], nodes.box)
    return arr, rp, col


@pytest.mark.parametrize("mode", [2, 3, 5])  # workgroup per node; persistent (uses the counter); rows
def test_noalloc_build_matches_allocating_build(dev, mode):
    from paper_2102_02019_amd import labfm

    prev = labfm._BuildConfig()
    assert labfm.lib().labfm_get_build_config(ctypes.byref(prev)) == 0
    assert labfm.lib().labfm_set_build_config(ctypes.byref(labfm._BuildConfig(mode, 0))) == 0
    try:
        big = inputs.jittered_lattice(64, seed=21, m=8)
        rng = np.random.default_rng(5)
        big.m = rng.choice(np.array([4, 6, 8], dtype=np.int8), big.n)
        small = inputs.jittered_lattice(24, seed=22, m=6)
        for nodes in (big, small):  # the second call on a smaller set
            arr, rp, col = _case(nodes, dev)
            ref = _outputs(nodes.n, col.numel(), dev)
            got = _outputs(nodes.n, col.numel(), dev)
            assert _call("labfm_build_weights", nodes, arr, rp, col, ref) == 0
            code = _call("labfm_build_weights_noalloc", nodes, arr, rp, col, got)
            assert code == 0, labfm.lib().labfm_last_error()
            torch.cuda.synchronize()
            for k in ref:
                a, b = got[k].cpu().numpy(), ref[k].cpu().numpy()
                assert np.array_equal(a, b, equal_nan=True), (nodes.n, k)
            assert int((got["status"] != 0).sum().item()) == 0
    finally:
        labfm.lib().labfm_set_build_config(ctypes.byref(prev))


def test_noalloc_rejects_more_nodes_than_its_scratch(dev):
    from paper_2102_02019_amd import labfm

    nodes = inputs.jittered_lattice(8, seed=1, m=4)
    arr, rp, col = _case(nodes, dev)
    out = _outputs(nodes.n, col.numel(), dev)
    P = labfm._ptr
    code = labfm.lib().labfm_build_weights_noalloc(
        P(arr["x"]), P(arr["y"]), P(arr["h"]), P(arr["s"]), P(arr["m"]),
        labfm.NOALLOC_MAX_NODES + 1, labfm._box(nodes.box), P(rp), P(col), col.numel(), 0x3F,
        P(out["w"]), P(out["w32"]), P(out["mom32"]), P(out["kappa"]), P(out["rowsum"]),
        P(out["status"]), labfm._stream())
    assert code == labfm.ERR_ARG
    assert b"maximum" in labfm.lib().labfm_last_error()
    # nothing was written
    assert int((out["status"] != -1).sum().item()) == 0
