"""The boundary's ownership rules and options on the GPU: op_mask selects the
operator rows a build writes, and the autotuners' choices persist in a cache
file that a second process reads instead of tuning again."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_2102_02019_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_02019_amd import labfm

    labfm.lib()
    return torch.device("cuda:0")


def _setup(nodes, dev):
    from paper_2102_02019_amd import labfm

    x, y, h, s, m = (T(getattr(nodes, k), dev) for k in ("x", "y", "h", "s", "m"))
    rp, col = labfm.build_neighbours(x, y, h, nodes.box)
    return x, y, h, s, m, rp, col


@pytest.mark.parametrize("mode", [1, 2, 5])  # wavefront, workgroup, rows per node
def test_op_mask_writes_the_selected_rows(dev, mode):
    """Each subset build holds, in labfm_op order, exactly the rows (float64,
    float32 copy, row sums) of the full build, and the same kappa and
    statuses; nodes of orders 4, 6 and 8 are mixed."""
    from paper_2102_02019_amd import labfm

    nodes = inputs.jittered_lattice(40, seed=31, m=8)
    nodes.m = np.random.default_rng(2).choice(np.array([4, 6, 8], dtype=np.int8), nodes.n)
    x, y, h, s, m, rp, col = _setup(nodes, dev)
    prev = labfm.get_build_config()
    labfm.set_build_config(mode)
    try:
        full = labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, f32=False, rowsum=True,
                                   tiles=False)
        full32 = labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, f32=True, tiles=False)
        for mask in (0b100011, 0b011100, 0b000001, 0b100000):
            rows = [d for d in range(6) if mask >> d & 1]
            sub = labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, f32=True, rowsum=True,
                                      tiles=False, op_mask=mask)
            assert sub.w.shape == (len(rows), col.numel())
            assert torch.equal(sub.w, full.w[rows]), (mode, mask)
            assert torch.equal(sub.rowsum, full.rowsum[rows]), (mode, mask)
            assert torch.equal(sub.w32, full32.w32[rows]), (mode, mask)
            assert torch.equal(sub.kappa, full.kappa) and torch.equal(sub.status, full.status)
            if mask & 0b011100 == 0b011100:  # the float32 moments come with L, xx and xy
                assert torch.equal(sub.mom32, full32.mom32)
            else:
                assert sub.mom32 is None
            with pytest.raises(ValueError):
                sub._c()  # the gather calls need all six operators
    finally:
        labfm.set_build_config(*prev)


def test_op_mask_arguments_are_checked(dev):
    from paper_2102_02019_amd import labfm

    nodes = inputs.jittered_lattice(16, seed=3, m=4)
    x, y, h, s, m, rp, col = _setup(nodes, dev)
    for mask in (0, 0x40):
        with pytest.raises(labfm.LabfmError):
            labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, op_mask=mask, tiles=False)
    # the float32 moments need the L, xx and xy rows (checked before any work)
    P = labfm._ptr
    n, nnz = nodes.n, col.numel()
    w = torch.empty((3, nnz), dtype=torch.float64, device=dev)
    mom = torch.empty((labfm.NUM_MOM32, n), dtype=torch.float32, device=dev)
    kap = torch.empty(n, dtype=torch.float64, device=dev)
    st = torch.empty(n, dtype=torch.int8, device=dev)
    ws = torch.empty(labfm.lib().labfm_build_workspace_bytes(n), dtype=torch.uint8, device=dev)
    code = labfm.lib().labfm_build_weights(P(x), P(y), P(h), P(s), P(m), n,
                                           labfm._box(nodes.box), P(rp), P(col), nnz, 0b100011,
                                           P(w), None, P(mom), P(kap), None, P(st), P(ws),
                                           ws.numel(), labfm._stream())
    assert code == labfm.ERR_ARG
    assert b"mom32" in labfm.lib().labfm_last_error()


CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
import numpy as np, torch
from paper_2102_02019_amd import inputs, labfm
dev = torch.device("cuda:0")
T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
nodes = inputs.jittered_lattice(48, seed=41, m=6)
x, y, h, s, m = (T(getattr(nodes, k)) for k in ("x", "y", "h", "s", "m"))
rp, col = labfm.build_neighbours(x, y, h, nodes.box)
ops = labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, tune=True, tune_cache={path!r})
l, u, v = (np.zeros(nodes.n),) + inputs.taylor_green_state(nodes.x, nodes.y)[1:]
q = T(np.concatenate([l, u, v]))
best = labfm.tune(ops, q, labfm.F64, reps=2, cache_path={path!r})
print(json.dumps({{"build": list(labfm.build_weights.last_tuned), "tune": best}}))
"""


def _child(path):
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, path=str(path))],
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_tune_cache_is_read_by_a_second_process(dev, tmp_path):
    """The first process tunes the build and the gather kernels and writes
    the cache; a second process on the same node set finds every choice in
    the file and installs it without tuning."""
    path = tmp_path / "tune.json"
    first = _child(path)
    assert first["build"][3] is False and first["tune"]["cached"] is False
    text = path.read_text()
    entries = json.loads(text)
    assert sum(k.startswith("build/") for k in entries) == 1
    assert sum(k.startswith("launch/") for k in entries) == 3
    second = _child(path)
    assert second["build"][3] is True and second["tune"]["cached"] is True
    assert second["build"][:2] == first["build"][:2]
    for k in ("stage", "filter", "apply"):
        assert second["tune"][k][:2] == first["tune"][k][:2]
    # a cache hit leaves the file as it was
    assert path.read_text() == text
