"""The FP64 oracle over large node sets, spread over worker processes.

Test infrastructure: each worker owns a contiguous range of nodes and runs the
oracle's own routines on it (``weights_batched`` for its rows, then
``ns_rhs`` and ``filter_fields`` on a copy of the operators whose other rows
are empty). Every row of the CSR is computed by exactly the arithmetic the
serial oracle applies to it (row sums in ascending j, the same per-node
solve), so the assembled results equal the serial oracle's bit for bit; the
time loop is the oracle's ``rk_integrate`` with the right-hand side and the
filter gathered from the workers.

Workers are started with the "spawn" method (never forked from a process
that may hold a GPU context) and exchange fields through memory-mapped
files, so each stage moves only the 3 x N state and the 3 x N rates.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import tempfile

import numpy as np


def _worker(conn, tmpdir, lo, hi, m, box, prm_tuple):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np  # noqa: F811

    from oracle import labfm_oracle as O

    def load(name):
        return np.load(os.path.join(tmpdir, name + ".npy"), mmap_mode="r")

    x, y, h, s = (np.asarray(load(k)) for k in ("x", "y", "h", "s"))
    rp_full = np.asarray(load("row_ptr"))
    col_full = load("col")
    N = x.size
    a, b = int(rp_full[lo]), int(rp_full[hi])
    # operators whose rows outside [lo, hi) are empty
    rp = np.zeros(N + 1, dtype=rp_full.dtype)
    rp[lo + 1:hi + 1] = rp_full[lo + 1:hi + 1] - a
    rp[hi + 1:] = b - a
    col = np.array(col_full[a:b])
    W = O.weights_batched(x, y, h, s, m, rp, col, box, start=lo, stop=hi)
    W.update(row_ptr=rp, col=col)
    state = np.load(os.path.join(tmpdir, "state.npy"), mmap_mode="r")
    out = np.load(os.path.join(tmpdir, "out.npy"), mmap_mode="r+")
    conn.send(("built", W["kappa"][lo:hi].copy(), W["status"][lo:hi].copy()))

    class Prm:
        pass

    prm = Prm()
    prm.c2, prm.mu, prm.gx, prm.gy = prm_tuple
    while True:
        cmd = conn.recv()
        if cmd == "stop":
            break
        f = tuple(np.array(state[k]) for k in range(3))
        if cmd == "rhs":
            r = O.ns_rhs(*f, W, prm)
        elif cmd == "filter":
            r = O.filter_fields(f, W)
        elif cmd == "weights":
            conn.send(W["w"][:, :].copy())
            continue
        else:
            raise ValueError(cmd)
        for k in range(3):
            out[k, lo:hi] = r[k][lo:hi]
        out.flush()
        conn.send("done")
    conn.close()


class OraclePool:
    """Oracle operators of a uniform-order node set, held by `workers`
    processes; ``rk_run`` matches ``labfm_oracle.rk_run``."""

    def __init__(self, nodes, row_ptr, col, prm, workers: int = 16):
        self.n = nodes.n
        self._tmp = tempfile.TemporaryDirectory(prefix="oracle_pool_")
        d = self._tmp.name
        for k, v in (("x", nodes.x), ("y", nodes.y), ("h", nodes.h), ("s", nodes.s),
                     ("row_ptr", row_ptr), ("col", col)):
            np.save(os.path.join(d, k + ".npy"), np.ascontiguousarray(v))
        np.save(os.path.join(d, "state.npy"), np.zeros((3, self.n)))
        np.save(os.path.join(d, "out.npy"), np.zeros((3, self.n)))
        m = int(np.asarray(nodes.m).flat[0])
        assert np.all(np.asarray(nodes.m) == m), "uniform order only"
        workers = max(1, min(workers, self.n))
        cuts = np.linspace(0, self.n, workers + 1).astype(int)
        ctx = mp.get_context("spawn")
        self._conns, self._procs = [], []
        self.kappa = np.empty(self.n)
        self.status = np.empty(self.n, dtype=np.int8)
        prm_tuple = (float(prm.c2), float(prm.mu), float(getattr(prm, "gx", 0.0)),
                     float(getattr(prm, "gy", 0.0)))
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            parent, child = ctx.Pipe()
            p = ctx.Process(target=_worker, args=(child, d, int(lo), int(hi), m, nodes.box,
                                                  prm_tuple), daemon=True)
            p.start()
            self._conns.append(parent)
            self._procs.append(p)
        for (lo, hi), c in zip(zip(cuts[:-1], cuts[1:]), self._conns):
            tag, kap, st = c.recv()
            assert tag == "built"
            self.kappa[lo:hi] = kap
            self.status[lo:hi] = st
        self._state = np.load(os.path.join(d, "state.npy"), mmap_mode="r+")
        self._out = np.load(os.path.join(d, "out.npy"), mmap_mode="r")

    def _eval(self, cmd, fields):
        for k in range(3):
            self._state[k, :] = fields[k]
        self._state.flush()
        for c in self._conns:
            c.send(cmd)
        for c in self._conns:
            assert c.recv() == "done"
        return tuple(np.array(self._out[k]) for k in range(3))

    def ns_rhs(self, l, u, v):
        return self._eval("rhs", (l, u, v))

    def filter_fields(self, fields):
        return self._eval("filter", fields)

    def rk_run(self, l, u, v, dt: float, n_steps: int, filt: bool = True):
        from oracle import labfm_oracle as O

        post = self.filter_fields if filt else None
        return O.rk_integrate((l, u, v), self.ns_rhs, dt, n_steps, post)

    def close(self):
        for c in self._conns:
            try:
                c.send("stop")
            except (BrokenPipeError, OSError):
                pass
        for p in self._procs:
            p.join(timeout=10)
            if p.is_alive():
                p.terminate()
        self._tmp.cleanup()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
