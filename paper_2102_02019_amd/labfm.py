"""Python binding of liblabfm.so (the gfx950 LABFM library).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/labfm.h. Tensors must be
contiguous HIP device tensors; work is enqueued on torch's current stream.
There is no CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; LABFM_LIBRARY may name another build of the same sources
LIB_PATH = os.environ.get("LABFM_LIBRARY") or os.path.join(_HERE, "liblabfm.so")

OPS = ("x", "y", "L", "xx", "xy", "hyp")
NUM_OPS = len(OPS)
OP_X, OP_Y, OP_L, OP_XX, OP_XY, OP_HYP = range(6)
F64, F32W, F32_COMP = 0, 1, 2

KERNEL_STAGE, KERNEL_FILTER, KERNEL_APPLY = 0, 1, 2
NUM_MOM32 = 6  # rows of the float32-weight first moments: (L,x) (L,y) (xx,x) (xx,y) (xy,x) (xy,y)
BUILD_WAVE, BUILD_BLOCK, BUILD_PERSISTENT, BUILD_BUCKETED, BUILD_ROWS = 1, 2, 3, 4, 5
XCD_ORDER, STREAMING = 1, 2
OK, ERR_ARG, ERR_HIP, ERR_CAPACITY, ERR_NONFINITE, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
NODE_OK, NODE_SINGULAR, NODE_FEW_NEIGHBOURS, NODE_BAD_FILTER, NODE_BAD_ORDER = range(5)


class LabfmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"labfm error {code}: {msg}")
        self.code = code


class NodeStatusError(RuntimeError):
    """Weight builds left nodes with a failure status (LABFM_NODE_SINGULAR,
    _FEW_NEIGHBOURS, _BAD_FILTER or _BAD_ORDER); ``counts`` holds the node
    builds per status, LABFM_NODE_OK first."""

    def __init__(self, counts):
        super().__init__("node builds with a failure status (singular, few neighbours, "
                         f"bad filter, bad order): {list(counts[1:])}")
        self.counts = list(counts)


class _Box(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
                ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32)]


class _Tiles(ctypes.Structure):
    _fields_ = [("ntiles", ctypes.c_int32), ("max_halo", ctypes.c_int32),
                ("halo_count", ctypes.c_void_p), ("halo_idx", ctypes.c_void_p),
                ("lcol", ctypes.c_void_p)]


class _Operators(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("w32", ctypes.c_void_p),
                ("mom32", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
                ("tiles", ctypes.POINTER(_Tiles)), ("wall_normal", ctypes.c_void_p)]


class _LagrangianStats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int32), ("builds", ctypes.c_int64),
                ("max_nnz", ctypes.c_int64), ("build_ms", ctypes.c_double),
                ("stage_ms", ctypes.c_double), ("node_status", ctypes.c_int64 * 5)]


class _Strips(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("column", ctypes.c_void_p),
                ("normal", ctypes.c_void_p)]


class _RKParams(ctypes.Structure):
    _fields_ = [("c2", ctypes.c_double), ("mu", ctypes.c_double),
                ("gx", ctypes.c_double), ("gy", ctypes.c_double),
                ("dt", ctypes.c_double), ("filter", ctypes.c_int32),
                ("check_finite", ctypes.c_int32)]


class _LaunchConfig(ctypes.Structure):
    _fields_ = [("lanes_per_node", ctypes.c_int32), ("flags", ctypes.c_int32)]


class _StencilOptParams(ctypes.Structure):
    _fields_ = [("shrink", ctypes.c_double), ("gain_max", ctypes.c_double),
                ("res_coef", ctypes.c_double), ("max_iter", ctypes.c_int32)]


class _Transpose(ctypes.Structure):
    _fields_ = [("tptr", ctypes.c_void_p), ("tsrc", ctypes.c_void_p), ("tw", ctypes.c_void_p),
                ("rowsum", ctypes.c_void_p)]


class _BuildConfig(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("workgroups_per_cu", ctypes.c_int32)]


class _Timing(ctypes.Structure):
    _fields_ = [("stage_ms", ctypes.c_double), ("filter_ms", ctypes.c_double),
                ("stage_launches", ctypes.c_int64), ("filter_launches", ctypes.c_int64),
                ("every", ctypes.c_int32)]


_P = ctypes.c_void_p
_SIGNATURES = {
    "labfm_last_error": (ctypes.c_char_p, []),
    "labfm_w32_stride": (ctypes.c_int64, [ctypes.c_int64]),
    "labfm_version": (ctypes.c_char_p, []),
    "labfm_morton_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "labfm_morton_order": (ctypes.c_int, [_P, _P, ctypes.c_int32, _Box, ctypes.c_double, _P, _P,
                                          ctypes.c_size_t, _P]),
    "labfm_neighbours_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "labfm_build_neighbours": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _Box, _P, _P,
                                              ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _P,
                                              ctypes.c_size_t, _P]),
    "labfm_build_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "labfm_optimise_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int64]),
    "labfm_build_weights": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32, _Box, _P, _P,
                                           ctypes.c_int64, ctypes.c_uint32, _P, _P, _P, _P, _P,
                                           _P, _P, ctypes.c_size_t, _P]),
    "labfm_build_weights_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32, _Box, _P,
                                                   _P, ctypes.c_int64, ctypes.c_uint32, _P, _P,
                                                   _P, _P, _P, _P, _P]),
    "labfm_solve_systems": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.c_int32, _P, _P, _P, _P]),
    "labfm_apply_operators": (ctypes.c_int, [ctypes.POINTER(_Operators), ctypes.c_uint32, _P, _P,
                                             ctypes.c_int, _P]),
    "labfm_time_step_workspace_bytes": (ctypes.c_size_t, []),
    "labfm_time_step": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_double), _P, ctypes.c_size_t,
                                       _P]),
    "labfm_ns_rhs": (ctypes.c_int, [_P, ctypes.POINTER(_Operators), ctypes.POINTER(_RKParams), _P,
                                    ctypes.c_int, _P]),
    "labfm_tile_count": (ctypes.c_int32, [ctypes.c_int32]),
    "labfm_mfma_f64_rate_scratch_bytes": (ctypes.c_size_t, []),
    "labfm_mfma_f64_rate": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.c_size_t,
                                           ctypes.POINTER(ctypes.c_double), _P]),
    "labfm_tiles_workspace_bytes": (ctypes.c_size_t, []),
    "labfm_build_tiles": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int64, _P, _P, _P,
                                         ctypes.POINTER(ctypes.c_int32), _P, ctypes.c_size_t,
                                         _P]),
    "labfm_transpose_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int64]),
    "labfm_build_transpose": (ctypes.c_int, [ctypes.POINTER(_Operators), _P, _P, _P, _P,
                                             ctypes.c_size_t, _P]),
    "labfm_adjoint_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32,
                                                        ctypes.c_int32]),
    "labfm_rk_adjoint": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(_Operators),
                                        ctypes.POINTER(_Transpose), ctypes.POINTER(_RKParams),
                                        ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_size_t, _P]),
    "labfm_boundary_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "labfm_boundary_weights": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, _Box, _P, _P,
                                              ctypes.c_int64, ctypes.POINTER(_Strips), _P, _P,
                                              _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "labfm_lagrangian_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int64]),
    "labfm_lagrangian_step": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.c_int32, _Box,
                                             ctypes.POINTER(_RKParams), ctypes.c_int32,
                                             ctypes.c_int64, _P, ctypes.c_size_t,
                                             ctypes.POINTER(_LagrangianStats), _P]),
    "labfm_set_build_config": (ctypes.c_int, [ctypes.POINTER(_BuildConfig)]),
    "labfm_get_build_config": (ctypes.c_int, [ctypes.POINTER(_BuildConfig)]),
    "labfm_optimise_stencils": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32, _Box, _P, _P,
                                               ctypes.c_int64,
                                               ctypes.POINTER(_StencilOptParams), _P, _P, _P,
                                               ctypes.c_size_t, _P]),
    "labfm_tune_build": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int32, _Box, _P, _P,
                                        ctypes.c_int64, ctypes.c_uint32, _P, _P, _P, _P, _P, _P,
                                        _P, ctypes.c_size_t, ctypes.c_char_p,
                                        ctypes.POINTER(_BuildConfig),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int32), _P]),
    "labfm_rk_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "labfm_get_launch_config": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int, ctypes.c_int32,
                                               ctypes.c_int64, ctypes.POINTER(_LaunchConfig)]),
    "labfm_set_launch_config": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int,
                                               ctypes.POINTER(_LaunchConfig)]),
    "labfm_tune": (ctypes.c_int, [ctypes.POINTER(_Operators), _P, ctypes.c_int, ctypes.c_int32, _P,
                                  ctypes.c_size_t, ctypes.c_char_p, ctypes.POINTER(_LaunchConfig),
                                  ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int32), _P]),
    "labfm_rk_step": (ctypes.c_int, [_P, ctypes.POINTER(_Operators), ctypes.POINTER(_RKParams),
                                     ctypes.c_int32, ctypes.c_int, ctypes.c_int32, _P,
                                     ctypes.c_size_t, ctypes.POINTER(_Timing), _P]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load liblabfm.so (built in-tree by ``__graft_entry__.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        # the tile size is compiled into the library (LABFM_TILE_NODES)
        if L.labfm_tile_count(TILE_NODES) != 1 or L.labfm_tile_count(TILE_NODES + 1) != 2:
            raise RuntimeError(f"{LIB_PATH} was built for another tile size than "
                               f"TILE_NODES = {TILE_NODES}")
        _lib = L
    return _lib


def exported_symbols() -> list:
    return list(_SIGNATURES)


def _check(code: int) -> None:
    if code != OK:
        raise LabfmError(code, lib().labfm_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("labfm expects HIP device tensors")
    if not t.is_contiguous():
        raise ValueError("labfm expects contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _w32_ptr(t: Optional[torch.Tensor]):
    """Pointer of a float32 weight copy held as the (rows, nnz) view of rows
    at the padded stride labfm_w32_stride(nnz)."""
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2:
        raise ValueError("labfm expects float32 weights of shape (rows, nnz) on the device")
    if t.stride() != (w32_stride(t.shape[1]), 1):
        raise ValueError("float32 weight rows must use the stride labfm_w32_stride(nnz)")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(nbytes: int, device) -> torch.Tensor:
    """A device workspace of nbytes bytes (allocated by torch on the current
    stream: the library's work on that stream may use it after the call)."""
    return torch.empty(max(1, int(nbytes)), dtype=torch.uint8, device=device)


def _cache_arg(path: Optional[str]):
    return None if path is None else os.fspath(path).encode()


def _box(box) -> _Box:
    return _Box(float(box.Lx), float(box.Ly), int(bool(box.periodic_x)), int(bool(box.periodic_y)))


def version() -> str:
    return lib().labfm_version().decode()


# ---------------------------------------------------------------------------

def morton_order(x: torch.Tensor, y: torch.Tensor, box, cell: float) -> torch.Tensor:
    """Z-order permutation (int32[n]) of the nodes' cells of side ``cell``."""
    n = x.numel()
    perm = torch.empty(n, dtype=torch.int32, device=x.device)
    ws = _workspace(lib().labfm_morton_workspace_bytes(n), x.device)
    _check(lib().labfm_morton_order(_ptr(x), _ptr(y), n, _box(box), float(cell), _ptr(perm),
                                    _ptr(ws), ws.numel(), _stream()))
    return perm


def build_neighbours(x: torch.Tensor, y: torch.Tensor, h: torch.Tensor, box):
    """CSR stencils (row_ptr int32[n+1], col int32[nnz]) on the device."""
    n = x.numel()
    row_ptr = torch.empty(n + 1, dtype=torch.int32, device=x.device)
    nnz = ctypes.c_int64(0)
    ws = _workspace(lib().labfm_neighbours_workspace_bytes(n), x.device)
    code = lib().labfm_build_neighbours(_ptr(x), _ptr(y), _ptr(h), n, _box(box), _ptr(row_ptr),
                                        None, 0, ctypes.byref(nnz), _ptr(ws), ws.numel(),
                                        _stream())
    if code != ERR_CAPACITY:
        _check(code)
    col = torch.empty(max(1, nnz.value), dtype=torch.int32, device=x.device)
    code = lib().labfm_build_neighbours(_ptr(x), _ptr(y), _ptr(h), n, _box(box), _ptr(row_ptr),
                                        _ptr(col), col.numel(), ctypes.byref(nnz), _ptr(ws),
                                        ws.numel(), _stream())
    _check(code)
    return row_ptr, col[: nnz.value]


@dataclass
class Operators:
    """Device-resident operators of one node set."""

    row_ptr: torch.Tensor
    col: torch.Tensor
    w: Optional[torch.Tensor]       # float64 (6, nnz): one row per operator of op_mask
    w32: Optional[torch.Tensor]     # float32 (6, nnz) view of rows at labfm_w32_stride(nnz)
    kappa: torch.Tensor             # float64 (n,)
    mom32: Optional[torch.Tensor] = None  # float32 (6, n) first moments of w32
    rowsum: Optional[torch.Tensor] = None
    status: Optional[torch.Tensor] = None
    # node tiles (labfm_build_tiles): halo_count, halo_idx, lcol, max_halo
    tiles: Optional[tuple] = None
    use_tiles: bool = True
    # transposed stencils for the adjoint (labfm_build_transpose): tptr, tsrc, tw
    transpose: Optional[tuple] = None
    # float64 (n, 2) inward normal at no-slip wall nodes, zero elsewhere
    # (labfm_boundary_weights)
    wall_normal: Optional[torch.Tensor] = None
    # operators whose weights w, w32 and rowsum hold (bit d for labfm_op d,
    # rows in that order); the gather calls need all six
    op_mask: int = 0x3F

    @property
    def n(self) -> int:
        return self.row_ptr.numel() - 1

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def _c(self) -> _Operators:
        if self.op_mask != 0x3F:
            raise ValueError(f"operators built with op_mask {self.op_mask:#x}: the gather calls "
                             "need all six operators (op_mask 0x3F)")
        tp = None
        if self.tiles is not None and self.use_tiles:
            hc, hi, lc, hmax = self.tiles
            self._ctiles = _Tiles(hc.numel(), hmax, _ptr(hc).value, _ptr(hi).value,
                                  _ptr(lc).value)
            tp = ctypes.pointer(self._ctiles)
        return _Operators(self.n, self.nnz, _ptr(self.row_ptr).value, _ptr(self.col).value,
                          None if self.w is None else _ptr(self.w).value,
                          None if self.w32 is None else _w32_ptr(self.w32).value,
                          None if self.mom32 is None else _ptr(self.mom32).value,
                          _ptr(self.kappa).value, tp,
                          None if self.wall_normal is None else _ptr(self.wall_normal).value)


def w32_stride(nnz: int) -> int:
    """Row stride of the float32 weight copy (labfm_w32_stride), at least 1
    so that an empty set still gets a valid allocation."""
    return max(1, int(lib().labfm_w32_stride(int(nnz))))


def build_weights(x, y, h, s, m, box, row_ptr, col, f32: bool = False,
                  rowsum: bool = False, tiles: bool = True, tune: bool = False,
                  op_mask: int = 0x3F, tune_cache: Optional[str] = None) -> Operators:
    """Weights of the operators in op_mask (all six by default), filter
    coefficients and node status; with ``tiles`` also the node tiles used by
    the LDS-staged kernels. ``tune`` picks the build distribution with
    labfm_tune_build (cached in ``tune_cache``, or the file LABFM_TUNE_CACHE
    names)."""
    n = x.numel()
    nnz = col.numel()
    dev = x.device
    k = bin(op_mask & 0x3F).count("1")
    if not torch.is_tensor(m):
        m = torch.full((n,), int(m), dtype=torch.int8, device=dev)
    # one extra element keeps the data pointer valid when nnz == 0
    w = torch.empty(k * nnz + 1, dtype=torch.float64, device=dev)[: k * nnz].view(k, nnz)
    # float32 rows at the library's padded stride (128-byte aligned rows); the
    # operators keep the (k, nnz) view of it
    w32 = (torch.empty((k, w32_stride(nnz)), dtype=torch.float32, device=dev)[:, :nnz]
           if f32 else None)
    # the first moments of the float32 L, xx and xy weights, when they are built
    second = (1 << OP_L) | (1 << OP_XX) | (1 << OP_XY)
    mom32 = (torch.empty((NUM_MOM32, n), dtype=torch.float32, device=dev)
             if f32 and (op_mask & second) == second else None)
    kappa = torch.empty(n, dtype=torch.float64, device=dev)
    rs = torch.empty((k, n), dtype=torch.float64, device=dev) if rowsum else None
    status = torch.empty(n, dtype=torch.int8, device=dev)
    ws = _workspace(lib().labfm_build_workspace_bytes(n), dev)
    args = (_ptr(x), _ptr(y), _ptr(h), _ptr(s), _ptr(m), n, _box(box), _ptr(row_ptr), _ptr(col),
            nnz, int(op_mask), _ptr(w), _w32_ptr(w32), _ptr(mom32), _ptr(kappa), _ptr(rs),
            _ptr(status), _ptr(ws), ws.numel())
    if tune:
        best, ms, hit = _BuildConfig(), ctypes.c_double(0.0), ctypes.c_int32(0)
        _check(lib().labfm_tune_build(*args, _cache_arg(tune_cache), ctypes.byref(best),
                                      ctypes.byref(ms), ctypes.byref(hit), _stream()))
        build_weights.last_tuned = (best.mode, best.workgroups_per_cu, ms.value, bool(hit.value))
    else:
        _check(lib().labfm_build_weights(*args, _stream()))
    ops = Operators(row_ptr, col, w, w32, kappa, mom32, rs, status, op_mask=int(op_mask))
    if tiles:
        build_tiles(ops)
    return ops


def boundary_weights(x, y, h, s, box, ops: Operators, column: torch.Tensor,
                     normal: torch.Tensor) -> Operators:
    """Boundary operators of the strip columns (labfm_boundary_weights),
    written over ops (built by build_weights on the same node set); sets
    ops.wall_normal. column: int32 (count, 5) node indices of levels 0..4;
    normal: float64 (count, 2) unit normals into the fluid."""
    if ops.op_mask != 0x3F:
        raise ValueError("boundary_weights rewrites the rows of all six operators: build the "
                         "operators with op_mask 0x3F")
    n = x.numel()
    count = int(column.shape[0]) if column.numel() else 0
    st = _Strips(count, _ptr(column).value if count else None,
                 _ptr(normal).value if count else None)
    if ops.status is None:
        ops.status = torch.zeros(n, dtype=torch.int8, device=x.device)
    wn = torch.empty((n, 2), dtype=torch.float64, device=x.device)
    ws = _workspace(lib().labfm_boundary_workspace_bytes(n), x.device)
    _check(lib().labfm_boundary_weights(
        _ptr(x), _ptr(y), _ptr(h), _ptr(s), n, _box(box), _ptr(ops.row_ptr), _ptr(ops.col),
        ops.nnz, ctypes.byref(st), _ptr(ops.w), _w32_ptr(ops.w32), _ptr(ops.mom32),
        _ptr(ops.kappa), _ptr(ops.status), _ptr(wn), _ptr(ws), ws.numel(), _stream()))
    ops.wall_normal = wn
    return ops


def lagrangian_step(x: torch.Tensor, y: torch.Tensor, q: torch.Tensor, h, s, m, box, flow,
                    dt: float, n_steps: int, filter: bool = True, check_finite: bool = False,
                    nnz_capacity: Optional[int] = None,
                    workspace: Optional[torch.Tensor] = None, strict: bool = False) -> dict:
    """Advance positions (x, y) and q = [ln rho | u | v] in place by n_steps
    Lagrangian RK steps (labfm_lagrangian_step). The stencil capacity
    defaults to 1.5 times the current stencil count (queried from
    labfm_build_neighbours). Returns the call's statistics, with
    ``node_status`` the node builds per LABFM_NODE_* status; with
    ``strict`` a build that left any node with a failure status raises
    LabfmError after the call."""
    n = x.numel()
    dev = x.device
    if not torch.is_tensor(m):
        m = torch.full((n,), int(m), dtype=torch.int8, device=dev)
    if nnz_capacity is None:
        rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
        nnz = ctypes.c_int64(0)
        ws = _workspace(lib().labfm_neighbours_workspace_bytes(n), dev)
        code = lib().labfm_build_neighbours(_ptr(x), _ptr(y), _ptr(h), n, _box(box), _ptr(rp),
                                            None, 0, ctypes.byref(nnz), _ptr(ws), ws.numel(),
                                            _stream())
        if code != ERR_CAPACITY:
            _check(code)
        nnz_capacity = int(1.5 * nnz.value) + 1024
    nbytes = lib().labfm_lagrangian_workspace_bytes(n, nnz_capacity)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    prm = _RKParams(float(flow.c2), float(flow.mu), float(getattr(flow, "gx", 0.0)),
                    float(getattr(flow, "gy", 0.0)), float(dt), int(filter), int(check_finite))
    st = _LagrangianStats()
    _check(lib().labfm_lagrangian_step(_ptr(x), _ptr(y), _ptr(q), _ptr(h), _ptr(s), _ptr(m), n,
                                       _box(box), ctypes.byref(prm), int(n_steps),
                                       int(nnz_capacity), _ptr(workspace), workspace.numel(),
                                       ctypes.byref(st), _stream()))
    status = [int(v) for v in st.node_status]
    out = {"steps_done": st.steps_done, "builds": st.builds, "max_nnz": st.max_nnz,
           "build_ms": st.build_ms, "stage_ms": st.stage_ms, "nnz_capacity": nnz_capacity,
           "node_status": status}
    if strict and sum(status[1:]) > 0:
        raise NodeStatusError(status)
    return out


TILE_NODES = 32
NOALLOC_MAX_NODES = 4194304  # LABFM_NOALLOC_MAX_NODES
TILE_HALO_MAX = 1024


def build_tiles(ops: Operators) -> bool:
    """Build the node tiles of ops' stencils (LDS-staged gathers in the RK
    stage and filter). Returns False, leaving ops untiled, when a tile's halo
    exceeds TILE_HALO_MAX."""
    n, nnz, dev = ops.n, ops.nnz, ops.row_ptr.device
    nt = lib().labfm_tile_count(n)
    hc = torch.empty(nt, dtype=torch.int32, device=dev)
    hi = torch.empty(nt * TILE_HALO_MAX, dtype=torch.int32, device=dev)
    lc = torch.empty(max(1, nnz), dtype=torch.int16, device=dev)
    hmax = ctypes.c_int32(0)
    ws = _workspace(lib().labfm_tiles_workspace_bytes(), dev)
    code = lib().labfm_build_tiles(_ptr(ops.row_ptr), _ptr(ops.col), n, nnz, _ptr(hc), _ptr(hi),
                                   _ptr(lc), ctypes.byref(hmax), _ptr(ws), ws.numel(), _stream())
    if code == ERR_CAPACITY:
        ops.tiles = None
        return False
    _check(code)
    ops.tiles = (hc, hi, lc, hmax.value)
    return True


def apply_operators(ops: Operators, phi: torch.Tensor, op_mask: int = 0x3F,
                    prec: int = F64) -> torch.Tensor:
    """L^d(phi) for the operators in op_mask; shape (popcount(mask), n)."""
    k = bin(op_mask).count("1")
    out = torch.empty((k, ops.n), dtype=torch.float64, device=phi.device)
    c = ops._c()
    _check(lib().labfm_apply_operators(ctypes.byref(c), op_mask, _ptr(phi), _ptr(out), prec,
                                       _stream()))
    return out


def time_step(q: torch.Tensor, s: torch.Tensor, c2: float, mu: float, conv: float = 1.0,
              visc: float = 0.4) -> float:
    """Eq. dt on the state q (coefficients conv, visc; the paper's 1.0, 0.4)."""
    dt = ctypes.c_double(0.0)
    n = s.numel()
    ws = _workspace(lib().labfm_time_step_workspace_bytes(), q.device)
    _check(lib().labfm_time_step(_ptr(q), _ptr(s), n, float(c2), float(mu), float(conv),
                                 float(visc), ctypes.byref(dt), _ptr(ws), ws.numel(), _stream()))
    return dt.value


def ns_rhs(q: torch.Tensor, ops: Operators, flow, prec: int = F64) -> torch.Tensor:
    """Right-hand side [R_l | R_u | R_v] of the state q = [ln rho | u | v]."""
    out = torch.empty_like(q)
    prm = _RKParams(float(flow.c2), float(flow.mu), float(getattr(flow, "gx", 0.0)),
                    float(getattr(flow, "gy", 0.0)), 1.0, 0, 0)
    c = ops._c()
    _check(lib().labfm_ns_rhs(_ptr(q), ctypes.byref(c), ctypes.byref(prm), _ptr(out), prec,
                              _stream()))
    return out


def rk_workspace(n: int, device) -> torch.Tensor:
    nbytes = lib().labfm_rk_workspace_bytes(n)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def rk_step(q: torch.Tensor, ops: Operators, flow, dt: float, n_steps: int, prec: int = F64,
            use_graph: bool = False, filter: bool = True, check_finite: bool = False,
            workspace: Optional[torch.Tensor] = None, timing: bool = False,
            timing_every: int = 1):
    """Advance q = [ln rho | u | v] (float64, 3n) in place by n_steps RK steps.
    Returns the per-kernel timing dict when ``timing`` is set (event timings
    of one step in every ``timing_every``)."""
    if workspace is None:
        workspace = rk_workspace(ops.n, q.device)
    prm = _RKParams(float(flow.c2), float(flow.mu), float(getattr(flow, "gx", 0.0)),
                    float(getattr(flow, "gy", 0.0)), float(dt), int(filter), int(check_finite))
    c = ops._c()
    tm = _Timing()
    tm.every = int(timing_every)
    code = lib().labfm_rk_step(_ptr(q), ctypes.byref(c), ctypes.byref(prm), int(n_steps), prec,
                               int(use_graph), _ptr(workspace), workspace.numel(),
                               ctypes.byref(tm) if timing else None, _stream())
    _check(code)
    if timing:
        return {"stage_ms": tm.stage_ms, "filter_ms": tm.filter_ms,
                "stage_launches": tm.stage_launches, "filter_launches": tm.filter_launches}
    return None


def get_launch_config(kernel: int, prec: int, n: int, nnz: int) -> tuple:
    c = _LaunchConfig()
    _check(lib().labfm_get_launch_config(kernel, prec, n, nnz, ctypes.byref(c)))
    return c.lanes_per_node, c.flags


def set_launch_config(kernel: int, prec: int, lanes_per_node: int = 0, flags: int = 0) -> None:
    """Pin a launch shape (lanes_per_node = 0 restores the built-in choice)."""
    c = _LaunchConfig(lanes_per_node, flags)
    _check(lib().labfm_set_launch_config(kernel, prec, ctypes.byref(c)))


def tune(ops: Operators, q: torch.Tensor, prec: int = F64, reps: int = 10,
         workspace: Optional[torch.Tensor] = None, cache_path: Optional[str] = None) -> dict:
    """Time every launch shape of the stage, filter and apply kernels and
    install the fastest, or install the shapes cached for this node set in
    ``cache_path`` (else the file LABFM_TUNE_CACHE names); returns
    {kernel: (lanes_per_node, flags, ms)} and "cached": whether the shapes
    came from the cache."""
    if workspace is None:
        workspace = rk_workspace(ops.n, q.device)
    best = (_LaunchConfig * 3)()
    ms = (ctypes.c_double * 3)()
    hit = ctypes.c_int32(0)
    c = ops._c()
    _check(lib().labfm_tune(ctypes.byref(c), _ptr(q), prec, reps, _ptr(workspace),
                            workspace.numel(), _cache_arg(cache_path), best, ms,
                            ctypes.byref(hit), _stream()))
    names = ("stage", "filter", "apply")
    out = {names[k]: (best[k].lanes_per_node, best[k].flags, ms[k]) for k in range(3)}
    out["cached"] = bool(hit.value)
    return out


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

def build_transpose(ops: Operators) -> None:
    """Transposed stencils and weights for the adjoint (needs ops.rowsum,
    i.e. build_weights(..., rowsum=True))."""
    if ops.rowsum is None:
        raise ValueError("build_transpose needs the operators' row sums (rowsum=True)")
    n, nnz, dev = ops.n, ops.nnz, ops.row_ptr.device
    tptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
    tsrc = torch.empty(max(1, nnz), dtype=torch.int32, device=dev)
    tw = torch.empty(6 * nnz + 1, dtype=torch.float64, device=dev)
    c = ops._c()
    ws = _workspace(lib().labfm_transpose_workspace_bytes(n, nnz), dev)
    _check(lib().labfm_build_transpose(ctypes.byref(c), _ptr(tptr), _ptr(tsrc), _ptr(tw),
                                       _ptr(ws), ws.numel(), _stream()))
    ops.transpose = (tptr, tsrc, tw)


def rk_adjoint(q0: torch.Tensor, qbar_end: torch.Tensor, ops: Operators, flow, dt: float,
               n_steps: int, ckpt_every: int = 20, filter: bool = True) -> torch.Tensor:
    """qbar_0 = (d q_end / d q0)^T qbar_end for n_steps filtered RK steps."""
    if ops.transpose is None:
        build_transpose(ops)
    tptr, tsrc, tw = ops.transpose
    tr = _Transpose(_ptr(tptr).value, _ptr(tsrc).value, _ptr(tw).value,
                    None if ops.rowsum is None else _ptr(ops.rowsum).value)
    nbytes = lib().labfm_adjoint_workspace_bytes(ops.n, n_steps, ckpt_every)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=q0.device)
    prm = _RKParams(float(flow.c2), float(flow.mu), float(getattr(flow, "gx", 0.0)),
                    float(getattr(flow, "gy", 0.0)), float(dt), int(filter), 0)
    out = torch.empty_like(q0)
    c = ops._c()
    _check(lib().labfm_rk_adjoint(_ptr(q0), _ptr(qbar_end), _ptr(out), ctypes.byref(c),
                                  ctypes.byref(tr), ctypes.byref(prm), int(n_steps),
                                  int(ckpt_every), _ptr(ws), ws.numel(), _stream()))
    return out


class RKSolve(torch.autograd.Function):
    """(rho0, u0, v0) -> (rho, u, v) after n_steps filtered RK steps, with a
    backward pass through labfm_rk_adjoint (checkpointed recomputation).

    The library evolves ln rho; this wrapper converts rho <-> ln rho (and the
    matching gradients) at the two ends of the solve."""

    @staticmethod
    def forward(ctx, rho0, u0, v0, ops, flow, dt, n_steps, ckpt_every=20, filter=True):
        q0 = torch.cat([torch.log(rho0), u0, v0]).contiguous()
        q = q0.clone()
        rk_step(q, ops, flow, dt, n_steps, filter=filter)
        n = ops.n
        rho = torch.exp(q[:n])
        ctx.save_for_backward(q0, rho)
        ctx.cfg = (ops, flow, dt, n_steps, ckpt_every, filter)
        return rho, q[n:2 * n].clone(), q[2 * n:].clone()

    @staticmethod
    def backward(ctx, grho, gu, gv):
        q0, rho = ctx.saved_tensors
        ops, flow, dt, n_steps, ckpt_every, filter = ctx.cfg
        n = ops.n
        z = torch.zeros(n, dtype=q0.dtype, device=q0.device)
        qbar = torch.cat([(grho if grho is not None else z) * rho,
                          gu if gu is not None else z, gv if gv is not None else z]).contiguous()
        g0 = rk_adjoint(q0, qbar, ops, flow, dt, n_steps, ckpt_every, filter)
        rho0 = torch.exp(q0[:n])
        return (g0[:n] / rho0, g0[n:2 * n], g0[2 * n:], None, None, None, None, None, None)


def solve_systems(m: int, systems: torch.Tensor):
    """The weight build's LU with partial pivoting and back substitution
    (the rows-in-registers kernel) on given systems: systems is float64
    [count, n, n + 6] on the GPU ([M~ | C~] per system, n = (m^2+3m)/2).
    Returns Psi [count, n, 6], the pivot row of each column [count, n] and
    the status of each system [count] (LABFM_NODE_OK or _SINGULAR)."""
    m = int(m)
    n = (m * m + 3 * m) // 2
    if systems.dtype != torch.float64 or not systems.is_cuda or systems.dim() != 3 \
            or tuple(systems.shape[1:]) != (n, n + NUM_OPS):
        raise ValueError(f"systems must be float64 [count, {n}, {n + NUM_OPS}] on the GPU")
    sys_c = systems.contiguous()
    count = sys_c.shape[0]
    psi = torch.zeros((count, n, NUM_OPS), dtype=torch.float64, device=sys_c.device)
    piv = torch.full((count, n), -1, dtype=torch.int32, device=sys_c.device)
    status = torch.full((count,), -1, dtype=torch.int8, device=sys_c.device)
    _check(lib().labfm_solve_systems(m, _ptr(sys_c), count, _ptr(psi), _ptr(piv), _ptr(status),
                                     _stream()))
    return psi, piv, status


def mfma_f64_rate(iters: int = 4096, device=None) -> float:
    """Measured FP64 MFMA rate of the device in TFLOP/s (a measurement aid:
    the ceiling the weight build's assembly is compared with)."""
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    nbytes = int(lib().labfm_mfma_f64_rate_scratch_bytes())
    scratch = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=dev)
    out = ctypes.c_double(0.0)
    _check(lib().labfm_mfma_f64_rate(int(iters), _ptr(scratch), nbytes, ctypes.byref(out),
                                     _stream()))
    return float(out.value)


def set_build_config(mode: int = 0, workgroups_per_cu: int = 0) -> None:
    """Choose how build_weights spreads nodes over the GPU (mode 0 restores
    the default, BUILD_ROWS)."""
    if mode == 0:
        _check(lib().labfm_set_build_config(None))
    else:
        c = _BuildConfig(mode, workgroups_per_cu)
        _check(lib().labfm_set_build_config(ctypes.byref(c)))


def get_build_config() -> tuple:
    c = _BuildConfig()
    _check(lib().labfm_get_build_config(ctypes.byref(c)))
    return c.mode, c.workgroups_per_cu


# ---------------------------------------------------------------------------
# stencil optimisation
# ---------------------------------------------------------------------------

def optimise_stencils(x, y, s, m, box, h0=None, shrink: float = 0.99, gain_max: float = 1.01,
                      res_coef: float = 1e4, max_iter: int = 200) -> tuple:
    """The paper's stencil optimisation: per-node h shrunk from h0 (default
    2.8 s) while the node's system stays solvable and no amplitude response
    exceeds gain_max. Returns (h, accepted shrinks per node)."""
    n = x.numel()
    dev = x.device
    if not torch.is_tensor(m):
        m = torch.full((n,), int(m), dtype=torch.int8, device=dev)
    if h0 is None:
        h0 = 2.8 * s
    h0 = h0.contiguous()
    rp, col = build_neighbours(x, y, h0, box)
    h = torch.empty(n, dtype=torch.float64, device=dev)
    iters = torch.empty(n, dtype=torch.int32, device=dev)
    prm = _StencilOptParams(float(shrink), float(gain_max), float(res_coef), int(max_iter))
    ws = _workspace(lib().labfm_optimise_workspace_bytes(n, col.numel()), dev)
    _check(lib().labfm_optimise_stencils(_ptr(x), _ptr(y), _ptr(h0), _ptr(s), _ptr(m), n,
                                         _box(box), _ptr(rp), _ptr(col), col.numel(),
                                         ctypes.byref(prm), _ptr(h), _ptr(iters), _ptr(ws),
                                         ws.numel(), _stream()))
    return h, iters
