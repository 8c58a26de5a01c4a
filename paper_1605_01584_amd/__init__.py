"""All-pairs Pearson correlation on MI355X: Python binding of libpcc.so.

Argument marshalling only.  Every step of the computation runs in the HIP
kernels of ``libpcc.so`` (see ``include/pcc.h`` for the C ABI); PyTorch is
used for device memory and streams.  Importing this package fails loudly if
the library has not been built (``python paper_1605_01584_amd/build.py`` or
``python __graft_entry__.py build`` from the repository root).

Names follow the C ABI: ``z_layout``, ``normalize``, ``allpairs``,
``allpairs_f64``, ``allpairs_to_host``, ``threshold_edges``, ``allpairs_xy``,
``threshold_edges_xy``, ``permtest``, ``BatchPlan``, the job maps and
``autotune``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python paper_1605_01584_amd/build.py, or python __graft_entry__.py build from the "
        "repository root). There is no CPU fallback.")

# One HIP runtime per process: torch's HIP libraries load the runtime bundled
# with torch under the name "libamdhip64.so" (through their own RPATH), while
# libpcc.so asks for "libamdhip64.so.7".  With torch loaded first, the
# request of libpcc.so matches the SONAME already in the process and both
# share torch's runtime; the other order would load a second runtime, which
# then sees no device.  So torch is imported before libpcc.so is opened.
import torch as _torch_for_hip_runtime  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# ---- enums ----------------------------------------------------------------
PCC_OK, PCC_E_ARG, PCC_E_SHAPE, PCC_E_MODE, PCC_E_CAPACITY, PCC_E_HIP, PCC_E_WORKSPACE, \
    PCC_E_DEVICE = 0, -1, -2, -3, -4, -5, -6, -7
IN_F32, IN_F64 = 0, 1
FP32, SPLIT_BF16X3, BF16, FP16, FP64 = 0, 1, 2, 3, 4
MODES = {"fp32": FP32, "split": SPLIT_BF16X3, "bf16": BF16, "fp16": FP16, "fp64": FP64}


class ZDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("l", ctypes.c_int64), ("n_pad", ctypes.c_int64),
                ("l_pad", ctypes.c_int64), ("row_bytes", ctypes.c_int64),
                ("bytes", ctypes.c_int64), ("mode", ctypes.c_int32), ("kchunk", ctypes.c_int32)]

    def __repr__(self):
        return (f"ZDesc(n={self.n}, l={self.l}, n_pad={self.n_pad}, l_pad={self.l_pad}, "
                f"row_bytes={self.row_bytes}, bytes={self.bytes}, mode={self.mode})")


class TileCfg(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("order", ctypes.c_int32), ("band", ctypes.c_int32),
                ("grid", ctypes.c_int32)]

    def as_tuple(self):
        return (self.tile, self.order, self.band, self.grid)

    def __repr__(self):
        return f"TileCfg(tile={self.tile}, order={self.order}, band={self.band}, grid={self.grid})"


class BatchItem(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("n", ctypes.c_int64),
                ("l", ctypes.c_int64), ("xt", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("z", ctypes.c_void_p), ("r", ctypes.c_void_p)]


_i64, _i32, _vp, _f32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_float
_i64p = ctypes.POINTER(ctypes.c_int64)
_zdp = ctypes.POINTER(ZDesc)
_cfgp = ctypes.POINTER(TileCfg)


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("pcc_status_string", ctypes.c_char_p, _i32)
_sig("pcc_version", _i32)
_sig("pcc_last_hip_error", _i32)
_sig("pcc_last_hip_error_string", ctypes.c_char_p)
_sig("pcc_z_layout", _i32, _i64, _i64, _i32, _zdp)
_sig("pcc_default_cfg", _i32, _zdp, _cfgp)
_sig("pcc_normalize", _i32, _vp, _i32, _i64, _zdp, _vp, _vp, _vp, _vp)
_sig("pcc_workspace_size", ctypes.c_size_t, _zdp, _i32)
_sig("pcc_allpairs", _i32, _zdp, _vp, _vp, _cfgp, _vp, _vp)
_sig("pcc_allpairs_f64", _i32, _zdp, _vp, _vp, _cfgp, _vp, _vp)
_sig("pcc_threshold_edges", _i32, _zdp, _vp, _f32, _vp, _vp, _i64, _vp, _cfgp, _vp, _vp)
PASS_FN = ctypes.CFUNCTYPE(None, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p)
_sig("pcc_stream_buffer_bytes", ctypes.c_size_t, _zdp, _cfgp, _i64)
_sig("pcc_allpairs_to_host", _i32, _zdp, _vp, _vp, _i64, _vp, ctypes.c_size_t, _cfgp, PASS_FN,
     _vp, _vp, _vp)
_sig("pcc_allpairs_xy", _i32, _zdp, _vp, _zdp, _vp, _vp, _i64, _cfgp, _vp, _vp)
_sig("pcc_threshold_edges_xy", _i32, _zdp, _vp, _zdp, _vp, _f32, _vp, _vp, _i64, _vp, _cfgp, _vp,
     _vp)
_sig("pcc_edges_status", _i32, _i64, _i64)
_sig("pcc_permtest", _i32, _zdp, _vp, _vp, _i32, _vp, _vp, _vp)
_sig("pcc_permtest_max_l", _i64, _i32)
_sig("pcc_permtest_tiles", _i32, _zdp, _vp, _vp, _i32, _vp, _cfgp, _vp, ctypes.c_size_t, _vp)
_sig("pcc_batch_workspace_size", ctypes.c_size_t, _i32)
_sig("pcc_batch_plan_create", _i32, _i32, ctypes.POINTER(BatchItem), _i32, _vp, ctypes.c_size_t,
     _vp, ctypes.POINTER(_vp))
_sig("pcc_batch_plan_launch", _i32, _vp, _vp)
_sig("pcc_batch_plan_jobs", _i64, _vp)
_sig("pcc_batch_plan_destroy", _i32, _vp)
_sig("pcc_batch_run_noalloc", _i32, _i32, ctypes.POINTER(BatchItem), _i32, _vp)
_sig("pcc_job_of_cell", _i64, _i64, _i64, _i64)
_sig("pcc_cell_of_job", None, _i64, _i64, _i64p, _i64p)
_sig("pcc_packed_index", _i64, _i64, _i64, _i64)
_sig("pcc_packed_cell", None, _i64, _i64, _i64p, _i64p)
_sig("pcc_cells_host", _i32, _i64, _i32, _i64, _i64, _vp, _vp)
_sig("pcc_tile_order_host", _i32, _i64, _cfgp, _i64, _i64, _vp, _vp)
_sig("pcc_rect_tile_order_host", _i32, _i64, _i64, _cfgp, _i64, _i64, _vp, _vp)
_sig("pcc_cells_device", _i32, _i64, _i32, _i64, _i64, _vp, _vp, _vp)
_sig("pcc_autotune", _i32, _zdp, _vp, _vp, _cfgp, _i32, _i32, _cfgp, _vp, _vp)
_sig("pcc_device_cus", _i32)
_sig("pcc_autotune_default_count", _i32)
_sig("pcc_tile_arith", _i32, _zdp)

EXPORTED = [
    "pcc_status_string", "pcc_version", "pcc_last_hip_error", "pcc_last_hip_error_string",
    "pcc_z_layout", "pcc_default_cfg", "pcc_normalize",
    "pcc_workspace_size", "pcc_allpairs", "pcc_allpairs_f64", "pcc_threshold_edges",
    "pcc_edges_status", "pcc_allpairs_xy", "pcc_threshold_edges_xy", "pcc_rect_tile_order_host",
    "pcc_stream_buffer_bytes", "pcc_allpairs_to_host",
    "pcc_permtest", "pcc_permtest_max_l", "pcc_batch_workspace_size", "pcc_batch_plan_create",
    "pcc_batch_plan_launch", "pcc_batch_plan_jobs", "pcc_batch_plan_destroy", "pcc_job_of_cell",
    "pcc_cell_of_job", "pcc_packed_index", "pcc_packed_cell", "pcc_cells_host",
    "pcc_tile_order_host", "pcc_cells_device", "pcc_autotune", "pcc_device_cus",
    "pcc_autotune_default_count", "pcc_tile_arith", "pcc_batch_run_noalloc",
    "pcc_permtest_tiles",
]

BATCH_NOALLOC_MAX_D = 256  # PCC_BATCH_NOALLOC_MAX_D


class PccError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = f"{where}: {status_string(status)}"
        if status == PCC_E_HIP:
            self.hip_error = _lib.pcc_last_hip_error()
            msg += f" ({_lib.pcc_last_hip_error_string().decode()} = {self.hip_error})"
        super().__init__(msg)


def status_string(s: int) -> str:
    return _lib.pcc_status_string(int(s)).decode()


def _check(s: int, where: str):
    if s != PCC_OK:
        raise PccError(s, where)


def version() -> int:
    return _lib.pcc_version()


def _mode(mode) -> int:
    if isinstance(mode, str):
        return MODES[mode]
    return int(mode)


# ---- layout & maps (host only) ----------------------------------------------

def z_layout(n: int, l: int, mode="fp32") -> ZDesc:
    zd = ZDesc()
    _check(_lib.pcc_z_layout(n, l, _mode(mode), ctypes.byref(zd)), "pcc_z_layout")
    return zd


def default_cfg(zd: ZDesc) -> TileCfg:
    c = TileCfg()
    _check(_lib.pcc_default_cfg(ctypes.byref(zd), ctypes.byref(c)), "pcc_default_cfg")
    return c


def tile_cfg(tile=256, order=1, band=8, grid=0) -> TileCfg:
    return TileCfg(tile, order, band, grid)


def job_of_cell(m: int, y: int, x: int) -> int:
    return _lib.pcc_job_of_cell(m, y, x)


def cell_of_job(m: int, J: int):
    y, x = ctypes.c_int64(), ctypes.c_int64()
    _lib.pcc_cell_of_job(m, J, ctypes.byref(y), ctypes.byref(x))
    return y.value, x.value


def packed_index(n: int, y: int, x: int) -> int:
    return _lib.pcc_packed_index(n, y, x)


def packed_cell(n: int, Jp: int):
    y, x = ctypes.c_int64(), ctypes.c_int64()
    _lib.pcc_packed_cell(n, Jp, ctypes.byref(y), ctypes.byref(x))
    return y.value, x.value


def cells_host(m: int, diag: bool, J0: int, count: int):
    y = np.empty(count, dtype=np.int64)
    x = np.empty(count, dtype=np.int64)
    _check(_lib.pcc_cells_host(m, 1 if diag else 0, J0, count, y.ctypes.data, x.ctypes.data),
           "pcc_cells_host")
    return y, x


def tile_order_host(m: int, cfg: TileCfg, J0: int, count: int):
    y = np.empty(count, dtype=np.int64)
    x = np.empty(count, dtype=np.int64)
    _check(_lib.pcc_tile_order_host(m, ctypes.byref(cfg), J0, count, y.ctypes.data,
                                    x.ctypes.data), "pcc_tile_order_host")
    return y, x


def rect_tile_order_host(mr: int, mc: int, cfg: TileCfg, J0: int, count: int):
    y = np.empty(count, dtype=np.int64)
    x = np.empty(count, dtype=np.int64)
    _check(_lib.pcc_rect_tile_order_host(mr, mc, ctypes.byref(cfg), J0, count, y.ctypes.data,
                                         x.ctypes.data), "pcc_rect_tile_order_host")
    return y, x


def permtest_max_l(mode="fp32") -> int:
    return _lib.pcc_permtest_max_l(_mode(mode))


def device_cus() -> int:
    return _lib.pcc_device_cus()


# ---- device entry points ------------------------------------------------------

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the pcc library runs on gfx950 only")
    return torch


def _stream(torch, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    return ctypes.c_void_p(t.data_ptr())


def empty_z(zd: ZDesc, device="cuda"):
    torch = _torch()
    return torch.empty(zd.bytes, dtype=torch.uint8, device=device)


def normalize(x, mode="fp32", z=None, stats: bool = False, degenerate: bool = False,
              stream=None):
    """Eq. (4) on device matrix x (n x l, FP32 or FP64, row pitch x.stride(0)).
    Returns (z, zd[, stats (n x 2 FP64: mean, M2)][, n_degenerate (int32 scalar tensor)])."""
    torch = _torch()
    if x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("x must be 2-D with unit stride along samples")
    if x.dtype == torch.float32:
        xt = IN_F32
    elif x.dtype == torch.float64:
        xt = IN_F64
    else:
        raise ValueError("x must be float32 or float64")
    n, l = x.shape
    zd = z_layout(n, l, mode)
    if z is None:
        z = torch.empty(zd.bytes, dtype=torch.uint8, device=x.device)
    elif z.numel() * z.element_size() < zd.bytes:
        raise ValueError("z too small")
    st = torch.empty((n, 2), dtype=torch.float64, device=x.device) if stats else None
    nd = torch.empty((), dtype=torch.int32, device=x.device) if degenerate else None
    _check(_lib.pcc_normalize(_dev_ptr(x, "x"), xt, x.stride(0), ctypes.byref(zd),
                              _dev_ptr(z, "z"), _dev_ptr(st, "stats") if st is not None else None,
                              _dev_ptr(nd, "n_degenerate") if nd is not None else None,
                              _stream(torch, stream)), "pcc_normalize")
    out = [z, zd]
    if stats:
        out.append(st)
    if degenerate:
        out.append(nd)
    return tuple(out)


def allpairs(z, zd: ZDesc, cfg: Optional[TileCfg] = None, out=None, stream=None):
    """Packed strict upper triangle of r, n(n-1)/2 FP32 (row y contiguous)."""
    torch = _torch()
    npairs = zd.n * (zd.n - 1) // 2
    if out is None:
        out = torch.empty(npairs, dtype=torch.float32, device=z.device)
    elif out.numel() < npairs or out.dtype != torch.float32:
        raise ValueError("out must hold n(n-1)/2 float32")
    _check(_lib.pcc_allpairs(ctypes.byref(zd), _dev_ptr(z, "z"), _dev_ptr(out, "r"),
                             ctypes.byref(cfg) if cfg is not None else None, None,
                             _stream(torch, stream)), "pcc_allpairs")
    return out


def allpairs_f64(z, zd: ZDesc, cfg: Optional[TileCfg] = None, out=None, stream=None):
    """FP64 mode only: packed strict upper triangle of r in FP64."""
    torch = _torch()
    npairs = zd.n * (zd.n - 1) // 2
    if out is None:
        out = torch.empty(npairs, dtype=torch.float64, device=z.device)
    elif out.numel() < npairs or out.dtype != torch.float64:
        raise ValueError("out must hold n(n-1)/2 float64")
    _check(_lib.pcc_allpairs_f64(ctypes.byref(zd), _dev_ptr(z, "z"), _dev_ptr(out, "r"),
                                 ctypes.byref(cfg) if cfg is not None else None, None,
                                 _stream(torch, stream)), "pcc_allpairs_f64")
    return out


def stream_buffer_bytes(zd: ZDesc, cfg: Optional[TileCfg], rows_per_pass: int) -> int:
    return _lib.pcc_stream_buffer_bytes(ctypes.byref(zd),
                                        ctypes.byref(cfg) if cfg is not None else None,
                                        rows_per_pass)


def allpairs_to_host(z, zd: ZDesc, rows_per_pass: int, cfg: Optional[TileCfg] = None, out=None,
                     on_pass=None, dev_buf=None, stream=None, copy_stream=None):
    """Multi-pass all pairs into host memory: passes of rows_per_pass tile rows,
    double-buffered on the device, each copied to its place in `out` (pinned
    host float32, n(n-1)/2) while the next pass computes.  on_pass(first, count)
    is called after each slice has landed.  Blocking."""
    torch = _torch()
    if cfg is None:
        cfg = default_cfg(zd)
    need = stream_buffer_bytes(zd, cfg, rows_per_pass)
    if need == 0:
        raise ValueError("invalid layout, schedule or rows_per_pass")
    npairs = zd.n * (zd.n - 1) // 2
    if out is None:
        out = torch.empty(npairs, dtype=torch.float32, pin_memory=True)
    if out.is_cuda or out.dtype != torch.float32 or out.numel() < npairs or not out.is_contiguous():
        raise ValueError("out must be a contiguous host float32 tensor of n(n-1)/2")
    if dev_buf is None:
        dev_buf = torch.empty(need, dtype=torch.uint8, device=z.device)
    cs = stream if stream is not None else torch.cuda.current_stream()
    xs = copy_stream if copy_stream is not None else torch.cuda.Stream(device=z.device)
    cb = PASS_FN(lambda f, c, u: on_pass(f, c)) if on_pass is not None else PASS_FN()
    _check(_lib.pcc_allpairs_to_host(ctypes.byref(zd), _dev_ptr(z, "z"),
                                     ctypes.c_void_p(out.data_ptr()), rows_per_pass,
                                     _dev_ptr(dev_buf, "dev_buf"),
                                     dev_buf.numel() * dev_buf.element_size(), ctypes.byref(cfg),
                                     cb, None, ctypes.c_void_p(cs.cuda_stream),
                                     ctypes.c_void_p(xs.cuda_stream)), "pcc_allpairs_to_host")
    return out


def allpairs_xy(zx, zdx: ZDesc, zy, zdy: ZDesc, cfg: Optional[TileCfg] = None, out=None,
                stream=None):
    """Non-symmetric all pairs (Eq. 7-8): r[y, x] = r(X_y, Y_x), an nx x ny FP32
    matrix (out may be a wider row-major matrix; its row pitch is used)."""
    torch = _torch()
    if out is None:
        out = torch.empty((zdx.n, zdy.n), dtype=torch.float32, device=zx.device)
    if (out.dtype != torch.float32 or out.dim() != 2 or out.shape[0] < zdx.n
            or out.shape[1] < zdy.n or out.stride(1) != 1):
        raise ValueError("out must be float32 (>= nx, >= ny) with unit column stride")
    _check(_lib.pcc_allpairs_xy(ctypes.byref(zdx), _dev_ptr(zx, "zx"), ctypes.byref(zdy),
                                _dev_ptr(zy, "zy"), _dev_ptr(out, "r"), out.stride(0),
                                ctypes.byref(cfg) if cfg is not None else None, None,
                                _stream(torch, stream)), "pcc_allpairs_xy")
    return out


def threshold_edges_xy(zx, zdx: ZDesc, zy, zdy: ZDesc, thr: float, cap: int,
                       cfg: Optional[TileCfg] = None, stream=None, sync: bool = True):
    """Edges (y in X, x in Y) with |r| >= thr; as threshold_edges."""
    torch = _torch()
    ij = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=zx.device)
    rv = torch.empty(max(cap, 1), dtype=torch.float32, device=zx.device)
    cnt = torch.empty((), dtype=torch.int64, device=zx.device)
    _check(_lib.pcc_threshold_edges_xy(ctypes.byref(zdx), _dev_ptr(zx, "zx"), ctypes.byref(zdy),
                                       _dev_ptr(zy, "zy"), float(thr), _dev_ptr(ij, "ij"),
                                       _dev_ptr(rv, "rv"), cap, _dev_ptr(cnt, "count"),
                                       ctypes.byref(cfg) if cfg is not None else None, None,
                                       _stream(torch, stream)), "pcc_threshold_edges_xy")
    if not sync:
        return ij, rv, cnt
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    c = int(cnt.item())
    _check(_lib.pcc_edges_status(c, cap), "pcc_threshold_edges_xy")
    return ij[:c], rv[:c], c


def threshold_edges(z, zd: ZDesc, thr: float, cap: int, cfg: Optional[TileCfg] = None,
                    stream=None, sync: bool = True):
    """Edges with |r| >= thr.  Returns (ij int32 [cap,2], r float32 [cap],
    count int64 device scalar).  With sync=True the count is read back and the
    arrays are cut to min(count, cap); PccError(PCC_E_CAPACITY) if it overflowed."""
    torch = _torch()
    ij = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=z.device)
    rv = torch.empty(max(cap, 1), dtype=torch.float32, device=z.device)
    cnt = torch.empty((), dtype=torch.int64, device=z.device)
    _check(_lib.pcc_threshold_edges(ctypes.byref(zd), _dev_ptr(z, "z"), float(thr),
                                    _dev_ptr(ij, "ij"), _dev_ptr(rv, "rv"), cap,
                                    _dev_ptr(cnt, "count"),
                                    ctypes.byref(cfg) if cfg is not None else None, None,
                                    _stream(torch, stream)), "pcc_threshold_edges")
    if not sync:
        return ij, rv, cnt
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    c = int(cnt.item())
    _check(_lib.pcc_edges_status(c, cap), "pcc_threshold_edges")
    return ij[:c], rv[:c], c


def workspace_size(zd: ZDesc, op: int) -> int:
    """pcc_workspace_size: 0 allpairs, 1 edges, 2 permtest, 3 permtest_tiles."""
    return _lib.pcc_workspace_size(ctypes.byref(zd), int(op))


def _perm_args(zd: ZDesc, perms, validate: bool):
    torch = _torch()
    if perms.dtype != torch.int32 or perms.dim() != 2 or perms.shape[1] != zd.l:
        raise ValueError("perms must be int32 (P, l)")
    perms = perms.contiguous()
    if validate and perms.numel():
        # every row must be a permutation of 0..l-1
        srt = torch.sort(perms, dim=1).values
        if not bool((srt == torch.arange(zd.l, device=perms.device, dtype=torch.int32)).all()):
            raise ValueError("every row of perms must be a permutation of 0..l-1")
    return perms


def _counts_out(torch, zd: ZDesc, out, device):
    npairs = zd.n * (zd.n - 1) // 2
    if out is None:
        return torch.empty(npairs, dtype=torch.int32, device=device)
    if out.numel() < npairs or out.dtype != torch.int32:
        raise ValueError("out must hold n(n-1)/2 int32")
    return out


def permtest(z, zd: ZDesc, perms, out=None, stream=None, validate: bool = True, workspace=None):
    """Counts of |r_perm| >= |r_obs| over the P rows of perms (device int32 P x l).
    z in the "fp32" or "split" layout (the arithmetic follows the layout).
    Rows longer than permtest_max_l take the tiled form, with a workspace of
    workspace_size(zd, 2) bytes (allocated here unless given).
    validate=True checks on the device that every row is a permutation."""
    torch = _torch()
    perms = _perm_args(zd, perms, validate)
    out = _counts_out(torch, zd, out, z.device)
    ws = workspace_size(zd, 2)
    if ws and workspace is None:
        workspace = torch.empty(ws, dtype=torch.uint8, device=z.device)
    _check(_lib.pcc_permtest(ctypes.byref(zd), _dev_ptr(z, "z"), _dev_ptr(perms, "perms"),
                             perms.shape[0], _dev_ptr(out, "counts"),
                             _dev_ptr(workspace, "workspace") if ws else None,
                             _stream(torch, stream)), "pcc_permtest")
    return out


def permtest_tiles(z, zd: ZDesc, perms, cfg: Optional[TileCfg] = None, out=None, stream=None,
                   validate: bool = True, workspace=None):
    """The tiled permutation test (any row length): as permtest, on the
    all-pairs tile schedule cfg; workspace of workspace_size(zd, 3) bytes."""
    torch = _torch()
    perms = _perm_args(zd, perms, validate)
    out = _counts_out(torch, zd, out, z.device)
    ws = workspace_size(zd, 3)
    if workspace is None:
        workspace = torch.empty(max(ws, 1), dtype=torch.uint8, device=z.device)
    nbytes = workspace.numel() * workspace.element_size()
    _check(_lib.pcc_permtest_tiles(ctypes.byref(zd), _dev_ptr(z, "z"), _dev_ptr(perms, "perms"),
                                   perms.shape[0], _dev_ptr(out, "counts"),
                                   ctypes.byref(cfg) if cfg is not None else None,
                                   _dev_ptr(workspace, "workspace"), nbytes,
                                   _stream(torch, stream)), "pcc_permtest_tiles")
    return out


def _batch_items(xs, mode: int, tiles=None, zs=None, rs=None):
    """BatchItem array for datasets xs, with z and r buffers (given or new)."""
    torch = _torch()
    D = len(xs)
    items = (BatchItem * D)()
    zds, zo, ro = [], [], []
    for d, x in enumerate(xs):
        if x.dim() != 2 or x.stride(1) != 1:
            raise ValueError("each x must be 2-D with unit stride along samples")
        n, l = x.shape
        zd = z_layout(n, l, mode)
        z = zs[d] if zs is not None else torch.empty(zd.bytes, dtype=torch.uint8, device=x.device)
        r = rs[d] if rs is not None else torch.empty(n * (n - 1) // 2, dtype=torch.float32,
                                                      device=x.device)
        if z.numel() * z.element_size() < zd.bytes or r.numel() < n * (n - 1) // 2 \
                or r.dtype != torch.float32:
            raise ValueError(f"dataset {d}: z or r too small")
        zds.append(zd)
        zo.append(z)
        ro.append(r)
        items[d] = BatchItem(x.data_ptr(), x.stride(0), n, l,
                             IN_F64 if x.dtype == torch.float64 else IN_F32,
                             int(tiles[d]) if tiles is not None else 0,
                             _dev_ptr(z, "z").value, _dev_ptr(r, "r").value)
    return items, zds, zo, ro


def batch_run_noalloc(xs: Sequence, mode="split", tiles: Optional[Sequence[int]] = None,
                      zs=None, rs=None, stream=None):
    """The batch of BatchPlan(xs, mode, tiles) run by pcc_batch_run_noalloc:
    no graph and no workspace (the library's static scratch).  zs / rs:
    optional output buffers (new ones otherwise).  Returns (zd, z, r) lists."""
    torch = _torch()
    if len(xs) > BATCH_NOALLOC_MAX_D:
        raise ValueError(f"at most {BATCH_NOALLOC_MAX_D} datasets")
    md = _mode(mode)
    items, zds, zo, ro = _batch_items(list(xs), md, tiles, zs, rs)
    _check(_lib.pcc_batch_run_noalloc(len(xs), items, md, _stream(torch, stream)),
           "pcc_batch_run_noalloc")
    return zds, zo, ro


class BatchPlan:
    """One hipGraph running the transformation and all pairs of D datasets.

    xs: list of device matrices (n_d x l_d, float32/float64).  Outputs: self.z[d]
    (layout self.zd[d]) and self.r[d] (packed triangle of dataset d)."""

    def __init__(self, xs: Sequence, mode="split", tiles: Optional[Sequence[int]] = None,
                 stream=None):
        torch = _torch()
        self.D = len(xs)
        self.mode = _mode(mode)
        self.xs = list(xs)
        items, self.zd, self.z, self.r = _batch_items(self.xs, self.mode, tiles)
        self._items = items
        ws = _lib.pcc_batch_workspace_size(self.D)
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.xs[0].device)
        plan = ctypes.c_void_p()
        _check(_lib.pcc_batch_plan_create(self.D, items, self.mode,
                                          _dev_ptr(self.workspace, "workspace"), ws,
                                          _stream(torch, stream), ctypes.byref(plan)),
               "pcc_batch_plan_create")
        self._plan = plan
        self.jobs = _lib.pcc_batch_plan_jobs(plan)

    def launch(self, stream=None):
        torch = _torch()
        _check(_lib.pcc_batch_plan_launch(self._plan, _stream(torch, stream)),
               "pcc_batch_plan_launch")

    def close(self):
        if self._plan:
            _lib.pcc_batch_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cells_device(m: int, diag: bool, J0: int, count: int, stream=None):
    torch = _torch()
    y = torch.empty(count, dtype=torch.int64, device="cuda")
    x = torch.empty(count, dtype=torch.int64, device="cuda")
    _check(_lib.pcc_cells_device(m, 1 if diag else 0, J0, count, _dev_ptr(y, "y"),
                                 _dev_ptr(x, "x"), _stream(torch, stream)), "pcc_cells_device")
    return y, x


AUTOTUNE_DEFAULT_CANDIDATES = _lib.pcc_autotune_default_count()


def tile_arith(zd: ZDesc) -> int:
    """The arithmetic the tile kernels use for layout zd (a MODES value):
    zd.mode, except FP32 for the split layout of rows of at most 64 samples."""
    return _lib.pcc_tile_arith(ctypes.byref(zd))


def autotune(z, zd: ZDesc, r=None, cands: Optional[Sequence[TileCfg]] = None, reps: int = 3,
             stream=None):
    """Time candidate schedules of allpairs on z; returns (best TileCfg, times_ms list)."""
    torch = _torch()
    if r is None:
        r = torch.empty(zd.n * (zd.n - 1) // 2, dtype=torch.float32, device=z.device)
    nc = len(cands) if cands else 0
    arr = (TileCfg * nc)(*cands) if nc else None
    times = (ctypes.c_float * max(nc, AUTOTUNE_DEFAULT_CANDIDATES))()
    best = TileCfg()
    _check(_lib.pcc_autotune(ctypes.byref(zd), _dev_ptr(z, "z"), _dev_ptr(r, "r"), arr, nc,
                             reps, ctypes.byref(best), times, _stream(torch, stream)),
           "pcc_autotune")
    return best, list(times)[:max(nc, AUTOTUNE_DEFAULT_CANDIDATES)]
