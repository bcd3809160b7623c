"""Python binding of libmsc.so (ctypes).  Argument marshalling only: every
step runs in the HIP library.  torch supplies device memory and streams.

    asc, desc, ms = msc.segment(field)          # field: float32 [Z, Y, X] on GPU
    labels = msc.cc_label_grid(mask)             # mask: uint8 [Z, Y, X]
    labels = msc.cc_label_csr(row_ptr, col_idx)  # int64 [n+1], int32 [nnz]

Importing this module loads the library and raises ImportError if it has not
been built (``python -m paper_2409_03771_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with "
        "`python -m paper_2409_03771_amd.build` (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

MSC_OK, MSC_EINVAL, MSC_ERANGE, MSC_ENAN, MSC_ENOMEM = 0, 1, 2, 3, 4
MSC_EBUDGET, MSC_EHIP, MSC_ECANCELED, MSC_EBUSY = 5, 6, 7, 8

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int


class msc_stats(ctypes.Structure):
    _fields_ = [("n_vertices", _I64), ("n_maxima", _I64), ("n_minima", _I64),
                ("n_cells", _I64), ("n_exits", _I64), ("jump_rounds", _I32),
                ("tile_x", _I32), ("tile_y", _I32), ("tile_z", _I32),
                ("exit_steps", _I64), ("status", _I32), ("reserved", _I32)]


class msc_phase(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", _I64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class msc_field(ctypes.Structure):
    _fields_ = [("field", _P), ("dims", _I64 * 3), ("asc", _P), ("desc", _P),
                ("ms", _P)]


class msc_mask(ctypes.Structure):
    _fields_ = [("mask", _P), ("dims", _I64 * 3), ("labels", _P)]


class msc_tune(ctypes.Structure):
    _fields_ = [("best", _I32), ("tile", _I32 * 3), ("n_shapes", _I32),
                ("ms", ctypes.c_float * 8)]


_SIGS = {
    "msc_strerror": ([_I32], ctypes.c_char_p),
    "msc_create": ([ctypes.POINTER(_P), _I32], _I32),
    "msc_destroy": ([_P], None),
    "msc_segment": ([_P, _P, ctypes.POINTER(_I64), _P, _P, _P, _P], _I32),
    "msc_last_stats": ([_P, ctypes.POINTER(msc_stats)], _I32),
    "msc_last_status": ([_P, ctypes.POINTER(_I32)], _I32),
    "msc_segment_batched": ([_P, _I32, ctypes.POINTER(msc_field), _P], _I32),
    "msc_segment_ranks": ([_P, _P, ctypes.POINTER(_I64), _I32, _P, _P, _P, _P],
                          _I32),
    "msc_last_field_stats": ([_P, _I32, ctypes.POINTER(msc_stats)], _I32),
    "msc_autotune": ([_P, _I32, ctypes.POINTER(msc_field), _P,
                      ctypes.POINTER(msc_tune)], _I32),
    "msc_tile_shapes": ([ctypes.POINTER(_I32), _I32], _I32),
    "msc_set_tile": ([_P, _I32, _I32, _I32], _I32),
    "msc_set_table_capacity": ([_P, ctypes.c_uint64], _I32),
    "msc_profile": ([_P, _I32], _I32),
    "msc_profile_read": ([_P, ctypes.POINTER(msc_phase), _I32,
                          ctypes.POINTER(_I32)], _I32),
    "cc_label_grid": ([_P, _P, ctypes.POINTER(_I64), _P, _P], _I32),
    "msc_segment_csr": ([_P, _I64, _P, _P, _P, _P, _P, _P, _P], _I32),
    "msc_critical_points": ([_P, _P, ctypes.POINTER(_I64), _P, _P], _I32),
    "msc_extremum_graph": ([_P, _P, ctypes.POINTER(_I64), _P, _P, _P, _I64,
                            ctypes.POINTER(_I64), _P], _I32),
    "msc_csr_from_tets": ([_P, _I64, _I64, _P, _P, _P, _I64,
                           ctypes.POINTER(_I64), _P], _I32),
    "cc_label_grid_ranks": ([_P, _P, ctypes.POINTER(_I64), _I32, _P, _P],
                            _I32),
    "cc_label_csr": ([_P, _I64, _P, _P, _P, _P, _P], _I32),
    "cc_label_grid_noalloc": ([_P, ctypes.POINTER(_I64), _P, _P], _I32),
    "cc_label_grid_batched": ([_P, _I32, ctypes.POINTER(msc_mask), _P], _I32),
    "msc_set_workspace": ([_P, _P, ctypes.c_size_t], _I32),
    "msc_debug_inject": ([_I32, _I32], _I32),
    "msc_graph_create": ([_P, _I32, ctypes.POINTER(msc_field), _P,
                          ctypes.POINTER(_P)], _I32),
    "msc_graph_launch": ([_P, _P], _I32),
    "msc_graph_field_stats": ([_P, _I32, ctypes.POINTER(msc_stats)], _I32),
    "msc_graph_destroy": ([_P], None),
    "msc_workspace_size": ([_P, _I32, _I32, _P, ctypes.POINTER(ctypes.c_size_t)],
                           _I32),
    "msc_pointer_jump": ([_P, _P, _I64, _I32, _I32, _P], _I32),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

EXPORTS = tuple(_SIGS)


class MscError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.msc_strerror(code).decode()
        super().__init__(f"{where}: {msg} (code {code})")


def _check(code: int, where: str):
    if code != MSC_OK:
        raise MscError(code, where)


_ctx_lock = threading.Lock()
_ctxs: dict[int, ctypes.c_void_p] = {}


def context(device: int | None = None) -> ctypes.c_void_p:
    """The library context of a device (created once, reused)."""
    if device is None:
        device = torch.cuda.current_device()
    with _ctx_lock:
        c = _ctxs.get(device)
        if c is None:
            c = _P()
            _check(_lib.msc_create(ctypes.byref(c), int(device)), "msc_create")
            _ctxs[device] = c
        return c


def _stream(t: torch.Tensor, stream=None):
    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    return _P(stream.cuda_stream)


def _dev_ptr(t: torch.Tensor | None, dtype, name: str):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return _P(t.data_ptr())


def grid_dims(shape) -> tuple[int, int, int]:
    """(X, Y, Z) of an array stored [Z][Y][X]; 1-D and 2-D shapes are the
    degenerate grids."""
    shape = tuple(int(s) for s in shape)
    if len(shape) == 1:
        return shape[0], 1, 1
    if len(shape) == 2:
        return shape[1], shape[0], 1
    if len(shape) == 3:
        return shape[2], shape[1], shape[0]
    raise ValueError("grid arrays are 1-D, 2-D or 3-D")


def _dims_arg(dims):
    return (_I64 * 3)(*[int(d) for d in dims])


def last_status(device: int | None = None) -> int:
    """Outcome of the last asynchronous call of a device's context, as the
    device found it (waits for that call's work): MSC_OK, MSC_ENAN, ..."""
    st = _I32(0)
    _check(_lib.msc_last_status(context(device), ctypes.byref(st)),
           "msc_last_status")
    return st.value


def _check_async(device, where):
    code = last_status(device)
    if code != MSC_OK:
        raise MscError(code, where)


def segment_into(field, asc=None, desc=None, ms=None, dims=None, stream=None,
                 check=True):
    """Write ascent roots, descent roots and Morse-Smale cell ids into the
    given int32 tensors (any may be None).  The call returns with the work
    enqueued on the stream; with `check` it then waits for the work and
    raises if the device found the field invalid (NaN)."""
    if dims is None:
        dims = grid_dims(field.shape)
    code = _lib.msc_segment(
        context(field.device.index), _dev_ptr(field, torch.float32, "field"),
        _dims_arg(dims), _dev_ptr(asc, torch.int32, "asc"),
        _dev_ptr(desc, torch.int32, "desc"), _dev_ptr(ms, torch.int32, "ms"),
        _stream(field, stream))
    _check(code, "msc_segment")
    if check:
        _check_async(field.device.index, "msc_segment")


def segment(field: torch.Tensor, want=("asc", "desc", "ms"), stream=None,
            check=True):
    """Morse-Smale segmentation of a float32 field on the GPU.  Returns a
    tuple (asc, desc, ms) of flat int32 tensors (None where not wanted)."""
    n = field.numel()
    out = {k: (torch.empty(n, dtype=torch.int32, device=field.device)
               if k in want else None) for k in ("asc", "desc", "ms")}
    segment_into(field, out["asc"], out["desc"], out["ms"], stream=stream,
                 check=check)
    return out["asc"], out["desc"], out["ms"]


def segment_ranks(field: torch.Tensor, ranks: int,
                  want=("asc", "desc", "ms"), stream=None):
    """The paper's distributed scheme with `ranks` z-slab virtual ranks on
    one device (see msc_segment_ranks); same outputs as segment()."""
    n = field.numel()
    out = {k: (torch.empty(n, dtype=torch.int32, device=field.device)
               if k in want else None) for k in ("asc", "desc", "ms")}
    segment_ranks_into(field, ranks, out["asc"], out["desc"], out["ms"],
                       stream)
    return out["asc"], out["desc"], out["ms"]


def segment_ranks_into(field, ranks, asc, desc, ms, stream=None):
    """segment_ranks into caller-owned int32 outputs (any may be None)."""
    code = _lib.msc_segment_ranks(
        context(field.device.index), _dev_ptr(field, torch.float32, "field"),
        _dims_arg(grid_dims(field.shape)), int(ranks),
        _dev_ptr(asc, torch.int32, "asc"), _dev_ptr(desc, torch.int32, "desc"),
        _dev_ptr(ms, torch.int32, "ms"), _stream(field, stream))
    _check(code, "msc_segment_ranks")


def critical_points(field: torch.Tensor, stream=None) -> torch.Tensor:
    """uint8 per vertex: lower-link components | upper-link components << 4."""
    code = torch.empty(field.numel(), dtype=torch.uint8, device=field.device)
    critical_points_into(field, code, stream)
    return code


def critical_points_into(field, code, stream=None):
    _check(_lib.msc_critical_points(
        context(field.device.index), _dev_ptr(field, torch.float32, "field"),
        _dims_arg(grid_dims(field.shape)), _dev_ptr(code, torch.uint8, "code"),
        _stream(field, stream)), "msc_critical_points")


def extremum_graph_into(field, asc, desc, edges, stream=None) -> int:
    """One call into a caller buffer (None or too small: nothing written);
    returns the edge count."""
    cnt = _I64(0)
    cap = 0 if edges is None else edges.numel() // 3
    _check(_lib.msc_extremum_graph(
        context(field.device.index), _dev_ptr(field, torch.float32, "field"),
        _dims_arg(grid_dims(field.shape)), _dev_ptr(asc, torch.int32, "asc"),
        _dev_ptr(desc, torch.int32, "desc"),
        _dev_ptr(edges, torch.int32, "edges"), int(cap), ctypes.byref(cnt),
        _stream(field, stream)), "msc_extremum_graph")
    return cnt.value


def extremum_graph(field: torch.Tensor, asc: torch.Tensor, desc: torch.Tensor,
                   stream=None) -> torch.Tensor:
    """int32 [m, 3] rows (vertex, extremum, +1 / -1) of the extremum graph
    (asc and desc from segment() of the same field)."""
    cnt = _I64(0)
    args = (context(field.device.index),
            _dev_ptr(field, torch.float32, "field"),
            _dims_arg(grid_dims(field.shape)),
            _dev_ptr(asc, torch.int32, "asc"),
            _dev_ptr(desc, torch.int32, "desc"))
    _check(_lib.msc_extremum_graph(*args, None, 0, ctypes.byref(cnt),
                                   _stream(field, stream)),
           "msc_extremum_graph")
    out = torch.empty((max(cnt.value, 1), 3), dtype=torch.int32,
                      device=field.device)
    _check(_lib.msc_extremum_graph(*args, _dev_ptr(out, torch.int32, "edges"),
                                   cnt.value, ctypes.byref(cnt),
                                   _stream(field, stream)),
           "msc_extremum_graph")
    return out[:cnt.value]


def csr_from_tets(n: int, tets: torch.Tensor, stream=None):
    """(row_ptr int64 [n+1], col_idx int32) of the 1-skeleton of the
    tetrahedra `tets` (int32 [T, 4] on the device): one call for the entry
    count, one to fill the rows."""
    dev = tets.device
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nnz = _I64(0)
    args = (context(dev.index), int(n), int(tets.numel() // 4),
            _dev_ptr(tets, torch.int32, "tets"),
            _dev_ptr(row_ptr, torch.int64, "row_ptr"))
    _check(_lib.msc_csr_from_tets(*args, None, 0, ctypes.byref(nnz),
                                  _stream(tets, stream)), "msc_csr_from_tets")
    col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
    _check(_lib.msc_csr_from_tets(*args, _dev_ptr(col, torch.int32, "col"),
                                  nnz.value, ctypes.byref(nnz),
                                  _stream(tets, stream)), "msc_csr_from_tets")
    return row_ptr, col[:nnz.value]


def csr_from_tets_into(n, tets, row_ptr, col_idx, stream=None) -> int:
    """One call into caller buffers (col_idx may be None or too small:
    then only row_ptr is written); returns the entry count."""
    nnz = _I64(0)
    cap = 0 if col_idx is None else col_idx.numel()
    _check(_lib.msc_csr_from_tets(
        context(tets.device.index), int(n), int(tets.numel() // 4),
        _dev_ptr(tets, torch.int32, "tets"),
        _dev_ptr(row_ptr, torch.int64, "row_ptr"),
        _dev_ptr(col_idx, torch.int32, "col_idx"), int(cap),
        ctypes.byref(nnz), _stream(tets, stream)), "msc_csr_from_tets")
    return nnz.value


def segment_csr(row_ptr: torch.Tensor, col_idx: torch.Tensor,
                field: torch.Tensor, want=("asc", "desc", "ms"), stream=None):
    """Segmentation of a field on the vertices of a complex given as CSR
    adjacency (int64 row_ptr [n+1], int32 col_idx, float32 field [n])."""
    n = row_ptr.numel() - 1
    out = {k: (torch.empty(n, dtype=torch.int32, device=field.device)
               if k in want else None) for k in ("asc", "desc", "ms")}
    segment_csr_into(row_ptr, col_idx, field, out["asc"], out["desc"],
                     out["ms"], stream)
    return out["asc"], out["desc"], out["ms"]


def segment_csr_into(row_ptr, col_idx, field, asc, desc, ms, stream=None):
    n = row_ptr.numel() - 1
    if field.numel() != n:
        raise ValueError(f"field has {field.numel()} values for {n} vertices")
    code = _lib.msc_segment_csr(
        context(field.device.index), int(n),
        _dev_ptr(row_ptr, torch.int64, "row_ptr"),
        _dev_ptr(col_idx, torch.int32, "col_idx"),
        _dev_ptr(field, torch.float32, "field"),
        _dev_ptr(asc, torch.int32, "asc"), _dev_ptr(desc, torch.int32, "desc"),
        _dev_ptr(ms, torch.int32, "ms"), _stream(field, stream))
    _check(code, "msc_segment_csr")


def _field_array(fields, outs, dims_list):
    arr = (msc_field * len(fields))()
    for i, (f, (a, d, m), dims) in enumerate(zip(fields, outs, dims_list)):
        arr[i].field = _dev_ptr(f, torch.float32, f"fields[{i}]")
        for k in range(3):
            arr[i].dims[k] = int(dims[k])
        arr[i].asc = _dev_ptr(a, torch.int32, "asc")
        arr[i].desc = _dev_ptr(d, torch.int32, "desc")
        arr[i].ms = _dev_ptr(m, torch.int32, "ms")
    return arr


def _batch_outputs(fields, want):
    return [tuple(torch.empty(f.numel(), dtype=torch.int32, device=f.device)
                  if k in want else None for k in ("asc", "desc", "ms"))
            for f in fields]


def segment_batched_into(fields, outs, dims=None, stream=None, check=True):
    """Segment several fields in one set of launches; `outs` holds an
    (asc, desc, ms) tuple of int32 tensors (or None) per field.  With
    `check`, waits for the work and raises if any field was invalid (each
    field's own outcome: last_field_stats(i)["status"])."""
    if not fields:
        return
    dims = dims or [grid_dims(f.shape) for f in fields]
    arr = _field_array(fields, outs, dims)
    code = _lib.msc_segment_batched(context(fields[0].device.index),
                                    len(fields), arr,
                                    _stream(fields[0], stream))
    _check(code, "msc_segment_batched")
    if check:
        _check_async(fields[0].device.index, "msc_segment_batched")


class Graph:
    """A batched segmentation captured into a HIP graph (msc_graph_*): the
    same fields and outputs, replayed with one launch call each time.  The
    constructor runs the call once (outputs valid on return)."""

    def __init__(self, fields, outs, dims=None, stream=None):
        if not fields:
            raise ValueError("a graph needs at least one field")
        dims = dims or [grid_dims(f.shape) for f in fields]
        arr = _field_array(fields, outs, dims)
        self._keep = (list(fields), [tuple(o) for o in outs])
        self._g = _P()
        _check(_lib.msc_graph_create(context(fields[0].device.index),
                                     len(fields), arr,
                                     _stream(fields[0], stream),
                                     ctypes.byref(self._g)),
               "msc_graph_create")
        self._device = fields[0]

    def launch(self, stream=None):
        _check(_lib.msc_graph_launch(self._g, _stream(self._device, stream)),
               "msc_graph_launch")

    def field_stats(self, index: int) -> dict:
        s = msc_stats()
        _check(_lib.msc_graph_field_stats(self._g, int(index), ctypes.byref(s)),
               "msc_graph_field_stats")
        return {k: getattr(s, k) for k, _ in msc_stats._fields_}

    def close(self):
        if self._g:
            _lib.msc_graph_destroy(self._g)
            self._g = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def segment_batched(fields, want=("asc", "desc", "ms"), stream=None,
                    check=True):
    """Batched segmentation of a list of float32 fields (any shapes).
    Returns one (asc, desc, ms) tuple per field."""
    outs = _batch_outputs(fields, want)
    segment_batched_into(fields, outs, stream=stream, check=check)
    return outs


def last_field_stats(index: int, device: int | None = None) -> dict:
    s = msc_stats()
    _check(_lib.msc_last_field_stats(context(device), int(index),
                                     ctypes.byref(s)), "msc_last_field_stats")
    return {k: getattr(s, k) for k, _ in msc_stats._fields_}


def autotune(fields, outs=None, stream=None) -> dict:
    """Time every compiled tile shape on this batch, keep the fastest for
    the device's context; returns {"tile", "best", "ms": {shape: ms}}."""
    outs = outs or _batch_outputs(fields, ("asc", "desc", "ms"))
    dims = [grid_dims(f.shape) for f in fields]
    arr = _field_array(fields, outs, dims)
    t = msc_tune()
    _check(_lib.msc_autotune(context(fields[0].device.index), len(fields), arr,
                             _stream(fields[0], stream), ctypes.byref(t)),
           "msc_autotune")
    shapes = tile_shapes()
    return {"tile": tuple(t.tile), "best": t.best,
            "ms": {shapes[i]: t.ms[i] for i in range(t.n_shapes)}}


def last_stats(device: int | None = None) -> dict:
    s = msc_stats()
    _check(_lib.msc_last_stats(context(device), ctypes.byref(s)),
           "msc_last_stats")
    return {k: getattr(s, k) for k, _ in msc_stats._fields_}


def tile_shapes() -> list[tuple[int, int, int]]:
    """Tile shapes of the fused segmentation pass compiled into the
    library; the first is the default."""
    n = _lib.msc_tile_shapes(None, 0)
    buf = (_I32 * (3 * n))()
    _lib.msc_tile_shapes(buf, n)
    return [tuple(buf[3 * i:3 * i + 3]) for i in range(n)]


def set_tile(tx: int, ty: int, tz: int, device: int | None = None):
    """Select the segmentation tile shape of a device's context."""
    _check(_lib.msc_set_tile(context(device), tx, ty, tz), "msc_set_tile")


def set_table_capacity(first_capacity: int, device: int | None = None):
    """First capacity of the cell pair table of a device's context (0 =
    sized from the extremum counts); an undersized table is grown."""
    _check(_lib.msc_set_table_capacity(context(device), int(first_capacity)),
           "msc_set_table_capacity")


def profile(enable: bool, device: int | None = None):
    """Start (clearing old records) or stop per-kernel event timing."""
    _check(_lib.msc_profile(context(device), int(bool(enable))), "msc_profile")


def profile_read(device: int | None = None) -> dict:
    """{kernel: {"launches", "total_ms", "bytes"}} recorded so far."""
    cnt = _I32(0)
    _check(_lib.msc_profile_read(context(device), None, 0, ctypes.byref(cnt)),
           "msc_profile_read")
    arr = (msc_phase * max(1, cnt.value))()
    _check(_lib.msc_profile_read(context(device), arr, cnt.value,
                                 ctypes.byref(cnt)), "msc_profile_read")
    return {arr[i].name.decode(): dict(launches=arr[i].launches,
                                       total_ms=arr[i].total_ms,
                                       bytes=arr[i].bytes)
            for i in range(cnt.value)}


def cc_label_grid_into(mask, labels, dims=None, stream=None):
    if dims is None:
        dims = grid_dims(mask.shape)
    code = _lib.cc_label_grid(
        context(mask.device.index), _dev_ptr(mask, torch.uint8, "mask"),
        _dims_arg(dims), _dev_ptr(labels, torch.int64, "labels"),
        _stream(mask, stream))
    _check(code, "cc_label_grid")


def cc_label_grid(mask: torch.Tensor, stream=None) -> torch.Tensor:
    """Components of a uint8 feature mask on the grid; int64 labels, flat."""
    labels = torch.empty(mask.numel(), dtype=torch.int64, device=mask.device)
    cc_label_grid_into(mask, labels, stream=stream)
    return labels


def cc_label_grid_batched_into(masks, labels, dims=None, stream=None):
    """Label several uint8 masks (any shapes) in shared launches; `labels`
    holds one int64 tensor per mask."""
    if not masks:
        return
    dims = dims or [grid_dims(m.shape) for m in masks]
    if len(labels) != len(masks):
        raise ValueError("one label tensor per mask")
    arr = (msc_mask * len(masks))()
    for i, (m, lab, d) in enumerate(zip(masks, labels, dims)):
        if lab.numel() < m.numel():
            raise ValueError(f"labels {i} shorter than its mask")
        arr[i].mask = _dev_ptr(m, torch.uint8, "mask")
        for k in range(3):
            arr[i].dims[k] = int(d[k])
        arr[i].labels = _dev_ptr(lab, torch.int64, "labels")
    code = _lib.cc_label_grid_batched(context(masks[0].device.index),
                                      len(masks), arr,
                                      _stream(masks[0], stream))
    _check(code, "cc_label_grid_batched")


def cc_label_grid_batched(masks, stream=None):
    """Batched cc_label_grid; one flat int64 label tensor per mask."""
    labels = [torch.empty(m.numel(), dtype=torch.int64, device=m.device)
              for m in masks]
    cc_label_grid_batched_into(masks, labels, stream=stream)
    return labels


def workspace_size(kind: int, dims_list, device: int | None = None) -> int:
    """Scratch bytes one call needs: kind REQ_SEGMENT (asc, desc and ms
    wanted) or REQ_CC_GRID, over fields / masks of the given dims."""
    n = len(dims_list)
    if kind == REQ_SEGMENT:
        arr = (msc_field * n)()
        for i, d in enumerate(dims_list):
            for k in range(3):
                arr[i].dims[k] = int(d[k])
            arr[i].field = arr[i].asc = arr[i].desc = arr[i].ms = 1
    else:
        arr = (msc_mask * n)()
        for i, d in enumerate(dims_list):
            for k in range(3):
                arr[i].dims[k] = int(d[k])
            arr[i].mask = arr[i].labels = 1
    out = ctypes.c_size_t(0)
    _check(_lib.msc_workspace_size(context(device), int(kind), n,
                                   ctypes.cast(arr, _P), ctypes.byref(out)),
           "msc_workspace_size")
    return out.value


def set_workspace(buf, device: int | None = None):
    """Make the device's context carve its scratch from `buf` (a uint8 CUDA
    tensor kept alive by the caller, 256-byte aligned), or from memory the
    library owns again when `buf` is None."""
    if buf is None:
        code = _lib.msc_set_workspace(context(device), None, 0)
    else:
        code = _lib.msc_set_workspace(context(buf.device.index),
                                      buf.data_ptr(), buf.numel())
    _check(code, "msc_set_workspace")


INJECT_ENOMEM, INJECT_EHIP = 1, 2


def debug_inject(what: int, after: int = 0):
    """Arm host-side fault injection: after `after` more successful checks
    of the kind (INJECT_ENOMEM: allocations, INJECT_EHIP: HIP runtime
    calls), the next one fails once; after < 0 disarms."""
    _check(_lib.msc_debug_inject(int(what), int(after)), "msc_debug_inject")


def cc_label_grid_noalloc_into(mask, labels, dims=None, stream=None):
    """cc_label_grid into a caller tensor through the entry point that
    allocates nothing (current device; at most 2^27 vertices)."""
    if dims is None:
        dims = grid_dims(mask.shape)
    code = _lib.cc_label_grid_noalloc(
        _dev_ptr(mask, torch.uint8, "mask"), _dims_arg(dims),
        _dev_ptr(labels, torch.int64, "labels"), _stream(mask, stream))
    _check(code, "cc_label_grid_noalloc")


def cc_label_grid_ranks(mask: torch.Tensor, ranks: int, dims=None,
                        stream=None) -> torch.Tensor:
    """cc_label_grid through `ranks` virtual z-slab ranks on one device
    (slab-local labelling, then the exchange across slab boundaries)."""
    labels = torch.empty(mask.numel(), dtype=torch.int64, device=mask.device)
    cc_label_grid_ranks_into(mask, ranks, labels, dims, stream)
    return labels


def cc_label_grid_ranks_into(mask, ranks, labels, dims=None, stream=None):
    if dims is None:
        dims = grid_dims(mask.shape)
    code = _lib.cc_label_grid_ranks(
        context(mask.device.index), _dev_ptr(mask, torch.uint8, "mask"),
        _dims_arg(dims), int(ranks), _dev_ptr(labels, torch.int64, "labels"),
        _stream(mask, stream))
    _check(code, "cc_label_grid_ranks")


def cc_label_csr_into(row_ptr, col_idx, labels, mask=None, stream=None):
    n = row_ptr.numel() - 1
    code = _lib.cc_label_csr(
        context(row_ptr.device.index), int(n),
        _dev_ptr(row_ptr, torch.int64, "row_ptr"),
        _dev_ptr(col_idx, torch.int32, "col_idx"),
        _dev_ptr(mask, torch.uint8, "mask"),
        _dev_ptr(labels, torch.int64, "labels"), _stream(row_ptr, stream))
    _check(code, "cc_label_csr")


def cc_label_csr(row_ptr, col_idx, mask=None, stream=None) -> torch.Tensor:
    """Components of a CSR graph (optionally restricted to a mask)."""
    n = row_ptr.numel() - 1
    labels = torch.empty(n, dtype=torch.int64, device=row_ptr.device)
    cc_label_csr_into(row_ptr, col_idx, labels, mask, stream)
    return labels


def pointer_jump(d: torch.Tensor, rounds: int = 0, synchronous: bool = False,
                 stream=None) -> torch.Tensor:
    """Compress an int64 pointer forest in place (see msc_pointer_jump)."""
    code = _lib.msc_pointer_jump(
        context(d.device.index), _dev_ptr(d, torch.int64, "d"), d.numel(),
        int(rounds), int(bool(synchronous)), _stream(d, stream))
    _check(code, "msc_pointer_jump")
    return d


# ---------------------------------------------------------------------------
# Serving: request queue with continuous batching (msc_queue_* in msc.h)
# ---------------------------------------------------------------------------

REQ_SEGMENT, REQ_CC_GRID = 1, 2


class msc_request(ctypes.Structure):
    _fields_ = [("kind", _I32), ("dims", _I64 * 3), ("host_input", _P)]


class msc_result(ctypes.Structure):
    _fields_ = [("kind", _I32), ("status", _I32), ("n", _I64), ("asc", _P),
                ("desc", _P), ("ms", _P), ("labels", _P),
                ("t_submit_ns", _I64), ("t_start_ns", _I64),
                ("t_done_ns", _I64), ("batch_size", _I32)]


class msc_queue_stats(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_size_t), ("arena_used", ctypes.c_size_t),
                ("workspace_reserved", ctypes.c_size_t), ("pending", _I64),
                ("running", _I64), ("finished", _I64),
                ("arena_size", ctypes.c_size_t), ("launches", _I64),
                ("workspace_grows", _I64), ("host_waits", _I64)]


_U64 = ctypes.c_uint64
_QSIGS = {
    "msc_queue_create": ([_I32, ctypes.c_size_t, _I32, ctypes.POINTER(_P)],
                         _I32),
    "msc_queue_destroy": ([_P], None),
    "msc_submit": ([_P, ctypes.POINTER(msc_request), ctypes.POINTER(_U64)],
                   _I32),
    "msc_poll": ([_P, _U64, ctypes.POINTER(_I32)], _I32),
    "msc_wait": ([_P, _U64], _I32),
    "msc_get_result": ([_P, _U64, ctypes.POINTER(msc_result)], _I32),
    "msc_copy_result": ([_P, _U64, _I32, _P], _I32),
    "msc_cancel": ([_P, _U64], _I32),
    "msc_release": ([_P, _U64], _I32),
    "msc_queue_info": ([_P, ctypes.POINTER(msc_queue_stats)], _I32),
}
for _name, (_args, _res) in _QSIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res
EXPORTS = EXPORTS + tuple(_QSIGS)


class Server:
    """Client of a device-side request queue.  Inputs are host arrays
    (page-locked torch tensors are copied asynchronously); results stay on
    the device until `release`."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30,
                 max_batch: int = 64):
        self._q = _P()
        _check(_lib.msc_queue_create(int(device), int(hbm_budget),
                                     int(max_batch), ctypes.byref(self._q)),
               "msc_queue_create")
        self._keep = {}

    def submit(self, kind: int, host_input) -> int:
        """Queue a segmentation (float32 field) or mask-CC (uint8 mask)
        request; `host_input` is a C-contiguous numpy array, or a host or
        device tensor, of shape [Z, Y, X] (or 1-D / 2-D)."""
        if isinstance(host_input, torch.Tensor):
            if not host_input.is_contiguous():
                raise ValueError("the input must be a contiguous tensor")
            want = torch.float32 if kind == REQ_SEGMENT else torch.uint8
            if host_input.dtype != want:
                raise TypeError(f"host_input must be {want}")
            ptr = host_input.data_ptr()
        else:
            import numpy as np
            want = np.float32 if kind == REQ_SEGMENT else np.uint8
            if host_input.dtype != want or not host_input.flags["C_CONTIGUOUS"]:
                raise TypeError(f"host_input must be contiguous {want}")
            ptr = host_input.ctypes.data
        req = msc_request()
        req.kind = int(kind)
        for k, d in enumerate(grid_dims(host_input.shape)):
            req.dims[k] = d
        req.host_input = ptr
        t = _U64(0)
        _check(_lib.msc_submit(self._q, ctypes.byref(req), ctypes.byref(t)),
               "msc_submit")
        self._keep[t.value] = host_input
        return t.value

    def poll(self, ticket: int) -> int:
        st = _I32(0)
        _check(_lib.msc_poll(self._q, ticket, ctypes.byref(st)), "msc_poll")
        return st.value

    def wait(self, ticket: int) -> int:
        return _lib.msc_wait(self._q, ticket)

    def result(self, ticket: int) -> dict:
        r = msc_result()
        _check(_lib.msc_get_result(self._q, ticket, ctypes.byref(r)),
               "msc_get_result")
        return {k: getattr(r, k) for k, _ in msc_result._fields_}

    def copy_output(self, ticket: int, which: int):
        """Host copy of one output of a finished request: 0 asc, 1 desc,
        2 ms (int32) of a segmentation, 3 labels (int64) of a CC."""
        import numpy as np
        r = self.result(ticket)
        a = np.empty(r["n"], np.int64 if which == 3 else np.int32)
        _check(_lib.msc_copy_result(self._q, ticket, int(which),
                                    a.ctypes.data_as(_P)), "msc_copy_result")
        return a

    def fetch(self, ticket: int):
        """Host copies of a finished request's outputs: (asc, desc, ms) for a
        segmentation, labels for a CC."""
        r = self.result(ticket)
        if r["status"] != MSC_OK:
            raise MscError(r["status"], "request")
        if r["kind"] == REQ_CC_GRID:
            return self.copy_output(ticket, 3)
        return tuple(self.copy_output(ticket, w) for w in range(3))

    def cancel(self, ticket: int):
        _check(_lib.msc_cancel(self._q, ticket), "msc_cancel")

    def release(self, ticket: int):
        _check(_lib.msc_release(self._q, ticket), "msc_release")
        self._keep.pop(ticket, None)

    def info(self) -> dict:
        s = msc_queue_stats()
        _check(_lib.msc_queue_info(self._q, ctypes.byref(s)), "msc_queue_info")
        return {k: getattr(s, k) for k, _ in msc_queue_stats._fields_}

    def close(self):
        if self._q:
            _lib.msc_queue_destroy(self._q)
            self._q = _P()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
