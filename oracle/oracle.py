"""CPU oracle for path-compression Morse-Smale segmentation and connected
components -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` import this module.  It loads ``liborc.so`` built by gcc from
``msc_oracle.c`` (plain serial C, see that file's header for the readings it
takes) and wraps it for numpy arrays.  It shares no code with the HIP library
and never imports it.

Paper: arXiv 2409.03771.  Definitions followed:
  * steepest ascent / descent and the manifold maps -- background section
    "Ascending and Descending Manifolds" and the initialisation of Alg. 1;
  * the (value, id) total order -- preprocessing section (simulation of
    simplicity by sorting on value with ties broken by global id);
  * Morse-Smale cells as (ascent root, descent root) classes -- methods
    section "Ascending and Descending Segmentation";
  * connected components of the masked graph, unmasked label -1 -- Alg. 3.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msc_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, -O3)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        L.orc_stencil.argtypes = [P]
        L.orc_stencil.restype = ctypes.c_int
        L.orc_successors.argtypes = [P, I64, I64, I64, P, P]
        L.orc_successors.restype = None
        L.orc_successors_csr.argtypes = [P, I64, P, P, P, P]
        L.orc_successors_csr.restype = None
        L.orc_critical.argtypes = [P, I64, I64, I64, P, P, P]
        L.orc_critical.restype = None
        L.orc_extremum_edges.argtypes = [P, I64, I64, I64, P, P, P, I64]
        L.orc_extremum_edges.restype = I64
        L.orc_walk_plain.argtypes = [P, I64, P]
        L.orc_walk_plain.restype = None
        L.orc_walk_memo.argtypes = [P, I64, P, P]
        L.orc_walk_memo.restype = None
        L.orc_walk_from.argtypes = [P, I64, I64, I64, I64, ctypes.c_int]
        L.orc_walk_from.restype = I64
        L.orc_ms_cells.argtypes = [P, P, I64, P, P]
        L.orc_ms_cells.restype = I64
        L.orc_sync_doubling.argtypes = [P, I64, ctypes.c_int, P]
        L.orc_sync_doubling.restype = None
        L.orc_cc_grid_uf.argtypes = [P, I64, I64, I64, P]
        L.orc_cc_grid_uf.restype = I64
        L.orc_cc_grid_bfs.argtypes = [P, I64, I64, I64, P, P]
        L.orc_cc_grid_bfs.restype = I64
        L.orc_cc_csr_uf.argtypes = [I64, P, P, P, P]
        L.orc_cc_csr_uf.restype = I64
        L.orc_cc_csr_bfs.argtypes = [I64, P, P, P, P, P]
        L.orc_cc_csr_bfs.restype = I64
        L.orc_check_roots.argtypes = [P, I64, I64, I64, P, ctypes.c_int, I64,
                                      I64, P]
        L.orc_check_roots.restype = I64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(f: np.ndarray):
    """(X, Y, Z) of a field stored as [Z][Y][X] (x fastest)."""
    if f.ndim == 1:
        return f.shape[0], 1, 1
    if f.ndim == 2:
        return f.shape[1], f.shape[0], 1
    return f.shape[2], f.shape[1], f.shape[0]


def stencil() -> np.ndarray:
    """Edge vectors (dx,dy,dz) of the Freudenthal triangulation, [14, 3]."""
    out = np.zeros((14, 3), np.int32)
    n = lib().orc_stencil(_p(out))
    return out[:n].copy()


def successors(f: np.ndarray):
    """(S+, S-) one-step steepest ascent / descent over {v} u N(v)."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    X, Y, Z = _dims(f)
    n = X * Y * Z
    sp = np.empty(n, np.int32)
    sm = np.empty(n, np.int32)
    lib().orc_successors(_p(f), X, Y, Z, _p(sp), _p(sm))
    return sp, sm


def walk(succ: np.ndarray, memo: bool | None = None) -> np.ndarray:
    succ = np.ascontiguousarray(succ, dtype=np.int32)
    n = succ.shape[0]
    root = np.empty(n, np.int32)
    if memo is None:
        memo = n > 128 ** 3
    if memo:
        stack = np.empty(n, np.int32)
        lib().orc_walk_memo(_p(succ), n, _p(root), _p(stack))
    else:
        lib().orc_walk_plain(_p(succ), n, _p(root))
    return root


def walk_from(f: np.ndarray, v: int, direction: int) -> int:
    """Extremum reached from vertex v (direction +1 ascent, -1 descent)."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    X, Y, Z = _dims(f)
    return int(lib().orc_walk_from(_p(f), X, Y, Z, int(v), int(direction)))


def ms_cells(asc: np.ndarray, desc: np.ndarray):
    """(ms, number of cells): ms[v] = smallest id with the same pair."""
    asc = np.ascontiguousarray(asc, dtype=np.int32)
    desc = np.ascontiguousarray(desc, dtype=np.int32)
    n = asc.shape[0]
    ms = np.empty(n, np.int32)
    order = np.empty(n, np.int64)
    k = lib().orc_ms_cells(_p(asc), _p(desc), n, _p(ms), _p(order))
    return ms, int(k)


def segment(f: np.ndarray, memo: bool | None = None):
    """Full Morse-Smale segmentation: (asc, desc, ms) int32 arrays, flat."""
    sp, sm = successors(f)
    asc = walk(sp, memo)
    desc = walk(sm, memo)
    ms, _ = ms_cells(asc, desc)
    return asc, desc, ms


def successors_csr(row_ptr: np.ndarray, col_idx: np.ndarray, f: np.ndarray):
    """(S+, S-) over the closed CSR neighbourhoods {v} u row(v)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    f = np.ascontiguousarray(f, dtype=np.float32).reshape(-1)
    n = row_ptr.shape[0] - 1
    assert f.shape[0] == n
    sp = np.empty(n, np.int32)
    sm = np.empty(n, np.int32)
    lib().orc_successors_csr(_p(f), n, _p(row_ptr), _p(col_idx), _p(sp),
                             _p(sm))
    return sp, sm


def segment_csr(row_ptr: np.ndarray, col_idx: np.ndarray, f: np.ndarray,
                memo: bool | None = None):
    """Morse-Smale segmentation of a field on the vertices of a complex
    given as CSR adjacency: (asc, desc, ms) int32 arrays."""
    sp, sm = successors_csr(row_ptr, col_idx, f)
    asc = walk(sp, memo)
    desc = walk(sm, memo)
    ms, _ = ms_cells(asc, desc)
    return asc, desc, ms


def csr_from_tets(n: int, tets: np.ndarray):
    """(row_ptr int64 [n+1], col_idx int32) of the 1-skeleton of a
    tetrahedral complex: u is a neighbour of v when some tetrahedron holds
    both and u != v; rows sorted, no duplicates, symmetric.  Written as its
    definition: every tetrahedron's six vertex pairs in both directions,
    self pairs dropped, duplicates merged by np.unique."""
    t = np.asarray(tets, np.int64).reshape(-1, 4)
    pairs = [(i, j) for i in range(4) for j in range(4) if i != j]
    a = np.concatenate([t[:, i] for i, _ in pairs])
    b = np.concatenate([t[:, j] for _, j in pairs])
    keep = a != b
    keys = np.unique(a[keep] * np.int64(n) + b[keep])
    src, dst = keys // n, keys % n
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return row_ptr, dst.astype(np.int32)


def critical(f: np.ndarray):
    """(lc, uc, chi): components of each vertex's lower and upper link and
    the Euler characteristic of its lower link (flat arrays)."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    X, Y, Z = _dims(f)
    n = X * Y * Z
    lc = np.empty(n, np.uint8)
    uc = np.empty(n, np.uint8)
    chi = np.empty(n, np.int32)
    lib().orc_critical(_p(f), X, Y, Z, _p(lc), _p(uc), _p(chi))
    return lc, uc, chi


def extremum_edges(f: np.ndarray, asc: np.ndarray, desc: np.ndarray):
    """int32 [m, 3] rows (vertex, extremum, +1 / -1) of the extremum
    graph, by increasing vertex, ascending edges first."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    X, Y, Z = _dims(f)
    asc = np.ascontiguousarray(asc, dtype=np.int32)
    desc = np.ascontiguousarray(desc, dtype=np.int32)
    m = lib().orc_extremum_edges(_p(f), X, Y, Z, _p(asc), _p(desc),
                                 None, 0)
    out = np.empty((max(m, 1), 3), np.int32)
    lib().orc_extremum_edges(_p(f), X, Y, Z, _p(asc), _p(desc), _p(out), m)
    return out[:m]


def sync_doubling(d: np.ndarray, rounds: int) -> np.ndarray:
    d = np.array(d, dtype=np.int64, copy=True)
    tmp = np.empty_like(d)
    lib().orc_sync_doubling(_p(d), d.shape[0], int(rounds), _p(tmp))
    return d


def cc_grid(mask: np.ndarray, method: str = "uf"):
    """(label int64 flat, #components) on the Freudenthal grid graph."""
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    X, Y, Z = _dims(mask)
    n = X * Y * Z
    label = np.empty(n, np.int64)
    if method == "uf":
        k = lib().orc_cc_grid_uf(_p(mask), X, Y, Z, _p(label))
    else:
        q = np.empty(n, np.int64)
        k = lib().orc_cc_grid_bfs(_p(mask), X, Y, Z, _p(label), _p(q))
    return label, int(k)


def cc_csr(row_ptr: np.ndarray, col_idx: np.ndarray, mask=None,
           method: str = "uf"):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = row_ptr.shape[0] - 1
    label = np.empty(n, np.int64)
    mp = None
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        mp = _p(mask)
    if method == "uf":
        k = lib().orc_cc_csr_uf(n, _p(row_ptr), _p(col_idx), mp, _p(label))
    else:
        q = np.empty(n, np.int64)
        k = lib().orc_cc_csr_bfs(n, _p(row_ptr), _p(col_idx), mp, _p(label),
                                 _p(q))
    if k == -2:
        raise ValueError("col_idx out of range")
    return label, int(k)


def check_roots(f: np.ndarray, root: np.ndarray, direction: int,
                threads: int = 8, chunk: int = 1 << 22):
    """Local-consistency check of a root map over all vertices; returns
    (violations, first bad vertex or -1).  Runs chunks on a thread pool (the
    C call releases the GIL)."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    root = np.ascontiguousarray(root, dtype=np.int32)
    X, Y, Z = _dims(f)
    n = X * Y * Z
    L = lib()

    def one(v0):
        first = ctypes.c_int64(-1)
        bad = L.orc_check_roots(_p(f), X, Y, Z, _p(root), int(direction), v0,
                                min(n, v0 + chunk), ctypes.byref(first))
        return bad, first.value

    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(one, range(0, n, chunk)))
    bad = sum(r[0] for r in res)
    firsts = [r[1] for r in res if r[1] >= 0]
    return bad, (min(firsts) if firsts else -1)
