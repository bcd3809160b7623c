"""Brute-force re-statement of the segmentation and CC definitions for tiny
grids, vectorised over a batch of fields -- TEST INFRASTRUCTURE ONLY.

It is written independently of ``msc_oracle.c`` so that the two can pin each
other:
  * adjacency comes from the lattice characterisation of the Freudenthal
    triangulation (u and v share an edge iff their coordinate difference is a
    non-zero vector with entries in {0, 1} or in {0, -1}), not from the Kuhn
    tetrahedra the C oracle enumerates;
  * roots come from iterating the successor map n times (a fixed point is
    reached after at most n steps), not from walking;
  * Morse-Smale cells come from an all-pairs comparison, not from sorting;
  * components come from min-label propagation over the edges, iterated n
    times, not from union-find.
"""
from __future__ import annotations

import itertools

import numpy as np


def coords(X: int, Y: int, Z: int):
    return [(v % X, (v // X) % Y, v // (X * Y)) for v in range(X * Y * Z)]


def edges(X: int, Y: int, Z: int):
    """Undirected edge list (u < v) of the Freudenthal grid."""
    cs = coords(X, Y, Z)
    out = []
    for u, v in itertools.combinations(range(X * Y * Z), 2):
        d = [cs[v][i] - cs[u][i] for i in range(3)]
        if max(abs(t) for t in d) > 1:
            continue
        if all(t >= 0 for t in d) or all(t <= 0 for t in d):
            out.append((u, v))
    return out


def closed_neighbourhoods(X: int, Y: int, Z: int):
    n = X * Y * Z
    nb = [[v] for v in range(n)]
    for u, v in edges(X, Y, Z):
        nb[u].append(v)
        nb[v].append(u)
    return [sorted(s) for s in nb]


def steepest_batch(F: np.ndarray, X: int, Y: int, Z: int, direction: int):
    """F: [B, n] float32 fields.  Returns [B, n] successor ids."""
    B, n = F.shape
    nbh = closed_neighbourhoods(X, Y, Z)
    S = np.empty((B, n), np.int64)
    for v in range(n):
        best = np.full(B, v, np.int64)
        for u in nbh[v]:
            fu = F[:, u]
            fb = np.take_along_axis(F, best[:, None], 1)[:, 0]
            if direction > 0:
                better = (fu > fb) | ((fu == fb) & (u > best))
            else:
                better = (fu < fb) | ((fu == fb) & (u < best))
            best = np.where(better, u, best)
        S[:, v] = best
    return S


def roots_batch(S: np.ndarray) -> np.ndarray:
    R = S.copy()
    for _ in range(S.shape[1]):
        R = np.take_along_axis(S, R, 1)
    return R


def ms_batch(A: np.ndarray, D: np.ndarray) -> np.ndarray:
    B, n = A.shape
    M = np.tile(np.arange(n, dtype=np.int64), (B, 1))
    for v in range(n):
        for u in range(v - 1, -1, -1):
            same = (A[:, u] == A[:, v]) & (D[:, u] == D[:, v])
            M[:, v] = np.where(same, u, M[:, v])
    return M


def segment_batch(F: np.ndarray, X: int, Y: int, Z: int):
    F = np.asarray(F, np.float32)
    A = roots_batch(steepest_batch(F, X, Y, Z, +1))
    D = roots_batch(steepest_batch(F, X, Y, Z, -1))
    return A, D, ms_batch(A, D)


def cc_batch(M: np.ndarray, X: int, Y: int, Z: int) -> np.ndarray:
    """M: [B, n] {0,1} masks.  Label = smallest id of the component, -1
    for unmasked vertices."""
    M = np.asarray(M).astype(bool)
    B, n = M.shape
    big = np.int64(n)
    L = np.where(M, np.arange(n, dtype=np.int64)[None, :], big)
    E = edges(X, Y, Z)
    for _ in range(n):
        for u, v in E:
            both = M[:, u] & M[:, v]
            m = np.minimum(L[:, u], L[:, v])
            L[:, u] = np.where(both, m, L[:, u])
            L[:, v] = np.where(both, m, L[:, v])
    return np.where(M, L, -1)


def segment_graph(rows, F: np.ndarray):
    """Segmentation on a general graph for a batch of fields: `rows[v]` lists
    the neighbours of v (the closed neighbourhood adds v), F is [B, n].  The
    successor is the candidate no other candidate beats under (f, id) --
    found by comparing every pair of candidates, not by a running maximum."""
    F = np.asarray(F, np.float32)
    B, n = F.shape

    def beats(b, u, w):
        return (F[b, u] > F[b, w]) or (F[b, u] == F[b, w] and u > w)

    Sp = np.empty((B, n), np.int64)
    Sm = np.empty((B, n), np.int64)
    for b in range(B):
        for v in range(n):
            cand = sorted(set([v] + [int(u) for u in rows[v]]))
            top = [u for u in cand if not any(beats(b, w, u) for w in cand
                                              if w != u)]
            bot = [u for u in cand if not any(beats(b, u, w) for w in cand
                                              if w != u)]
            assert len(top) == 1 and len(bot) == 1
            Sp[b, v], Sm[b, v] = top[0], bot[0]
    A = roots_batch(Sp)
    D = roots_batch(Sm)
    return A, D, ms_batch(A, D)


def link_components(f: np.ndarray, X: int, Y: int, Z: int):
    """(lc, uc) per vertex from the lattice characterisation alone: the link
    of v is the graph on v's neighbours in which two are joined when they
    are neighbours of each other (the Freudenthal triangulation is a flag
    complex, so such a pair and v span a triangle)."""
    f = np.asarray(f, np.float32).reshape(-1)
    n = X * Y * Z
    nb = [set() for _ in range(n)]
    for u, v in edges(X, Y, Z):
        nb[u].add(v)
        nb[v].add(u)

    def below(a, b):
        return f[a] < f[b] or (f[a] == f[b] and a < b)

    def count(v, side):
        verts = [u for u in nb[v] if (below(v, u) if side > 0 else below(u, v))]
        seen, comps = set(), 0
        for s in verts:
            if s in seen:
                continue
            comps += 1
            stack = [s]
            seen.add(s)
            while stack:
                a = stack.pop()
                for b in verts:
                    if b not in seen and b in nb[a]:
                        seen.add(b)
                        stack.append(b)
        return comps

    lc = np.array([count(v, -1) for v in range(n)], np.int64)
    uc = np.array([count(v, +1) for v in range(n)], np.int64)
    return lc, uc
