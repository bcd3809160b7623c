"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds none of the segmentation or connected-components
arithmetic: it only draws fields, masks, meshes and request traces.

Field recipe (sum of Gaussian bumps plus uniform noise), evaluated in float64
and rounded once to float32:

    f(p) = sum_k A_k exp(-|p - c_k|^2 / (2 s_k^2)) + e(p)

with, drawn in this order from ``numpy.random.default_rng(seed)``:
  centres c_k ~ U[0, n_axis - 1] per axis (x, y, z), shape [nb, 3];
  amplitudes A_k ~ U[-1, 1];
  widths s_k ~ U[0.02, 0.1] * scale, scale = geometric mean of the dims;
  noise e ~ U[-1e-4, 1e-4], one draw per vertex in id order.
The Gaussian is evaluated as the product of its three 1-D factors.  The field
is stored [Z][Y][X] (x fastest), so vertex (x, y, z) has id x + X*y + X*Y*z.
"""
from __future__ import annotations

import math

import numpy as np

NOISE = 1e-4


def gaussian_params(dims, nbumps: int, seed: int):
    X, Y, Z = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    hi = np.array([X - 1, Y - 1, Z - 1], np.float64)
    centres = rng.uniform(0.0, 1.0, size=(nbumps, 3)) * hi
    amps = rng.uniform(-1.0, 1.0, size=nbumps)
    scale = (X * Y * Z) ** (1.0 / 3.0)
    sigmas = rng.uniform(0.02, 0.1, size=nbumps) * scale
    return rng, centres, amps, sigmas


def _factors(n: int, c: np.ndarray, s: np.ndarray) -> np.ndarray:
    t = np.arange(n, dtype=np.float64)[None, :] - c[:, None]
    return np.exp(-(t * t) / (2.0 * s[:, None] ** 2))


def gaussian_field(dims, nbumps: int, seed: int, noise: bool = True,
                   z_chunk: int = 16, device=None):
    """float32 field of shape [Z, Y, X]: a numpy array, or a torch tensor
    on `device` when one is given (the bump sum is then evaluated there in
    float64; the noise is the same numpy draw)."""
    X, Y, Z = (int(d) for d in dims)
    rng, c, a, s = gaussian_params((X, Y, Z), nbumps, seed)
    gx = _factors(X, c[:, 0], s)          # [nb, X]
    gy = _factors(Y, c[:, 1], s)          # [nb, Y]
    gz = _factors(Z, c[:, 2], s) * a[:, None]  # [nb, Z], amplitude folded in
    if device is not None:
        import torch
        out_t = torch.empty((Z, Y, X), dtype=torch.float32, device=device)
        gx_t = torch.from_numpy(gx).to(device)
        gy_t = torch.from_numpy(gy).to(device)
        gz_t = torch.from_numpy(gz).to(device)
        zc = max(z_chunk, 64)
        for z0 in range(0, Z, zc):
            z1 = min(Z, z0 + zc)
            P = gz_t[:, z0:z1, None] * gy_t[:, None, :]
            blk = P.reshape(P.shape[0], -1).T @ gx_t
            if noise:
                e = rng.uniform(-NOISE, NOISE, size=tuple(blk.shape))
                blk += torch.from_numpy(e).to(device)
            out_t[z0:z1] = blk.reshape(z1 - z0, Y, X).to(torch.float32)
        return out_t
    out = np.empty((Z, Y, X), np.float32)
    for z0 in range(0, Z, z_chunk):
        z1 = min(Z, z0 + z_chunk)
        P = gz[:, z0:z1, None] * gy[:, None, :]              # [nb, zc, Y]
        blk = P.reshape(P.shape[0], -1).T @ gx                # [zc*Y, X]
        if noise:
            blk += rng.uniform(-NOISE, NOISE, size=blk.shape)
        out[z0:z1] = blk.reshape(z1 - z0, Y, X).astype(np.float32)
    return out


def perlin_perm(seed: int) -> np.ndarray:
    """The lattice hash of the noise: a seeded permutation of 0..255,
    repeated once so that sums of two entries index it directly."""
    p = np.random.default_rng(seed).permutation(256).astype(np.int64)
    return np.concatenate([p, p])


def perlin_field(dims, seed: int, frequency: float = 0.1,
                 amplitude: float = 1.0, z_chunk: int = 8, device=None):
    """float32 field [Z, Y, X] of one layer of Perlin gradient noise,
    f(x, y, z) = amplitude * noise(frequency * (x, y, z)).

    The noise is Perlin's lattice gradient noise (Perlin 1985) in its
    improved form (Perlin 2002): the lattice corners of the point's cell
    each hash, through a seeded permutation, to one of twelve gradient
    directions (the cube's edge midpoints, two repeated); the dot products
    of those gradients with the offsets to the point are blended with the
    quintic fade 6t^5 - 15t^4 + 10t^3 along each axis.  It is zero at lattice
    points.  Evaluated in float64 with torch (on `device`, default CPU) and
    rounded once to float32; returns a torch tensor when `device` is given,
    a numpy array otherwise."""
    import torch
    X, Y, Z = (int(d) for d in dims)
    dev = torch.device("cpu") if device is None else torch.device(device)
    perm = torch.from_numpy(perlin_perm(seed)).to(dev)
    out = torch.empty((Z, Y, X), dtype=torch.float32, device=dev)
    xs = torch.arange(X, dtype=torch.float64, device=dev) * frequency
    ys = torch.arange(Y, dtype=torch.float64, device=dev) * frequency
    xi0 = torch.floor(xs)
    yi0 = torch.floor(ys)

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    def grad(h, x, y, z):
        h = h & 15
        u = torch.where(h < 8, x, y)
        v = torch.where(h < 4, y, torch.where((h == 12) | (h == 14), x, z))
        return (torch.where((h & 1) == 0, u, -u) +
                torch.where((h & 2) == 0, v, -v))

    def lerp(t, a, b):
        return a + t * (b - a)

    fx = (xs - xi0)[None, None, :]
    fy = (ys - yi0)[None, :, None]
    u = fade(fx)
    v = fade(fy)
    Xi = (xi0.to(torch.int64) & 255)[None, None, :]
    Yi = (yi0.to(torch.int64) & 255)[None, :, None]
    for z0 in range(0, Z, z_chunk):
        z1 = min(Z, z0 + z_chunk)
        zs = torch.arange(z0, z1, dtype=torch.float64, device=dev) * frequency
        zi0 = torch.floor(zs)
        fz = (zs - zi0)[:, None, None]
        w = fade(fz)
        Zi = (zi0.to(torch.int64) & 255)[:, None, None]
        A = perm[Xi] + Yi
        B = perm[Xi + 1] + Yi
        AA, AB = perm[A] + Zi, perm[A + 1] + Zi
        BA, BB = perm[B] + Zi, perm[B + 1] + Zi
        n0 = lerp(v, lerp(u, grad(perm[AA], fx, fy, fz),
                          grad(perm[BA], fx - 1, fy, fz)),
                  lerp(u, grad(perm[AB], fx, fy - 1, fz),
                       grad(perm[BB], fx - 1, fy - 1, fz)))
        n1 = lerp(v, lerp(u, grad(perm[AA + 1], fx, fy, fz - 1),
                          grad(perm[BA + 1], fx - 1, fy, fz - 1)),
                  lerp(u, grad(perm[AB + 1], fx, fy - 1, fz - 1),
                       grad(perm[BB + 1], fx - 1, fy - 1, fz - 1)))
        out[z0:z1] = (amplitude * lerp(w, n0, n1)).to(torch.float32)
    return out if device is not None else out.numpy()


def normalized_mask(f, level: float):
    """uint8 feature mask of the threshold study: the field is normalised
    to [0, 1] by its minimum and maximum, and a vertex is a feature when its
    normalised value is above `level` (0.9, 0.5 and 0.1 in the study).
    Works on numpy arrays and torch tensors alike (the comparison is
    f - min > level * (max - min), in float64)."""
    try:
        import torch
        if isinstance(f, torch.Tensor):
            lo, hi = f.min().double(), f.max().double()
            return ((f.double() - lo) > level * (hi - lo)).to(torch.uint8)
    except ImportError:  # pragma: no cover
        pass
    lo, hi = float(f.min()), float(f.max())
    return ((f.astype(np.float64) - lo) > level * (hi - lo)).astype(np.uint8)


WORKLOADS = {
    # name: (kind, dims, bumps, seed); Perlin fields take frequency 0.1 and
    # amplitude 1 (the paper's synthetic workload).
    "gauss64": ("gauss", (64, 64, 64), 8, 0),
    "gauss1024": ("gauss", (1024, 1024, 1024), 512, 1),
    "perlin512": ("perlin", (512, 512, 512), 0, 5),
    "perlin1024": ("perlin", (1024, 1024, 1024), 0, 5),
    # z-planes [0, 256) of the 2048^3 Perlin field: one GPU's share when the
    # 2048^3 field is split into eight z-slabs (its 2^33 ids do not fit the
    # int32 labels of a single call).
    "perlin2048s": ("perlin", (2048, 2048, 256), 0, 5),
}


def config_field(name: str, device=None):
    """The named single-field workloads: "gauss64" (64^3, 8 bumps, seed 0),
    "gauss1024" (1024^3, 512 bumps, seed 1), and one-layer Perlin noise at
    frequency 0.1 and amplitude 1, "perlin512" and "perlin1024" (seed 5),
    and "perlin2048s", the first of eight 2048x2048x256 z-slabs of the
    2048^3 field (the noise at a point does not depend on the grid's
    extent, so the slab is the field generated at its own dims)."""
    alias = {"c1": "gauss64", "c2": "gauss1024"}
    kind, dims, nb, seed = WORKLOADS[alias.get(name, name)]
    if kind == "perlin":
        return perlin_field(dims, seed, device=device)
    return gaussian_field(dims, nb, seed, device=device)


def threshold_mask(f, quantile: float = 0.7):
    """uint8 mask f > tau, tau the k-th smallest value, k = floor(q*N)
    (0-based): about (1-q) of the vertices are foreground.  A torch tensor
    gives a tensor on its device (tau from a sort there)."""
    try:
        import torch
        if isinstance(f, torch.Tensor):
            flat = f.reshape(-1)
            k = min(max(int(math.floor(quantile * flat.numel())), 0),
                    flat.numel() - 1)
            tau = torch.sort(flat).values[k]
            return (f > tau).to(torch.uint8)
    except ImportError:  # pragma: no cover
        pass
    flat = f.reshape(-1)
    k = int(math.floor(quantile * flat.size))
    k = min(max(k, 0), flat.size - 1)
    tau = np.partition(flat, k)[k]
    return (f > tau).astype(np.uint8)


def random_field(dims, seed: int, levels: int | None = None) -> np.ndarray:
    """Small test fields: uniform float32, or integers in [0, levels) to
    force ties (exercising the id tie-break)."""
    X, Y, Z = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    if levels is None:
        return rng.standard_normal((Z, Y, X)).astype(np.float32)
    return rng.integers(0, levels, size=(Z, Y, X)).astype(np.float32)


def batch_specs(count: int = 256, seed: int = 3, lo: int = 32, hi: int = 256):
    """Uneven batch: per field (dims, nbumps, field seed); each axis
    round(exp(U[ln lo, ln hi])), bumps ~ U{8..128}."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        d = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=3)))
        nb = int(rng.integers(8, 129))
        specs.append(((int(d[0]), int(d[1]), int(d[2])), nb, seed * 100003 + i))
    return specs


# ---------------------------------------------------------------------------
# Unstructured input: jittered Kuhn tetrahedralisation as CSR adjacency
# ---------------------------------------------------------------------------

_KUHN_EDGES = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0],
                        [1, 0, 1], [0, 1, 1], [1, 1, 1]], np.int64)


def kuhn_csr(n_axis: int, seed: int, nbumps: int | None = None,
             quantile: float = 0.7, jitter: float = 0.25,
             permute: bool = True):
    """Mesh input for CSR connected components.

    Vertices of an n^3 grid, positions jittered by U[-jitter, jitter] per axis
    (topology unchanged), edges of its Kuhn tetrahedralisation, vertex ids
    randomly permuted.  A Gaussian-sum field is evaluated at the jittered
    positions and thresholded at the quantile.  Returns a dict with
    ``row_ptr`` (int64 [n+1]), ``col_idx`` (int32, symmetric, rows sorted),
    ``mask`` (uint8 [n], in permuted ids), ``perm`` (new id of grid vertex
    g) and the explicit-geometry CSR ``fg_row_ptr``/``fg_col_idx`` that
    keeps only edges whose two endpoints are foreground.  ``field`` holds
    the float32 field values in grid order (vertex g at grid id g).  With
    ``permute=False`` the ids are the grid ids (the same draws are made, so
    the field is the same), which makes the CSR the Freudenthal grid's own
    adjacency.
    """
    n3 = n_axis ** 3
    if nbumps is None:
        nbumps = max(1, int(round(512 * (n_axis / 1024.0) ** 3)))
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n3).astype(np.int64)             # grid -> new id
    if not permute:
        perm = np.arange(n3, dtype=np.int64)
    # Field at jittered positions (per-axis jitter, then the bump sum).
    _, c, a, s = gaussian_params((n_axis,) * 3, nbumps, seed)
    g = np.arange(n3, dtype=np.int64)
    f = np.zeros(n3, np.float64)
    chunk = 1 << 22
    for g0 in range(0, n3, chunk):
        gg = g[g0:g0 + chunk]
        p = np.stack([gg % n_axis, (gg // n_axis) % n_axis,
                      gg // (n_axis * n_axis)], 1).astype(np.float64)
        p += rng.uniform(-jitter, jitter, size=p.shape)
        acc = np.zeros(gg.shape[0], np.float64)
        for k in range(nbumps):
            d2 = ((p - c[k]) ** 2).sum(1)
            acc += a[k] * np.exp(-d2 / (2.0 * s[k] ** 2))
        f[g0:g0 + chunk] = acc
    f32 = f.astype(np.float32)
    kq = min(int(math.floor(quantile * n3)), n3 - 1)
    tau = np.partition(f32, kq)[kq]
    fg_grid = (f32 > tau)
    mask = np.empty(n3, np.uint8)
    mask[perm] = fg_grid.astype(np.uint8)

    # Adjacency: for each grid vertex the up-to-14 neighbours.
    offs = np.concatenate([_KUHN_EDGES, -_KUHN_EDGES])
    inv = np.empty(n3, np.int64)
    inv[perm] = g
    rows = []
    for g0 in range(0, n3, chunk):
        new_ids = np.arange(g0, min(n3, g0 + chunk), dtype=np.int64)
        gv = inv[new_ids]
        x, y, z = gv % n_axis, (gv // n_axis) % n_axis, gv // (n_axis * n_axis)
        nb = np.full((gv.shape[0], 14), -1, np.int64)
        for k, (dx, dy, dz) in enumerate(offs):
            xx, yy, zz = x + dx, y + dy, z + dz
            ok = ((xx >= 0) & (xx < n_axis) & (yy >= 0) & (yy < n_axis) &
                  (zz >= 0) & (zz < n_axis))
            gid = xx + n_axis * yy + n_axis * n_axis * zz
            nb[:, k] = np.where(ok, perm[np.where(ok, gid, 0)], -1)
        rows.append(nb.astype(np.int32))
    nbr = np.concatenate(rows)                               # [n3, 14]
    nbr.sort(axis=1)                                         # -1 first
    valid = nbr >= 0
    deg = valid.sum(1)
    row_ptr = np.zeros(n3 + 1, np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    col_idx = nbr[valid]
    # Explicit geometry: keep edges between two foreground vertices.
    keep = valid & (mask[:, None] == 1) & (mask[np.where(valid, nbr, 0)] == 1)
    fdeg = keep.sum(1)
    fg_row_ptr = np.zeros(n3 + 1, np.int64)
    np.cumsum(fdeg, out=fg_row_ptr[1:])
    fg_col_idx = nbr[keep]
    return dict(row_ptr=row_ptr, col_idx=np.ascontiguousarray(col_idx),
                mask=mask, perm=perm, fg_row_ptr=fg_row_ptr,
                fg_col_idx=np.ascontiguousarray(fg_col_idx), field=f32)


def kuhn_tets(n_axis: int, perm: np.ndarray | None = None,
              z_chunk: int = 16) -> np.ndarray:
    """Tetrahedra of the Kuhn subdivision of an n^3 grid of vertices: each
    cube with lower corner p splits into the six tetrahedra
    {p, p+e_a, p+e_a+e_b, p+e_a+e_b+e_c}, (a, b, c) a permutation of the
    axes.  int32 [6 (n-1)^3, 4] vertex ids (grid ids x + n y + n^2 z, or
    perm[grid id] when a permutation is given), cubes in id order."""
    import itertools
    m = n_axis - 1
    if m <= 0:
        return np.zeros((0, 4), np.int32)
    unit = np.eye(3, dtype=np.int64)
    corners = []
    for a, b, c in itertools.permutations(range(3)):
        o = np.zeros(3, np.int64)
        path = [o.copy()]
        for ax in (a, b, c):
            o = o + unit[ax]
            path.append(o.copy())
        corners.append(path)
    corners = np.array(corners)                      # [6, 4, 3]
    off = corners[..., 0] + n_axis * corners[..., 1] + \
        n_axis * n_axis * corners[..., 2]            # [6, 4]
    out = []
    for z0 in range(0, m, z_chunk):
        z = np.arange(z0, min(m, z0 + z_chunk))
        y = np.arange(m)
        x = np.arange(m)
        base = (x[None, None, :] + n_axis * y[None, :, None] +
                n_axis * n_axis * z[:, None, None]).reshape(-1)
        t = base[:, None, None] + off[None, :, :]    # [cubes, 6, 4]
        t = t.reshape(-1, 4)
        out.append(t if perm is None else perm[t])
    return np.ascontiguousarray(np.concatenate(out).astype(np.int32))


def poisson_trace(rate: float, count: int, seed: int = 4, lo: int = 64,
                  hi: int = 512, ms_frac: float = 0.7):
    """Open-loop request trace: arrival times (s), kind ('ms' or 'cc'),
    dims log-uniform per axis, per-request field seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    out = []
    for i in range(count):
        kind = "ms" if rng.uniform() < ms_frac else "cc"
        d = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=3)))
        nb = int(rng.integers(8, 129))
        out.append(dict(t=float(t[i]), kind=kind,
                        dims=(int(d[0]), int(d[1]), int(d[2])), nbumps=nb,
                        seed=seed * 1000003 + i))
    return out
