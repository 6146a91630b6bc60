"""Scalar per-point reference for tiny grids (oracle).

Everything here is a plain Python loop over points, written from the
definitions rather than from the vectorized oracle: the pass of a point is found
from its coordinates alone (the largest power of two h dividing every
coordinate gives the level; the last dimension whose level coordinate is odd
gives the pass), neighbours are looked up one by one, chunk positions are found
by sorting the targets of each chunk, and bitplanes are assembled bit by bit.
Used only to check the vectorized oracle on small inputs.
"""

from __future__ import annotations

import itertools

import numpy as np

from .predict import stencil_1d, quantize_scalar


def _v2(v: int, cap: int) -> int:
    """Exponent of the largest power of two dividing v (cap for v == 0)."""
    if v == 0:
        return cap
    e = 0
    while v % 2 == 0 and e < cap:
        v //= 2
        e += 1
    return e


def levels(dims) -> int:
    m = max(dims)
    if m == 1:
        return 0
    k = 0
    while (1 << k) < m - 1:
        k += 1
    return max(1, k)


def pass_of_point(i, dims, K):
    """(pass index, level, dim) of one point; pass 0 = anchors."""
    D = len(dims)
    e = min(_v2(c, K) for c in i)
    if e >= K:
        return 0, 0, -1
    lev = e + 1
    h = 1 << e
    k = max(j for j in range(D) if (i[j] // h) % 2 == 1)
    return 1 + (K - lev) * D + k, lev, k


def all_points(dims):
    return itertools.product(*[range(d) for d in dims])


def compress_brute(x: np.ndarray, eb: float, interp: int, chunk_log2):
    """Returns dict with xhat, codes {pass: {(chunk, local): q}}, outliers, errq."""
    dims = x.shape
    D = len(dims)
    K = levels(dims)
    dt = x.dtype
    C = [1 << c for c in chunk_log2]
    P = 1 + D * K
    by_pass = {s: [] for s in range(P)}
    for i in all_points(dims):
        s, lev, k = pass_of_point(i, dims, K)
        by_pass[s].append((i, lev, k))
    work = x.copy()
    codes = {}
    outliers = {}
    for s in range(P):
        entries = by_pass[s]
        res = {}
        for (i, lev, k) in entries:
            if s == 0:
                pred = dt.type(0.0)
            else:
                h = 1 << (lev - 1)
                t = i[k]

                def val(off):
                    j = list(i)
                    j[k] = t + off * h
                    return work[tuple(j)]

                def has(off):
                    return 0 <= t + off * h < dims[k]

                pred = stencil_1d(interp, val(-1), val(1) if has(1) else 0.0,
                                  val(-3) if has(-3) else 0.0, val(3) if has(3) else 0.0,
                                  has(1), has(-3), has(3), dt)
            q, xh, out = quantize_scalar(x[i], pred, eb, dt)
            res[i] = (q, xh, out)
        for i, (q, xh, out) in res.items():
            work[i] = xh
        # chunk positions by sorting
        chunks = {}
        for (i, lev, k) in entries:
            if s == 0:
                cid = 0
            else:
                h = 1 << (lev - 1)
                ld = [(d - 1) // h + 1 for d in dims]
                tiles = [-(-ld[j] // C[j]) for j in range(D)]
                tix = [(i[j] // h) // C[j] for j in range(D)]
                cid = 0
                for j in range(D):
                    cid = cid * tiles[j] + tix[j]
            chunks.setdefault(cid, []).append(i)
        cmap = {}
        for cid, pts in chunks.items():
            for local, i in enumerate(sorted(pts)):
                cmap[(cid, local)] = i
        codes[s] = {key: res[i][0] for key, i in cmap.items()}
        outliers[s] = sorted((key, x[i]) for key, i in cmap.items() if res[i][2])
    return {"xhat": work, "codes": codes, "outliers": outliers, "K": K}


def negabinary_digits(q: int, n: int = 32):
    """Base -2 digits of q by repeated division (least significant first)."""
    digits = []
    v = q
    for _ in range(n):
        r = v % 2          # Python: 0 or 1
        digits.append(r)
        v = (v - r) // -2
    if v != 0:
        raise ValueError("value needs more digits")
    return digits


def planes_brute(codes_in_order, n_planes: int = 32):
    """Plane words of one chunk, one bit at a time."""
    n = len(codes_in_order)
    W = -(-n // 32)
    planes = [[0] * W for _ in range(n_planes)]
    for j, e in enumerate(codes_in_order):
        for k in range(n_planes):
            if (e >> k) & 1:
                planes[k][j // 32] |= 1 << (j % 32)
    return planes
