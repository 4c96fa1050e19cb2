"""Brute-force ray marcher (test infrastructure only).

A third, deliberately naive formulation of the column ray of Sec. 2.1: walk the
normalised ray in fixed small steps (the approach the paper's DDA replaces) and
report the first sample that lands in a blocking tile.  With step h the hit
parameter is known to within h, and the hit tile is exact except where the ray
passes within about h of a tile corner.
"""
from __future__ import annotations

import numpy as np


def march(grid: np.ndarray, x: float, y: float, rx: float, ry: float, h: float = 1e-4,
          door: int = -1, door_open: int = 1, t_max: float | None = None):
    """Returns (hit tile id, t at the first blocking sample) for ray (rx, ry)
    from (x, y); t is in units of the (unnormalised) ray parameter."""
    N = grid.shape[0]
    norm = float(np.hypot(rx, ry))
    ux, uy = rx / norm, ry / norm
    if t_max is None:
        t_max = 2.0 * N
    s = np.arange(1, int(t_max / h) + 2, dtype=np.float64) * h
    px = x + s * ux
    py = y + s * uy
    tx = np.floor(px).astype(np.int64)
    ty = np.floor(py).astype(np.int64)
    inside = (tx >= 0) & (ty >= 0) & (tx < N) & (ty < N)
    blk = np.ones_like(inside)
    ids = np.where(inside, ty * N + tx, 0)
    flat = grid.reshape(-1)
    blk[inside] = flat[ids[inside]] != 0
    if door >= 0 and not door_open:
        blk |= inside & (ids == door)
    k = int(np.argmax(blk))
    if not blk[k]:
        return -1, float("inf")
    hit = int(ids[k]) if inside[k] else -1
    return hit, float(s[k] / norm)
