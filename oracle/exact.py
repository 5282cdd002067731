"""Exact-rational brute-force traversal for tiny grids (test infrastructure).

Independent of ``orc.c``: every crossing time of the ray x(t) = p - t w with
an integer plane is formed as an exact Fraction (the float32 direction is
taken at its exact binary value), the set is sorted, equal times collapse,
and each piece's voxel is floor(x(t_mid)) evaluated exactly.  The adapted
grid's cells follow by mapping each voxel to its block's level
(FloorToStep, Alg. 1), dropping empty blocks and merging repeats.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def ray_cells_exact(dim, n, pv, w):
    p = [Fraction(2 * int(pv[a]) + 1, 2) for a in range(dim)]
    wf = [Fraction(float(np.float32(w[a]))) for a in range(dim)]
    texit = None
    times = set()
    for a in range(dim):
        if wf[a] == 0:
            continue
        for k in range(0, int(n[a]) + 1):
            t = (p[a] - k) / wf[a]
            if t > 0:
                times.add(t)
        tb = p[a] / wf[a] if wf[a] > 0 else (p[a] - int(n[a])) / wf[a]
        texit = tb if texit is None else min(texit, tb)
    ts = sorted(t for t in times if t < texit)
    ts = [Fraction(0)] + ts + [texit]
    cells, tin, tout = [], [], []
    for t0, t1 in zip(ts[:-1], ts[1:]):
        if t1 <= t0:
            continue
        tm = (t0 + t1) / 2
        c = [math.floor(p[a] - tm * wf[a]) for a in range(dim)] + [0] * (3 - dim)
        cells.append(c)
        tin.append(t0)
        tout.append(t1)
    return cells, tin, tout


def adapted_cells_exact(dim, n, B, levels, pv, w, level_dist=None, grade="entry"):
    """Adapted-grid cells (coarse coords, level, t_in, t_out) from the exact dense list.

    level_dist: level m only where t >= level_dist[m] (exact compare), t being the path
    length at which the ray entered the block (grade "entry") or that of each point of
    the ray (grade "path": a voxel piece straddling level_dist[m] is split there)."""
    cells, tin, tout = ray_cells_exact(dim, n, pv, w)
    nb = [int(n[a]) // B for a in range(dim)] + [1] * (3 - dim)

    def cap_at(t):
        cap = 0
        for m in range(1, len(level_dist)):
            if not Fraction(level_dist[m]) <= t:
                break
            cap = m
        return cap

    out = []
    cur_blk, cur_cap = None, 127
    for c, a, b in zip(cells, tin, tout):
        blk = c[0] // B + nb[0] * (c[1] // B + nb[1] * (c[2] // B))
        if blk != cur_blk:
            cur_blk = blk
            if level_dist is not None:
                cur_cap = cap_at(a)
        Lb = int(levels[blk]) if levels is not None else 0
        if Lb < 0:
            continue
        pieces = [(a, b)]
        if level_dist is not None and grade == "path":
            cuts = sorted(set(Fraction(x) for x in level_dist[1:] if a < Fraction(x) < b))
            ends = [a] + cuts + [b]
            pieces = list(zip(ends[:-1], ends[1:]))
        for p0, p1 in pieces:
            cap = cap_at(p0) if (level_dist is not None and grade == "path") else cur_cap
            L = min(Lb, cap)
            cc = [x & ~((1 << L) - 1) for x in c]
            if out and out[-1][0] == cc and out[-1][1] == L:
                out[-1][3] = p1
                continue
            out.append([cc, L, p0, p1])
    return out
