"""Brick and probe orderings of the sparse grid (test infrastructure).

Sect. 2.3.1 stores the active blocks of the sparse grid in Morton (z-order)
order.  The functions here enumerate that order and the probe order of an
all-probes trace straight from the definition: interleave the bits of the
block coordinates (x lowest), sort, then list each active block's voxels
x fastest.  Pinned in tests/test_oracle_levels.py against a hand-written
z-order of a 4 x 4 block grid and its 3D analogue.
"""
from __future__ import annotations

import numpy as np


def _interleave(coord, dim, nbits):
    """Morton code of one block coordinate: bit b of axis a goes to bit b*dim + a."""
    code = 0
    for b in range(nbits):
        for a in range(dim):
            code |= ((int(coord[a]) >> b) & 1) << (b * dim + a)
    return code


def morton_order(nb_axes):
    """Linear block indices (x fastest) of every block of a block grid, in Morton order."""
    dim = len(nb_axes)
    nbits = max(1, int(max(nb_axes) - 1).bit_length())
    blocks = []
    total = int(np.prod(nb_axes))
    for lin in range(total):
        c, r = [], lin
        for a in range(dim):
            c.append(r % nb_axes[a])
            r //= nb_axes[a]
        blocks.append((_interleave(c, dim, nbits), lin))
    blocks.sort()
    return np.array([lin for _, lin in blocks], np.int64)


def probe_voxels(scene) -> np.ndarray:
    """Voxel linear indices of the probes of an all-probes trace: voxel centres of the active
    blocks, blocks in Morton order, voxels inside a block x fastest."""
    dim, n, B = scene["dim"], [int(v) for v in scene["n"]], int(scene["brick"])
    nb = [n[a] // B for a in range(dim)]
    act = np.asarray(scene["block_active"]).astype(bool)
    out = []
    for blk in morton_order(nb):
        if not act[blk]:
            continue
        bc, r = [], int(blk)
        for a in range(dim):
            bc.append(r % nb[a])
            r //= nb[a]
        # voxels of the block, x fastest then y then z
        kk, jj, ii = np.meshgrid(np.arange(B if dim == 3 else 1), np.arange(B), np.arange(B), indexing="ij")
        v = (bc[0] * B + ii) + n[0] * (bc[1] * B + jj)
        if dim == 3:
            v = v + n[0] * n[1] * (bc[2] * B + kk)
        out.append(v.reshape(-1))
    return np.concatenate(out).astype(np.int32) if out else np.zeros(0, np.int32)
