"""Fuzz of the oracle's adapted-grid traversal against the exact-rational brute force (CPU only, slow).

More than 10^5 rays over random block-level maps on small 2D and 3D grids, each
ray's (cell, level, t_in, t_out) list from the oracle's HDDA (Alg. 1 with exact
predicates) compared with the list the Fraction-based brute force builds from
every plane crossing (FloorToStep per block level, empty blocks dropped,
repeats merged).  Directions mix random unit vectors with tie-heavy families:
axis-aligned, equal components (45 degrees, exact corner crossings) and
components in exact power-of-two ratios, so tie-breaking at corners and on
block faces is exercised throughout.  Distance-graded caps are taken at block
entry and along the path.
"""
import math
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from oracle.exact import adapted_cells_exact

N_RAYS = 102_400
CASES = [  # (n, B, n_levels)
    ((16, 16), 4, 3),
    ((32, 32), 8, 4),
    ((24, 16), 8, 4),
    ((8, 8, 8), 4, 3),
    ((16, 8, 8), 8, 4),
]
SCHEDS = [None, (0, 2, 6, 12), (0, 0, 3, 3)]


def _tie_dirs(rng, dim, k):
    """Unit-ish FP32 directions whose components are equal or in exact power-of-two ratios."""
    out = []
    for _ in range(k):
        mag = rng.integers(0, 3, size=dim)  # component ratios 1, 2, 4
        if rng.random() < 0.3:
            mag[rng.integers(0, dim)] = -1  # one axis-parallel-to-plane component (w_a = 0)
        v = np.where(mag < 0, 0.0, 2.0 ** mag.clip(0))
        if not v.any():
            v[0] = 1.0
        f = np.float32(1.0 / np.linalg.norm(v))
        w = (v.astype(np.float32) * f).astype(np.float32)  # exact: power-of-two multiples of f
        w *= np.where(rng.random(dim) < 0.5, -1, 1).astype(np.float32)
        out.append(w)
    return out


def _rand_dirs(rng, dim, k):
    d = rng.normal(size=(k, dim))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return [x.astype(np.float32) for x in d]


def _chunk(args):
    """One worker: rays of one case and seed; returns (n_rays, first mismatch or None)."""
    ci, seed, n_rays = args
    import oracle as orc
    n, B, L = CASES[ci]
    dim = len(n)
    rng = np.random.default_rng(seed)
    nb = int(np.prod([v // B for v in n]))
    n3 = tuple(n) + (1,) * (3 - dim)
    z = np.zeros((1, int(np.prod(n))), np.float32)
    sc = dict(dim=dim, n=n3, brick=B, n_levels=L, model="static", eta=z, chi=z,
              dirs=np.zeros((1, dim), np.float32), block_active=np.ones(nb, np.uint8), ds0=1.0, I0=0.0)
    s = orc.Scene(sc)
    done = 0
    while done < n_rays:
        lv = rng.integers(-1, L, size=nb).astype(np.int8)
        sched = SCHEDS[int(rng.integers(0, len(SCHEDS)))]
        grade = "path" if rng.random() < 0.5 else "entry"
        if sched is not None:
            s.set_level_dist(sched[:L], mode=grade)
        else:
            s.set_level_dist(None)
        dirs = _rand_dirs(rng, dim, 8) + _tie_dirs(rng, dim, 8)
        for w in dirs:
            for _ in range(4):
                pv = tuple(int(rng.integers(0, n[a])) for a in range(dim))
                cells, lvl, ti, to = orc.ray_segments(s, lv, pv, w)
                ex = adapted_cells_exact(dim, n, B, lv, pv, w, level_dist=None if sched is None else sched[:L],
                                         grade=grade)
                bad = len(ex) != len(cells)
                if not bad:
                    for i, (cc, Lc, a, b) in enumerate(ex):
                        if list(cells[i][:3]) != list(cc) or lvl[i] != Lc or \
                                abs(ti[i] - float(a)) > 1e-13 * max(1.0, float(a)) or \
                                abs(to[i] - float(b)) > 1e-13 * max(1.0, float(b)):
                            bad = True
                            break
                if bad:
                    return done, dict(case=ci, seed=seed, pv=pv, w=[float(x) for x in w], lv=lv.tolist(),
                                      sched=sched, grade=grade)
                done += 1
    return done, None


@pytest.mark.slow
def test_hdda_fuzz_exact_rationals(orc):
    """>= 10^5 fuzzed rays: the oracle's HDDA lists equal the exact brute force."""
    per = 2048
    jobs = [(ci, 1000 * ci + j, per) for ci in range(len(CASES)) for j in range(N_RAYS // per // len(CASES))]
    workers = max(1, min(8, os.cpu_count() or 1))
    total = 0
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for done, bad in ex.map(_chunk, jobs):
            assert bad is None, bad
            total += done
    assert total >= 100_000
