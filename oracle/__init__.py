"""FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and never imports it.  The arithmetic lives in ``orc.c`` (plain C, FP64, one
loop per definition in the paper); this module marshals numpy arrays into it
and adds the few steps that are plain numpy: the minimum of per-wavelength
levels over a wavelength batch, the 3-bit state packing and the error
percentiles.

Parity status per function (pins live in tests/test_oracle_*.py):
  ray_cells / ray_segments  pinned: exact-rational brute force, closed forms
  march (static)            pinned: homogeneous slab, pass-through, two-slab
                            order dependence, worked-example "Average" column
  levels                    pinned: constant field, linear ramp variance,
                            thin bypass, hand-built IoD cases
  voigt_h                   pinned: scipy.special.wofz, H(0,x), H(a,0)
  march (velinterp)         pinned: zero velocity reduces to the rest-frame
                            static march; second-order convergence in the node
                            spacing; at merged levels, rays whose projected
                            velocity falls on a node equal the box-filtered
                            Doppler-shifted static march (uniform velocity, and
                            cells mixing speeds, which fixes V = max |v|, the
                            mean velocity vbar, the node frame and the orthant
                            ranges of both grid modes)
  march (cav)               pinned: level 0 equals Classic; CaV wavelength scalings
  prefilter / march (PREFILTER)  pinned: homogeneous field is its own prefilter;
                            the worked example's voxel pair reproduces the
                            two-slab solution in each propagation order; axis
                            rays through a stratified merged block equal the
                            MIP-0 march (2D, 3D, both signs); all levels 0 =
                            static march bit for bit
  VLM approximation error   parity unpinned (no closed form; judged against
                            the dense march at the p99.9 bound)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STATIC, CLASSIC, VELINTERP, CAV, PREFILTER = 0, 1, 2, 3, 4
GAUSS, VOIGT = 0, 1
AVG_LOG, AVG_LINEAR = 0, 1
VGRID = {"full": 0, "orthant": 1}

_P = ctypes.c_void_p


class OrcScene(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("brick", ctypes.c_int32),
        ("n_levels", ctypes.c_int32), ("n_lam", ctypes.c_int32), ("profile", ctypes.c_int32),
        ("n_lines", ctypes.c_int32), ("n_v", ctypes.c_int32), ("avg_mode", ctypes.c_int32),
        ("grade_mode", ctypes.c_int32), ("ds0", ctypes.c_double), ("I0", ctypes.c_double),
        ("st_eta", _P), ("st_chi", _P), ("lam", _P), ("lam0", _P), ("eta_star", _P),
        ("chi_star", _P), ("damp", _P), ("inv_dld", _P), ("eta_bg", _P), ("chi_bg", _P),
        ("vel", _P), ("level_dist", _P), ("vgrid_mode", ctypes.c_int32), ("pf_eta", _P), ("pf_chi", _P),
    ]


def build():
    import subprocess
    subprocess.check_call(["sh", os.path.join(_HERE, "build.sh")])


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liborc.so")
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        L.orc_level_total.restype = ctypes.c_int64
        L.orc_level_total.argtypes = [ctypes.c_int32, _P, ctypes.c_int32]
        L.orc_ray_cells.restype = ctypes.c_int
        L.orc_ray_cells.argtypes = [ctypes.c_int32, _P, _P, _P, ctypes.c_int, _P, _P, _P]
        L.orc_ray_segments.restype = ctypes.c_int
        L.orc_ray_segments.argtypes = [_P, _P, _P, _P, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int]
        L.orc_voigt_h.restype = ctypes.c_double
        L.orc_voigt_h.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_voigt_h_vec.restype = None
        L.orc_voigt_h_vec.argtypes = [ctypes.c_int64, _P, _P, _P]
        L.orc_lines_mip0.restype = None
        L.orc_lines_mip0.argtypes = [_P, ctypes.c_int, ctypes.c_int, _P, _P]
        L.orc_levels.restype = ctypes.c_int64
        L.orc_levels.argtypes = [_P, _P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _P, _P, _P]
        L.orc_prefilter.restype = None
        L.orc_prefilter.argtypes = [_P, _P, _P, _P, _P]
        L.orc_march.restype = ctypes.c_int
        L.orc_march.argtypes = [_P, ctypes.c_int32, _P, _P, ctypes.c_int64, _P, _P, _P, ctypes.c_int32, _P]
        L.orc_march_interval.restype = ctypes.c_int
        L.orc_march_interval.argtypes = [_P, ctypes.c_int32, _P, _P, ctypes.c_int64, _P, _P, ctypes.c_double,
                                         ctypes.c_double, _P, _P, ctypes.c_int32]
        _LIB = L
    return _LIB


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


class Scene:
    """Keeps numpy inputs alive and exposes an OrcScene struct."""

    def __init__(self, sc: dict, lam_idx=None, n_v: int = 21, avg_mode: int = AVG_LINEAR, vgrid: str = "orthant"):
        self.sc = sc
        self.dim = sc["dim"]
        self.n = tuple(int(v) for v in sc["n"])
        self.nvox = int(np.prod(self.n))
        s = OrcScene()
        s.dim = self.dim
        for a in range(3):
            s.n[a] = self.n[a]
        s.brick = sc["brick"]
        s.n_levels = sc["n_levels"]
        s.ds0 = float(sc.get("ds0", 1.0))
        s.I0 = float(sc.get("I0", 0.0))
        s.n_v = int(n_v)
        s.avg_mode = int(avg_mode)
        s.vgrid_mode = VGRID[vgrid]
        self._keep = {}
        if sc["model"] == "lines":
            lam = np.asarray(sc["lam"], np.float64)
            if lam_idx is not None:
                lam = lam[np.asarray(lam_idx)]
            self.lam = np.ascontiguousarray(lam)
            s.n_lam = self.lam.size
            s.profile = VOIGT if sc.get("profile") == "voigt" else GAUSS
            s.n_lines = len(sc["lam0"])
            for k in ("eta_star", "chi_star", "damp", "inv_dld", "eta_bg", "chi_bg", "vel"):
                arr = _c(sc[k], np.float32)
                self._keep[k] = arr
                setattr(s, k, _ptr(arr))
            lam0 = _c(sc["lam0"], np.float64)
            self._keep["lam0"] = lam0
            self._keep["lam"] = self.lam
            s.lam = _ptr(self.lam)
            s.lam0 = _ptr(lam0)
        else:
            s.n_lam = 0
        self.s = s
        self.level_total = int(lib().orc_level_total(self.dim, _ptr(np.array(self.n, np.int32)), s.n_levels))

    def set_level_dist(self, level_dist, mode="entry"):
        """Distance-graded level cap: level m only where the path length is >= level_dist[m],
        taken at the ray's entry into each block (mode "entry") or at every point of the ray
        (mode "path"); None disables the grading."""
        self.s.grade_mode = {"entry": 0, "path": 1}[mode]
        if level_dist is None:
            self.s.level_dist = None
            return
        ld = np.full(8, np.inf)  # levels beyond the given schedule are never allowed
        ld[: len(level_dist)] = level_dist
        self._keep["level_dist"] = ld
        self.s.level_dist = _ptr(ld)

    def set_static_levels(self, st_eta, st_chi):
        """Level grids [n_lam][level_total] FP64 for the static march."""
        st_eta = _c(st_eta, np.float64)
        st_chi = _c(st_chi, np.float64)
        assert st_eta.shape == st_chi.shape and st_eta.shape[1] == self.level_total
        self._keep["st_eta"], self._keep["st_chi"] = st_eta, st_chi
        self.s.st_eta, self.s.st_chi = _ptr(st_eta), _ptr(st_chi)
        self.s.n_lam = st_eta.shape[0]

    def set_prefilter(self, pf_eta, pf_chi):
        """Prefiltered level cells [n_lam][level_total][2 dim] FP64 (levels >= 1 read by the PREFILTER march,
        which takes level 0 from set_static_levels)."""
        pf_eta = _c(pf_eta, np.float64)
        pf_chi = _c(pf_chi, np.float64)
        assert pf_eta.shape == pf_chi.shape and pf_eta.shape[1:] == (self.level_total, 2 * self.dim)
        self._keep["pf_eta"], self._keep["pf_chi"] = pf_eta, pf_chi
        self.s.pf_eta, self.s.pf_chi = _ptr(pf_eta), _ptr(pf_chi)

    @property
    def ref(self):
        return ctypes.byref(self.s)


# ----------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------
def ray_cells(dim, n, pv, w):
    """Dense MIP-0 cells (x, y, z), t_in, t_out of the ray from voxel pv upwind along -w."""
    n3 = np.array(list(n) + [1] * (3 - len(n)), np.int32)[:3]
    pv3 = np.array(list(pv) + [0] * (3 - len(pv)), np.int32)[:3]
    w3 = np.zeros(3, np.float32)
    w3[:dim] = np.asarray(w, np.float32)[:dim]
    cap = int(n3.sum()) + 8
    cell = np.zeros((cap, 3), np.int32)
    ti = np.zeros(cap)
    to = np.zeros(cap)
    k = lib().orc_ray_cells(dim, _ptr(n3), _ptr(pv3), _ptr(w3), cap, _ptr(cell), _ptr(ti), _ptr(to))
    assert k >= 0
    return cell[:k], ti[:k], to[:k]


def ray_segments(scene: Scene, levels, pv, w):
    """Adapted-grid cells (coarse coords), level, t_in, t_out."""
    dim = scene.dim
    pv3 = np.array(list(pv) + [0] * (3 - len(pv)), np.int32)[:3]
    w3 = np.zeros(3, np.float32)
    w3[:dim] = np.asarray(w, np.float32)[:dim]
    cap = int(sum(scene.n)) + 8
    cell = np.zeros((cap, 3), np.int32)
    lv = np.zeros(cap, np.int32)
    ti, to = np.zeros(cap), np.zeros(cap)
    sc_, sti, sto = np.zeros((cap, 3), np.int32), np.zeros(cap), np.zeros(cap)
    lev = None if levels is None else _c(levels, np.int8)
    k = lib().orc_ray_segments(scene.ref, _ptr(lev), _ptr(pv3), _ptr(w3), cap, _ptr(cell), _ptr(lv),
                               _ptr(ti), _ptr(to), _ptr(sc_), _ptr(sti), _ptr(sto), cap)
    assert k >= 0
    return cell[:k], lv[:k], ti[:k], to[:k]


# ----------------------------------------------------------------------
# mip chain / levels
# ----------------------------------------------------------------------
def levels_one(scene: Scene, eta0, chi0, block_active, T, tau_thin=0.25, cap=-1, want_values=False):
    """VLM level per block for one wavelength (MIP-0 eta0/chi0 FP64 [nvox])."""
    eta0 = _c(eta0, np.float64)
    chi0 = _c(chi0, np.float64)
    act = _c(block_active, np.uint8)
    lv = np.zeros(act.size, np.int8)
    oe = np.zeros(scene.level_total) if want_values else None
    oc = np.zeros(scene.level_total) if want_values else None
    clamped = lib().orc_levels(scene.ref, _ptr(eta0), _ptr(chi0), _ptr(act), float(T), float(tau_thin),
                               int(cap), _ptr(lv), _ptr(oe), _ptr(oc))
    if want_values:
        return lv, oe, oc, int(clamped)
    return lv


def batch_levels(per_lambda_levels):
    """Level of a wavelength batch: minimum over its wavelengths (empty stays -1)."""
    L = np.stack(per_lambda_levels).astype(np.int16)
    out = L.min(axis=0)
    return out.astype(np.int8)


def lines_mip0(scene: Scene, il: int, rule: int):
    """MIP-0 eta, chi of the line model at scene.lam[il]; rule 0 rest, 1 core-closest shift."""
    e = np.zeros(scene.nvox)
    c = np.zeros(scene.nvox)
    lib().orc_lines_mip0(scene.ref, int(il), int(rule), _ptr(e), _ptr(c))
    return e, c


def pack_states(levels) -> np.ndarray:
    """3 bits per block (state = level + 1, 0 = empty), 21 blocks per 64-bit word."""
    lv = np.asarray(levels, np.int64)
    nw = (lv.size + 20) // 21
    out = np.zeros(nw, np.uint64)
    for b in range(lv.size):
        st = int(lv[b]) + 1
        out[b // 21] |= np.uint64(st << (3 * (b % 21)))
    return out


# ----------------------------------------------------------------------
# march
# ----------------------------------------------------------------------
def march(scene: Scene, emis: int, levels, ray_vox, ray_dir, n_threads: int = 0, want_nseg=False):
    """I[ray][lam] in FP64 (upwind boundary -> probe recurrence)."""
    dirs = _c(scene.sc["dirs"], np.float32)
    rv = _c(ray_vox, np.int32)
    rd = _c(ray_dir, np.int32)
    nl = scene.s.n_lam
    out = np.zeros((rv.size, nl))
    nseg = np.zeros(rv.size, np.int32) if want_nseg else None
    lev = None if levels is None else _c(levels, np.int8)
    rc = lib().orc_march(scene.ref, int(emis), _ptr(lev), _ptr(dirs), rv.size, _ptr(rv), _ptr(rd),
                         _ptr(out), int(n_threads), _ptr(nseg))
    assert rc == 0, "oracle march: segment buffer overflow"
    return (out, nseg) if want_nseg else out


def march_interval(scene: Scene, emis: int, levels, ray_vox, ray_dir, t1, t2, n_threads: int = 0):
    """(I, T)[ray][lam] in FP64 over the path interval [t1, t2] of each ray (radiance interval):
    I starts from 0 at the far end unless the ray leaves the grid inside the interval (then from I0);
    T is the interval's transmittance."""
    dirs = _c(scene.sc["dirs"], np.float32)
    rv = _c(ray_vox, np.int32)
    rd = _c(ray_dir, np.int32)
    nl = scene.s.n_lam
    I = np.zeros((rv.size, nl))
    T = np.zeros((rv.size, nl))
    lev = None if levels is None else _c(levels, np.int8)
    rc = lib().orc_march_interval(scene.ref, int(emis), _ptr(lev), _ptr(dirs), rv.size, _ptr(rv), _ptr(rd),
                                  float(t1), float(t2), _ptr(I), _ptr(T), int(n_threads))
    assert rc != -2, "oracle interval march: need 0 <= t1 <= t2"
    assert rc == 0, "oracle interval march: segment buffer overflow"
    return I, T


def cap_levels(levels, max_level):
    """Block levels with a per-call MIP cap (empty blocks stay -1)."""
    lv = np.asarray(levels, np.int8).copy()
    if max_level >= 0:
        lv[lv > max_level] = max_level
    return lv


def voigt_h(a, x):
    a = np.ascontiguousarray(np.broadcast_to(a, np.broadcast(a, x).shape), np.float64).ravel()
    xx = np.ascontiguousarray(np.broadcast_to(x, np.broadcast(a, x).shape), np.float64).ravel()
    out = np.zeros(a.size)
    lib().orc_voigt_h_vec(a.size, _ptr(a), _ptr(xx), _ptr(out))
    return out


# ----------------------------------------------------------------------
# static scenes: level grids for every wavelength
# ----------------------------------------------------------------------
def static_level_values(scene: Scene, eta, chi, block_active, T, tau_thin=0.25, cap=-1):
    """Per-wavelength levels and FP64 level grids of a static [n_lam][nvox] scene."""
    nl = eta.shape[0]
    st_e = np.zeros((nl, scene.level_total))
    st_c = np.zeros((nl, scene.level_total))
    lvs = []
    for il in range(nl):
        lv, oe, oc, _ = levels_one(scene, eta[il].astype(np.float64), chi[il].astype(np.float64),
                                   block_active, T, tau_thin, cap, want_values=True)
        st_e[il], st_c[il] = oe, oc
        lvs.append(lv)
    return lvs, st_e, st_c


def prefilter_values(scene: Scene, eta, chi):
    """Prefiltered cells (Sect. 5.1) of every level for each wavelength of [n_lam][nvox] MIP-0 values:
    equivalent eta, chi per signed axis, [n_lam][level_total][2 dim]."""
    nl = eta.shape[0]
    K = 2 * scene.dim
    pe = np.zeros((nl, scene.level_total, K))
    pc = np.zeros((nl, scene.level_total, K))
    for il in range(nl):
        e = _c(eta[il], np.float64)
        c = _c(chi[il], np.float64)
        oe = np.zeros((scene.level_total, K))
        oc = np.zeros((scene.level_total, K))
        lib().orc_prefilter(scene.ref, _ptr(e), _ptr(c), _ptr(oe), _ptr(oc))
        pe[il], pc[il] = oe, oc
    return pe, pc


# ----------------------------------------------------------------------
# metrics
# ----------------------------------------------------------------------
PCTS = (100.0, 99.9, 99.0, 98.0, 95.0, 67.0, 50.0)


def rel_err_stats(I, I_ref):
    """Relative error percentiles; where I_ref == 0 the result must be exactly 0."""
    I = np.asarray(I, np.float64).ravel()
    R = np.asarray(I_ref, np.float64).ravel()
    zero = R == 0.0
    bad_zero = int(np.count_nonzero(I[zero] != 0.0))
    rel = np.abs(I[~zero] - R[~zero]) / np.abs(R[~zero])
    out = {"n": int(rel.size), "n_ref_zero": int(zero.sum()), "n_ref_zero_mismatch": bad_zero}
    if rel.size:
        for p in PCTS:
            out["p%g" % p] = float(np.percentile(rel, p, method="higher"))
    return out
