"""Python binding of the MI355X formal-solution library (librt.so, include/rt.h).

Argument marshalling only: every step of the formal solution runs in the HIP
kernels of librt.so.  PyTorch supplies device memory and streams.  The
library must be built (``python paper_2511_08498_amd/build.py`` or
``__graft_entry__.build()``); importing works without it, but any call that
needs the library raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librt.so")

RT_OK, RT_E_ARG, RT_E_UNSUPPORTED, RT_E_STATE, RT_E_HIP, RT_E_DEVICE = range(6)
LAM_BATCH = 8
MAX_LINES = 4
MODEL = {"static": 0, "lines": 1}
PROFILE = {"gauss": 0, "voigt": 1}
EMISSION = {"static": 0, "velinterp": 1, "cav": 2}
AVG = {"log": 0, "linear": 1}
DTYPE = {"f32": 0, "bf16": 1, "f16": 2}
MODE = {"level0": 0, "vlm": 1}

EXPORTS = (
    "rt_scene_create", "rt_scene_build", "rt_trace", "rt_scene_get_info", "rt_scene_active_blocks",
    "rt_scene_levels", "rt_scene_states", "rt_scene_cell_values", "rt_debug_visited",
    "rt_scene_device_error", "rt_scene_reset_device_error", "rt_scene_destroy", "rt_last_error",
    "rt_version",
)

_P = ctypes.c_void_p


class RtSceneDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("brick", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("model", ctypes.c_int32), ("emission", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("n_lines", ctypes.c_int32), ("n_v", ctypes.c_int32),
                ("dense", ctypes.c_int32), ("n_lam", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("ds0", ctypes.c_double), ("h_lam", _P), ("h_lam0", _P)]


class RtSceneInputs(ctypes.Structure):
    _fields_ = [(k, _P) for k in ("d_eta", "d_chi", "d_eta_star", "d_chi_star", "d_damp", "d_inv_dld",
                                  "d_eta_bg", "d_chi_bg", "d_vel", "d_block_mask")]


class RtBuildParams(ctypes.Structure):
    _fields_ = [("iod_threshold", ctypes.c_double), ("tau_thin", ctypes.c_double), ("max_level", ctypes.c_int32),
                ("avg_mode", ctypes.c_int32), ("storage", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class RtTraceParams(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_level", ctypes.c_int32), ("I0", ctypes.c_float),
                ("step_cap", ctypes.c_int32), ("d_stats", _P), ("level_dist", ctypes.c_float * 5),
                ("reserved_", ctypes.c_int32)]


# Level m only beyond 1.5 x 4^m voxels: the paper's cascade caps [0,0,1,2,3,4]
# over radiance intervals ending at 1.5 x 4^i voxels (Sect. 4.1).
CASCADE_LEVEL_DIST = (0.0, 6.0, 24.0, 96.0, 384.0)


class RtSceneInfo(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("n_active", ctypes.c_int64), ("n_probes", ctypes.c_int64),
                ("cells_per_brick", ctypes.c_int64), ("storage_bytes", ctypes.c_int64),
                ("batch_begin", ctypes.c_int32), ("batch_end", ctypes.c_int32),
                ("n_state_words", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class RtDeviceErr(ctypes.Structure):
    _fields_ = [("step_cap_hits", ctypes.c_ulonglong), ("first_ray", ctypes.c_longlong)]


_LIB = None


class RtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("rt status %d: %s" % (status, msg))
        self.status = status


def lib():
    """Loads librt.so; raises if it has not been built (there is no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("librt.so is missing: build it with paper_2511_08498_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.rt_scene_create.argtypes = [_P, _P, _P, ctypes.POINTER(_P)]
    L.rt_scene_build.argtypes = [_P, _P, i32, i32, _P]
    L.rt_trace.argtypes = [_P, _P, _P, i32, _P, i64, _P, _P]
    L.rt_scene_get_info.argtypes = [_P, _P]
    L.rt_scene_active_blocks.argtypes = [_P, _P]
    L.rt_scene_levels.argtypes = [_P, _P]
    L.rt_scene_states.argtypes = [_P, _P]
    L.rt_scene_cell_values.argtypes = [_P, i32, _P, _P]
    L.rt_debug_visited.argtypes = [_P, _P, i32, _P, i32, _P, _P, _P, _P]
    L.rt_scene_device_error.argtypes = [_P, _P]
    L.rt_scene_reset_device_error.argtypes = [_P, _P]
    L.rt_scene_destroy.argtypes = [_P]
    L.rt_scene_destroy.restype = None
    L.rt_last_error.restype = ctypes.c_char_p
    L.rt_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("rt_scene_destroy", "rt_last_error", "rt_version"):
            getattr(L, name).restype = ctypes.c_int
    _LIB = L
    return L


def _check(st):
    if st != RT_OK:
        raise RtError(st, lib().rt_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(_P)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _P(s.cuda_stream)


class Scene:
    """A scene resident on the GPU: inputs (device tensors) + the library's handle.

    Inputs are given as numpy arrays or torch tensors with the layouts of
    include/rt.h (float32, x fastest); they are copied to the device once and
    kept alive with the handle.
    """

    def __init__(self, *, dim, n, brick, n_levels, model="static", emission="static", profile="gauss",
                 n_v=21, dense=False, ds0=1.0, lam=None, lam0=None, n_lam=None, eta=None, chi=None,
                 eta_star=None, chi_star=None, damp=None, inv_dld=None, eta_bg=None, chi_bg=None, vel=None,
                 block_mask=None, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.dim = int(dim)
        self.n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
        self.brick = int(brick)
        self.model = model
        self.emission = emission
        self._keep = {}

        def dev(a, dt=torch.float32):
            if a is None:
                return None
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            t = t.to(device=self.device, dtype=dt).contiguous()
            return t

        d = RtSceneDesc()
        d.dim = self.dim
        for a in range(3):
            d.n[a] = self.n[a]
        d.brick = self.brick
        d.n_levels = int(n_levels)
        d.model = MODEL[model]
        d.emission = EMISSION[emission]
        d.profile = PROFILE[profile]
        d.n_v = int(n_v)
        d.dense = 1 if dense else 0
        d.ds0 = float(ds0)
        inp = RtSceneInputs()
        if model == "static":
            te, tc = dev(eta), dev(chi)
            self._keep.update(eta=te, chi=tc)
            d.n_lam = int(te.shape[0])
            inp.d_eta, inp.d_chi = te.data_ptr(), tc.data_ptr()
            self.lam = None
        else:
            self.lam = np.ascontiguousarray(lam, np.float64)
            self.lam0 = np.ascontiguousarray(lam0, np.float64)
            d.n_lam = self.lam.size
            d.n_lines = self.lam0.size
            d.h_lam, d.h_lam0 = _np_ptr(self.lam), _np_ptr(self.lam0)
            for k, v in (("eta_star", eta_star), ("chi_star", chi_star), ("damp", damp), ("inv_dld", inv_dld),
                         ("eta_bg", eta_bg), ("chi_bg", chi_bg), ("vel", vel)):
                t = dev(v)
                self._keep[k] = t
                setattr(inp, "d_" + k, t.data_ptr())
        if block_mask is not None:
            tm = dev(block_mask, torch.uint8)
            self._keep["mask"] = tm
            inp.d_block_mask = tm.data_ptr()
        self.n_lam = d.n_lam
        self.desc = d
        h = _P()
        _check(lib().rt_scene_create(ctypes.byref(d), ctypes.byref(inp), _stream(stream), ctypes.byref(h)))
        self.h = h
        self.info = self.get_info()

    @classmethod
    def from_dict(cls, sc, emission=None, **kw):
        """Scene from a synthetic scene dict (keys as produced by the synth package)."""
        args = dict(dim=sc["dim"], n=sc["n"], brick=sc["brick"], n_levels=sc["n_levels"], model=sc["model"],
                    ds0=sc.get("ds0", 1.0))
        if sc["model"] == "static":
            args.update(eta=sc["eta"], chi=sc["chi"])
        else:
            args.update(emission=emission or "static", profile=sc.get("profile", "gauss"), lam=sc["lam"],
                        lam0=sc["lam0"], eta_star=sc["eta_star"], chi_star=sc["chi_star"], damp=sc["damp"],
                        inv_dld=sc["inv_dld"], eta_bg=sc["eta_bg"], chi_bg=sc["chi_bg"], vel=sc["vel"])
        args.update(kw)
        return cls(**args)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.rt_scene_destroy(h)
            self.h = None

    # ------------------------------------------------------------------ calls
    def get_info(self):
        inf = RtSceneInfo()
        _check(lib().rt_scene_get_info(self.h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in RtSceneInfo._fields_ if k != "reserved_"}

    def build(self, lam_begin, lam_end, iod_threshold=1e-2, tau_thin=0.25, max_level=-1, avg_mode="log",
              storage="f32", stream=None):
        p = RtBuildParams()
        p.iod_threshold = float(iod_threshold)
        p.tau_thin = float(tau_thin)
        p.max_level = int(max_level)
        p.avg_mode = AVG[avg_mode]
        p.storage = DTYPE[storage]
        _check(lib().rt_scene_build(self.h, ctypes.byref(p), int(lam_begin), int(lam_end), _stream(stream)))
        self.batch = (int(lam_begin), int(lam_end))

    def _tparams(self, mode, max_level, I0, step_cap, stats, level_dist=None):
        p = RtTraceParams()
        p.mode = MODE[mode]
        p.max_level = int(max_level)
        p.I0 = float(I0)
        p.step_cap = int(step_cap)
        p.d_stats = stats.data_ptr() if stats is not None else None
        if level_dist is not None:  # levels beyond the given schedule are never allowed
            for m in range(5):
                p.level_dist[m] = float(level_dist[m]) if m < len(level_dist) else 3.0e38
            p.level_dist[0] = 0.0
        return p

    def trace(self, dirs, probes=None, mode="vlm", I0=0.0, max_level=-1, step_cap=0, out=None, stats=None,
              level_dist=None, stream=None):
        """I[n_dir][batch wavelengths][n_probes] (float32, device)."""
        torch = self.torch
        td = dirs if isinstance(dirs, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(dirs, np.float32))
        td = td.to(device=self.device, dtype=torch.float32).contiguous()
        if probes is None:
            n_probes = self.info["n_probes"]
            tp = None
        else:
            tp = probes if isinstance(probes, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(probes, np.int32))
            tp = tp.to(device=self.device, dtype=torch.int32).contiguous()
            n_probes = tp.numel()
        nl = self.batch[1] - self.batch[0]
        if out is None:
            out = torch.empty((td.shape[0], nl, n_probes), dtype=torch.float32, device=self.device)
        p = self._tparams(mode, max_level, I0, step_cap, stats, level_dist)
        _check(lib().rt_trace(self.h, ctypes.byref(p), td.data_ptr(), int(td.shape[0]),
                              tp.data_ptr() if tp is not None else None, int(n_probes), out.data_ptr(),
                              _stream(stream)))
        self._last = (td, tp)
        return out

    def active_blocks(self):
        out = np.zeros(self.info["n_active"], np.int32)
        _check(lib().rt_scene_active_blocks(self.h, _np_ptr(out)))
        return out

    def probe_voxels(self):
        """Voxel linear index of every probe of the all-probes order."""
        B, dim, n = self.brick, self.dim, self.n
        nb = [n[a] // B for a in range(3)]
        ab = self.active_blocks().astype(np.int64)
        bx, by, bz = ab % nb[0], (ab // nb[0]) % nb[1], ab // (nb[0] * nb[1])
        loc = np.arange(B ** dim)
        lx, ly = loc % B, (loc // B) % B
        lz = loc // (B * B) if dim == 3 else np.zeros_like(loc)
        x = bx[:, None] * B + lx[None]
        y = by[:, None] * B + ly[None]
        z = bz[:, None] * B + lz[None]
        return (x + n[0] * (y + n[1] * z)).reshape(-1).astype(np.int32)

    def levels(self):
        out = np.zeros(self.info["n_blocks"], np.int8)
        _check(lib().rt_scene_levels(self.h, _np_ptr(out)))
        return out

    def states(self):
        out = np.zeros(self.info["n_state_words"], np.uint64)
        _check(lib().rt_scene_states(self.h, _np_ptr(out)))
        return out

    def cell_values(self, cells):
        c = np.ascontiguousarray(cells, np.int32).reshape(-1, 4)
        out = np.zeros((c.shape[0], LAM_BATCH, 2), np.float32)
        _check(lib().rt_scene_cell_values(self.h, c.shape[0], _np_ptr(c), _np_ptr(out)))
        return out

    def visited(self, probe_vox, w, mode="vlm", max_level=-1, step_cap=0, cap=None, level_dist=None, stream=None):
        cap = cap or (sum(self.n) + 16)
        cells = np.zeros((cap, 4), np.int32)
        tt = np.zeros((cap, 2), np.float64)
        cnt = ctypes.c_int32(0)
        wd = np.zeros(3, np.float32)
        wd[: self.dim] = np.asarray(w, np.float32)[: self.dim]
        p = self._tparams(mode, max_level, 0.0, step_cap, None, level_dist)
        _check(lib().rt_debug_visited(self.h, ctypes.byref(p), int(probe_vox), _np_ptr(wd), int(cap),
                                      _np_ptr(cells), _np_ptr(tt), ctypes.byref(cnt), _stream(stream)))
        k = cnt.value
        return cells[:k], tt[:k]

    def device_error(self):
        e = RtDeviceErr()
        _check(lib().rt_scene_device_error(self.h, ctypes.byref(e)))
        return int(e.step_cap_hits), int(e.first_ray)

    def reset_device_error(self, stream=None):
        _check(lib().rt_scene_reset_device_error(self.h, _stream(stream)))


def version():
    return lib().rt_version().decode()
