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
EMISSION = {"static": 0, "velinterp": 1, "cav": 2, "prefilter": 3}
AVG = {"log": 0, "linear": 1}
DTYPE = {"f32": 0, "bf16": 1, "f16": 2}
MODE = {"level0": 0, "vlm": 1}

EXPORTS = (
    "rt_scene_create", "rt_scene_build", "rt_trace", "rt_scene_get_info", "rt_scene_active_blocks",
    "rt_scene_levels", "rt_scene_states", "rt_scene_cell_values", "rt_debug_visited",
    "rt_scene_device_error", "rt_scene_reset_device_error", "rt_scene_destroy", "rt_last_error",
    "rt_version", "rt_batch_create", "rt_batch_run", "rt_batch_tiles", "rt_batch_device_error",
    "rt_batch_destroy", "rt_batch_autotune", "rt_graph_begin", "rt_graph_end", "rt_graph_launch",
    "rt_graph_destroy", "rt_trace_truncated", "rt_nrc_num_params", "rt_nrc_create", "rt_nrc_destroy",
    "rt_nrc_get_weights", "rt_nrc_set_weights", "rt_nrc_pack", "rt_nrc_train", "rt_nrc_loss", "rt_nrc_gradients",
    "rt_nrc_predict", "rt_nrc_compose", "rt_nrc_validate", "rt_scene_workspace_bytes", "rt_nrc_workspace_bytes",
    "rt_trace_j", "rt_trace_j_workspace_bytes", "rt_trace_j_noalloc", "rt_trace_interval", "rt_nrc_get_state", "rt_nrc_set_state",
    "rt_scene_count_active", "rt_batch_workspace_bytes", "rt_nrc_fallback_unverified",
)
_VOID = ("rt_scene_destroy", "rt_last_error", "rt_version", "rt_batch_destroy", "rt_graph_destroy", "rt_nrc_destroy")

_P = ctypes.c_void_p


class RtSceneDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("brick", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("model", ctypes.c_int32), ("emission", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("n_lines", ctypes.c_int32), ("n_v", ctypes.c_int32),
                ("dense", ctypes.c_int32), ("n_lam", ctypes.c_int32), ("vgrid", ctypes.c_int32),
                ("ds0", ctypes.c_double), ("h_lam", _P), ("h_lam0", _P)]


class RtSceneInputs(ctypes.Structure):
    _fields_ = [(k, _P) for k in ("d_eta", "d_chi", "d_eta_star", "d_chi_star", "d_damp", "d_inv_dld",
                                  "d_eta_bg", "d_chi_bg", "d_vel", "d_block_mask")]


class RtBuildParams(ctypes.Structure):
    _fields_ = [("iod_threshold", ctypes.c_double), ("tau_thin", ctypes.c_double), ("max_level", ctypes.c_int32),
                ("avg_mode", ctypes.c_int32), ("storage", ctypes.c_int32), ("iod_frame", ctypes.c_int32)]


class RtTraceParams(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_level", ctypes.c_int32), ("I0", ctypes.c_float),
                ("step_cap", ctypes.c_int32), ("d_stats", _P), ("level_dist", ctypes.c_float * 5),
                ("grade_mode", ctypes.c_int32)]


GRADE = {"entry": 0, "path": 1}


# Level m only beyond 1.5 x 4^m voxels: the paper's cascade caps [0,0,1,2,3,4]
# over radiance intervals ending at 1.5 x 4^i voxels (Sect. 4.1).
CASCADE_LEVEL_DIST = (0.0, 6.0, 24.0, 96.0, 384.0)


class RtSceneInfo(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("n_active", ctypes.c_int64), ("n_probes", ctypes.c_int64),
                ("cells_per_brick", ctypes.c_int64), ("storage_bytes", ctypes.c_int64),
                ("batch_begin", ctypes.c_int32), ("batch_end", ctypes.c_int32),
                ("n_state_words", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class RtDeviceErr(ctypes.Structure):
    _fields_ = [("step_cap_hits", ctypes.c_ulonglong), ("first_ray", ctypes.c_longlong),
                ("bad_probes", ctypes.c_ulonglong)]


class RtBatchJob(ctypes.Structure):
    _fields_ = [("scene", _P), ("d_dirs", _P), ("n_dir", ctypes.c_int32), ("reserved_", ctypes.c_int32),
                ("d_I", _P), ("params", RtTraceParams)]


class RtNrcDesc(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("freq_max", ctypes.c_float), ("seed", ctypes.c_uint64)]


class RtBatchParams(ctypes.Structure):
    _fields_ = [("wg_waves", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32), ("tiles_per_pop", ctypes.c_int32),
                ("order", ctypes.c_int32), ("d_claims", _P), ("tile_shape", ctypes.c_int32),
                ("reserved_", ctypes.c_int32)]


TILE_SHAPE = {"rows": 0, "cubes": 1}


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
    L.rt_scene_create.argtypes = [_P, _P, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]
    L.rt_scene_count_active.argtypes = [_P, _P, _P, ctypes.c_size_t, _P, ctypes.POINTER(ctypes.c_int64)]
    L.rt_scene_build.argtypes = [_P, _P, i32, i32, _P]
    L.rt_trace.argtypes = [_P, _P, _P, i32, _P, i64, _P, _P]
    L.rt_trace_interval.argtypes = [_P, _P, _P, i32, _P, i64, ctypes.c_double, ctypes.c_double, _P, _P, _P]
    L.rt_scene_get_info.argtypes = [_P, _P]
    L.rt_scene_active_blocks.argtypes = [_P, _P, _P]
    L.rt_scene_levels.argtypes = [_P, _P, _P]
    L.rt_scene_states.argtypes = [_P, _P, _P]
    L.rt_scene_cell_values.argtypes = [_P, i32, _P, _P, _P]
    L.rt_debug_visited.argtypes = [_P, _P, i32, _P, i32, _P, _P, _P, _P]
    L.rt_scene_device_error.argtypes = [_P, _P, _P]
    L.rt_scene_reset_device_error.argtypes = [_P, _P]
    L.rt_scene_destroy.argtypes = [_P]
    L.rt_scene_destroy.restype = None
    L.rt_batch_create.argtypes = [_P, i32, _P, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]
    L.rt_batch_workspace_bytes.argtypes = [i32, ctypes.POINTER(ctypes.c_size_t)]
    L.rt_batch_run.argtypes = [_P, _P]
    L.rt_batch_tiles.argtypes = [_P, _P]
    L.rt_batch_device_error.argtypes = [_P, _P, _P]
    L.rt_batch_destroy.argtypes = [_P]
    L.rt_batch_destroy.restype = None
    L.rt_batch_autotune.argtypes = [_P, i32, i32, _P, ctypes.c_size_t, _P, _P, _P]
    L.rt_graph_begin.argtypes = [_P]
    L.rt_graph_end.argtypes = [_P, ctypes.POINTER(_P)]
    L.rt_graph_launch.argtypes = [_P, _P]
    L.rt_graph_destroy.argtypes = [_P]
    L.rt_graph_destroy.restype = None
    L.rt_trace_truncated.argtypes = [_P, _P, ctypes.c_float, i32, _P, _P, i32, _P, i64, _P, _P, _P, _P, _P, _P]
    L.rt_scene_workspace_bytes.argtypes = [_P, i64, ctypes.POINTER(ctypes.c_size_t)]
    L.rt_trace_j.argtypes = [_P, _P, _P, _P, i32, _P, i64, _P, _P, _P, ctypes.c_size_t, _P]
    L.rt_trace_j_noalloc.argtypes = [_P, _P, _P, _P, i32, _P, i64, _P, _P, _P]
    L.rt_trace_j_workspace_bytes.argtypes = [_P, i32, i64, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.rt_nrc_workspace_bytes.argtypes = [_P, ctypes.POINTER(ctypes.c_size_t)]
    L.rt_nrc_num_params.argtypes = [_P]
    L.rt_nrc_create.argtypes = [_P, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]
    L.rt_nrc_destroy.argtypes = [_P]
    L.rt_nrc_destroy.restype = None
    L.rt_nrc_get_weights.argtypes = [_P, _P, _P]
    L.rt_nrc_set_weights.argtypes = [_P, _P, _P]
    L.rt_nrc_get_state.argtypes = [_P, _P, _P, _P, _P, _P]
    L.rt_nrc_set_state.argtypes = [_P, _P, _P, _P, i32, _P]
    L.rt_nrc_pack.argtypes = [_P, _P, i32, i64, _P, _P, _P, _P, _P, i64, _P]
    L.rt_nrc_train.argtypes = [_P, _P, _P, i64, i32, i32, ctypes.c_float, _P]
    L.rt_nrc_loss.argtypes = [_P, _P, _P]
    L.rt_nrc_gradients.argtypes = [_P, _P, _P, i64, _P, _P]
    L.rt_nrc_predict.argtypes = [_P, _P, i64, _P, _P]
    L.rt_nrc_compose.argtypes = [_P, _P, _P, i32, i64, _P, _P, _P, _P, _P, _P]
    L.rt_nrc_validate.argtypes = [_P, _P, _P, i32, i64, _P, _P, _P, _P, _P, ctypes.c_float, _P, _P, _P, _P, _P]
    L.rt_nrc_fallback_unverified.argtypes = [_P, _P, i32, _P, _P]
    L.rt_last_error.restype = ctypes.c_char_p
    L.rt_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in _VOID:
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


VGRID = {"full": 0, "orthant": 1}


def _scene_desc(dim, n, brick, n_levels, model, emission, profile, n_v, dense, ds0, n_lam_static, lam, lam0,
                vgrid="orthant"):
    """rt_scene_desc of a scene (plus the wavelength arrays it points to, which must stay alive)."""
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    d = RtSceneDesc()
    d.dim = int(dim)
    for a in range(3):
        d.n[a] = n[a]
    d.brick = int(brick)
    d.n_levels = int(n_levels)
    d.model = MODEL[model]
    d.emission = EMISSION[emission]
    d.profile = PROFILE[profile]
    d.n_v = int(n_v)
    d.vgrid = VGRID[vgrid]
    d.dense = 1 if dense else 0
    d.ds0 = float(ds0)
    if model == "static":
        d.n_lam = int(n_lam_static)
        return d, None, None
    lam = np.ascontiguousarray(lam, np.float64)
    lam0 = np.ascontiguousarray(lam0, np.float64)
    d.n_lam, d.n_lines = lam.size, lam0.size
    d.h_lam, d.h_lam0 = _np_ptr(lam), _np_ptr(lam0)
    return d, lam, lam0


def scene_workspace_bytes(sc, n_active=None, emission=None, n_v=21, dense=False, vgrid="orthant"):
    """Device bytes a scene made from the synthetic scene dict `sc` holds (host only; n_active
    defaults to the dict's active-block count, or every block when dense)."""
    model = sc["model"]
    emis = emission or "static"
    d, lam, lam0 = _scene_desc(sc["dim"], sc["n"], sc["brick"], sc["n_levels"], model, emis,
                               sc.get("profile", "gauss"), n_v, dense, sc.get("ds0", 1.0),
                               sc["eta"].shape[0] if model == "static" else None, sc.get("lam"), sc.get("lam0"),
                               vgrid)
    if n_active is None:
        n_active = sc["block_active"].size if dense else int(sc["block_active"].sum())
    v = ctypes.c_size_t(0)
    _check(lib().rt_scene_workspace_bytes(ctypes.byref(d), int(n_active), ctypes.byref(v)))
    return v.value


C_KMS = 299792.458  # speed of light, km/s


class VelocityGridWarning(UserWarning):
    """Velocity-interpolation node spacing coarser than the configured number of thermal widths."""


def velocity_grid_ratio(vel, inv_dld, lam0, n_v, vgrid="orthant"):
    """Per line, the largest ratio over voxels of the velocity-node spacing to the line's thermal (Doppler)
    width c / (lam0 inv_dld) (host arithmetic on the inputs, no device work).  The spacing of a voxel's grid is
    2 |v| / (n_v - 1) for the full grid, and the widest of its orthant ranges / (n_v - 1) for orthant grids."""
    def host(a):
        return a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)
    v = host(vel).astype(np.float64)
    if vgrid == "full":
        width = 2.0 * np.sqrt((v * v).sum(axis=0))
    else:
        width = np.zeros(v.shape[1:])
        for q in range(1 << v.shape[0]):
            b = np.stack([-v[a] if (q >> a) & 1 else v[a] for a in range(v.shape[0])])
            pos, neg = np.clip(b, 0, None), np.clip(b, None, 0)
            hi = np.where((b > 0).any(axis=0), np.sqrt((pos * pos).sum(axis=0)), b.max(axis=0))
            lo = np.where((b < 0).any(axis=0), -np.sqrt((neg * neg).sum(axis=0)), b.min(axis=0))
            width = np.maximum(width, hi - lo)
    spacing = width / max(int(n_v) - 1, 1)
    idl = host(inv_dld).astype(np.float32)
    out = []
    for k, l0 in enumerate(np.asarray(lam0, np.float64).reshape(-1)):
        vd = np.where(idl[k] > 0, C_KMS / (l0 * np.where(idl[k] > 0, idl[k], 1.0)), np.inf)
        out.append(float(np.max(spacing / vd)) if spacing.size else 0.0)
    return np.array(out)


class Scene:
    """A scene resident on the GPU: inputs (device tensors) + the library's handle.

    Inputs are given as numpy arrays or torch tensors with the layouts of
    include/rt.h (float32, x fastest); they are copied to the device once and
    kept alive with the handle.
    """

    def __init__(self, *, dim, n, brick, n_levels, model="static", emission="static", profile="gauss",
                 n_v=21, vgrid="orthant", dense=False, ds0=1.0, lam=None, lam0=None, n_lam=None, eta=None, chi=None,
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

        d, self.lam, self.lam0 = _scene_desc(self.dim, self.n, self.brick, n_levels, model, emission, profile, n_v,
                                             dense, ds0, None if eta is None else eta.shape[0], lam, lam0, vgrid)
        inp = RtSceneInputs()
        if model == "static":
            te, tc = dev(eta), dev(chi)
            self._keep.update(eta=te, chi=tc)
            inp.d_eta, inp.d_chi = te.data_ptr(), tc.data_ptr()
        else:
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
        self.velocity_grid_ratio = None
        if model != "static" and emission == "velinterp":
            self.velocity_grid_ratio = velocity_grid_ratio(vel, inv_dld, lam0, n_v, vgrid)
        # two-phase creation: count the active blocks, then lay the scene out in a workspace of the exact size
        # (the caller -- here this binding -- owns all device memory)
        v = ctypes.c_size_t(0)
        _check(lib().rt_scene_workspace_bytes(ctypes.byref(d), 0, ctypes.byref(v)))
        tmp = torch.empty(v.value, dtype=torch.uint8, device=self.device)
        na = ctypes.c_int64(0)
        _check(lib().rt_scene_count_active(ctypes.byref(d), ctypes.byref(inp), tmp.data_ptr(), v.value,
                                           _stream(stream), ctypes.byref(na)))
        del tmp
        _check(lib().rt_scene_workspace_bytes(ctypes.byref(d), na.value, ctypes.byref(v)))
        self._ws = torch.empty(v.value, dtype=torch.uint8, device=self.device)
        h = _P()
        _check(lib().rt_scene_create(ctypes.byref(d), ctypes.byref(inp), self._ws.data_ptr(), v.value,
                                     _stream(stream), ctypes.byref(h)))
        self.h = h
        self.info = self.get_info()

    @classmethod
    def from_dict(cls, sc, emission=None, **kw):
        """Scene from a synthetic scene dict (keys as produced by the synth package)."""
        args = dict(dim=sc["dim"], n=sc["n"], brick=sc["brick"], n_levels=sc["n_levels"], model=sc["model"],
                    ds0=sc.get("ds0", 1.0))
        if sc["model"] == "static":
            args.update(eta=sc["eta"], chi=sc["chi"], emission=emission or "static")
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

    def build(self, lam_begin, lam_end, iod_threshold=1e-2, tau_thin=0.25, max_level=-1, avg_mode="linear",
              storage="f32", iod_frame="rest", velocity_grid_warn=2.0, stream=None):
        """Builds the level structure for wavelengths [lam_begin, lam_end).  Velocity interpolation: warns
        (VelocityGridWarning) when the node spacing exceeds `velocity_grid_warn` thermal widths of the line whose
        rest wavelength is closest to the batch (Sect. 3.1)."""
        if self.velocity_grid_ratio is not None and velocity_grid_warn:
            mid = 0.5 * (self.lam[int(lam_begin)] + self.lam[int(lam_end) - 1])
            k = int(np.argmin(np.abs(np.asarray(self.lam0) - mid)))
            r = float(self.velocity_grid_ratio[k])
            if r > velocity_grid_warn:
                import warnings
                warnings.warn("velocity nodes are %.2f thermal widths of line %d apart (more than %g): raise n_v"
                              % (r, k, velocity_grid_warn), VelocityGridWarning, stacklevel=2)
        p = RtBuildParams()
        p.iod_frame = {"rest": 0, "core": 1}[iod_frame]
        p.iod_threshold = float(iod_threshold)
        p.tau_thin = float(tau_thin)
        p.max_level = int(max_level)
        p.avg_mode = AVG[avg_mode]
        p.storage = DTYPE[storage]
        _check(lib().rt_scene_build(self.h, ctypes.byref(p), int(lam_begin), int(lam_end), _stream(stream)))
        self.batch = (int(lam_begin), int(lam_end))

    def _tparams(self, mode, max_level, I0, step_cap, stats, level_dist=None, grade="entry"):
        p = RtTraceParams()
        p.grade_mode = GRADE[grade]
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
              level_dist=None, grade="entry", stream=None):
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
        p = self._tparams(mode, max_level, I0, step_cap, stats, level_dist, grade)
        _check(lib().rt_trace(self.h, ctypes.byref(p), td.data_ptr(), int(td.shape[0]),
                              tp.data_ptr() if tp is not None else None, int(n_probes), out.data_ptr(),
                              _stream(stream)))
        self._last = (td, tp)
        return out

    def trace_interval(self, dirs, t1, t2, probes=None, mode="vlm", I0=0.0, max_level=-1, step_cap=0,
                       level_dist=None, grade="entry", want_T=True, out=None, out_T=None, stats=None, stream=None):
        """Radiance interval [t1, t2] of every ray (rt_trace_interval): (I, T) [n_dir][batch][n_probes]
        (T is None when want_T is false)."""
        torch = self.torch
        td = dirs if isinstance(dirs, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(dirs, np.float32))
        td = td.to(device=self.device, dtype=torch.float32).contiguous()
        if probes is None:
            n_probes, tp = self.info["n_probes"], None
        else:
            tp = probes if isinstance(probes, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(probes, np.int32))
            tp = tp.to(device=self.device, dtype=torch.int32).contiguous()
            n_probes = tp.numel()
        nd, nl = int(td.shape[0]), self.batch[1] - self.batch[0]
        if out is None:
            out = torch.empty((nd, nl, n_probes), dtype=torch.float32, device=self.device)
        if want_T and out_T is None:
            out_T = torch.empty((nd, nl, n_probes), dtype=torch.float32, device=self.device)
        if not want_T:
            out_T = None
        p = self._tparams(mode, max_level, I0, step_cap, stats, level_dist, grade)
        _check(lib().rt_trace_interval(self.h, ctypes.byref(p), td.data_ptr(), nd,
                                       tp.data_ptr() if tp is not None else None, int(n_probes), float(t1),
                                       float(t2), out.data_ptr(), out_T.data_ptr() if out_T is not None else None,
                                       _stream(stream)))
        self._last = (td, tp)
        return out, out_T

    def trace_truncated(self, dirs, t_trunc, gen=True, fallback=None, probes=None, mode="vlm", I0=0.0,
                        max_level=-1, step_cap=0, level_dist=None, grade="entry", stream=None):
        """Truncated trace (rt_trace_truncated).  Returns a dict of device tensors:
        I_near, T_near, I_far (generation mode only) [n_dir][batch][n_probes],
        feat [n_dir][n_probes][4] (truncation point x, y, z, query flag) and
        fstat [n_dir][batch][n_probes][4] (level statistics there)."""
        torch = self.torch
        td = dirs if isinstance(dirs, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(dirs, np.float32))
        td = td.to(device=self.device, dtype=torch.float32).contiguous()
        if probes is None:
            n_probes, tp = self.info["n_probes"], None
        else:
            tp = probes if isinstance(probes, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(probes, np.int32))
            tp = tp.to(device=self.device, dtype=torch.int32).contiguous()
            n_probes = tp.numel()
        nd, nl = int(td.shape[0]), self.batch[1] - self.batch[0]
        f32 = dict(dtype=torch.float32, device=self.device)
        out = dict(I_near=torch.empty((nd, nl, n_probes), **f32), T_near=torch.empty((nd, nl, n_probes), **f32),
                   I_far=torch.empty((nd, nl, n_probes), **f32) if gen else None,
                   feat=torch.empty((nd, n_probes, 4), **f32), fstat=torch.empty((nd, nl, n_probes, 4), **f32))
        fb = None
        if fallback is not None:
            fb = fallback.to(device=self.device, dtype=torch.uint8).contiguous()
        p = self._tparams(mode, max_level, I0, step_cap, None, level_dist, grade)
        _check(lib().rt_trace_truncated(self.h, ctypes.byref(p), float(t_trunc), 1 if gen else 0,
                                        fb.data_ptr() if fb is not None else None, td.data_ptr(), nd,
                                        tp.data_ptr() if tp is not None else None, int(n_probes),
                                        out["I_near"].data_ptr(), out["T_near"].data_ptr(),
                                        out["I_far"].data_ptr() if gen else None, out["feat"].data_ptr(),
                                        out["fstat"].data_ptr(), _stream(stream)))
        out["dirs"], out["n_probes"], out["probes"] = td, n_probes, tp
        return out

    def trace_j(self, dirs, weights=None, probes=None, mode="vlm", I0=0.0, max_level=-1, step_cap=0,
                level_dist=None, grade="entry", with_psi=True, chunked=True, J=None, psi=None, stream=None):
        """Angle-integrated trace (rt_trace_j): J[batch][n_probes] = sum_d w_d I_d and, with_psi,
        psi = sum_d w_d (1 - exp(-tau of the first segment)).  weights default to 1/n_dir."""
        torch = self.torch
        td = dirs if isinstance(dirs, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(dirs, np.float32))
        td = td.to(device=self.device, dtype=torch.float32).contiguous()
        nd = int(td.shape[0])
        if weights is None:
            tw = torch.full((nd,), 1.0 / nd, dtype=torch.float32, device=self.device)
        else:
            tw = weights if isinstance(weights, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(weights, np.float32))
            tw = tw.to(device=self.device, dtype=torch.float32).contiguous()
        if probes is None:
            n_probes, tp = self.info["n_probes"], None
        else:
            tp = probes if isinstance(probes, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(probes, np.int32))
            tp = tp.to(device=self.device, dtype=torch.int32).contiguous()
            n_probes = tp.numel()
        nl = self.batch[1] - self.batch[0]
        if J is None:
            J = torch.empty((nl, n_probes), dtype=torch.float32, device=self.device)
        if with_psi and psi is None:
            psi = torch.empty((nl, n_probes), dtype=torch.float32, device=self.device)
        work, wb = None, 0
        if chunked:
            v = ctypes.c_size_t(0)
            _check(lib().rt_trace_j_workspace_bytes(self.h, nd, int(n_probes), 1 if with_psi else 0, ctypes.byref(v)))
            wb = v.value
            if wb:
                work = torch.empty(wb // 4, dtype=torch.float32, device=self.device)
        p = self._tparams(mode, max_level, I0, step_cap, None, level_dist, grade)
        _check(lib().rt_trace_j(self.h, ctypes.byref(p), td.data_ptr(), tw.data_ptr(), nd,
                                tp.data_ptr() if tp is not None else None, int(n_probes), J.data_ptr(),
                                psi.data_ptr() if with_psi else None, work.data_ptr() if work is not None else None,
                                int(wb), _stream(stream)))
        self._last_j = (td, tw, tp, work)
        return J, (psi if with_psi else None)

    def trace_j_noalloc(self, dirs, weights, J, psi=None, probes=None, mode="vlm", I0=0.0, max_level=-1,
                        step_cap=0, level_dist=None, grade="entry", stream=None):
        """rt_trace_j_noalloc: rt_trace_j with the library's own device scratch for the chunk partials.
        Every argument is a device tensor the caller already holds (dirs [n_dir][dim], weights [n_dir],
        probes int32 or None, J / psi [batch][n_probes]); nothing is allocated here or in the library."""
        nd = int(dirs.shape[0])
        n_probes = self.info["n_probes"] if probes is None else probes.numel()
        p = self._tparams(mode, max_level, I0, step_cap, None, level_dist, grade)
        _check(lib().rt_trace_j_noalloc(self.h, ctypes.byref(p), dirs.data_ptr(), weights.data_ptr(), nd,
                                        probes.data_ptr() if probes is not None else None, int(n_probes),
                                        J.data_ptr(), psi.data_ptr() if psi is not None else None, _stream(stream)))
        return J, psi

    def active_blocks(self, stream=None):
        out = np.zeros(self.info["n_active"], np.int32)
        _check(lib().rt_scene_active_blocks(self.h, _np_ptr(out), _stream(stream)))
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

    def levels(self, stream=None):
        out = np.zeros(self.info["n_blocks"], np.int8)
        _check(lib().rt_scene_levels(self.h, _np_ptr(out), _stream(stream)))
        return out

    def states(self, stream=None):
        out = np.zeros(self.info["n_state_words"], np.uint64)
        _check(lib().rt_scene_states(self.h, _np_ptr(out), _stream(stream)))
        return out

    def cell_values(self, cells, stream=None):
        c = np.ascontiguousarray(cells, np.int32).reshape(-1, 4)
        out = np.zeros((c.shape[0], LAM_BATCH, 2), np.float32)
        _check(lib().rt_scene_cell_values(self.h, c.shape[0], _np_ptr(c), _np_ptr(out), _stream(stream)))
        return out

    def visited(self, probe_vox, w, mode="vlm", max_level=-1, step_cap=0, cap=None, level_dist=None, grade="entry",
                stream=None):
        cap = cap or (sum(self.n) + 16)
        cells = np.zeros((cap, 4), np.int32)
        tt = np.zeros((cap, 2), np.float64)
        cnt = ctypes.c_int32(0)
        wd = np.zeros(3, np.float32)
        wd[: self.dim] = np.asarray(w, np.float32)[: self.dim]
        p = self._tparams(mode, max_level, 0.0, step_cap, None, level_dist, grade)
        _check(lib().rt_debug_visited(self.h, ctypes.byref(p), int(probe_vox), _np_ptr(wd), int(cap),
                                      _np_ptr(cells), _np_ptr(tt), ctypes.byref(cnt), _stream(stream)))
        k = cnt.value
        return cells[:k], tt[:k]

    def device_error(self, stream=None):
        e = RtDeviceErr()
        _check(lib().rt_scene_device_error(self.h, ctypes.byref(e), _stream(stream)))
        return int(e.step_cap_hits), int(e.first_ray)

    def bad_probes(self, stream=None):
        """Probe indices outside the grid met by traces since the last reset (their outputs are NaN)."""
        e = RtDeviceErr()
        _check(lib().rt_scene_device_error(self.h, ctypes.byref(e), _stream(stream)))
        return int(e.bad_probes)

    def reset_device_error(self, stream=None):
        _check(lib().rt_scene_reset_device_error(self.h, _stream(stream)))


def version():
    return lib().rt_version().decode()


# --------------------------------------------------------------------- batching
def _batch_jobs(jobs):
    """jobs: list of dicts {scene, dirs (device tensor), out (device tensor), trace kwargs...}."""
    arr = (RtBatchJob * len(jobs))()
    keep = []
    for i, j in enumerate(jobs):
        sc = j["scene"]
        d = j["dirs"].contiguous()
        o = j["out"]
        keep += [d, o]
        arr[i].scene = sc.h
        arr[i].d_dirs = d.data_ptr()
        arr[i].n_dir = int(d.shape[0])
        arr[i].d_I = o.data_ptr()
        arr[i].params = sc._tparams(j.get("mode", "vlm"), j.get("max_level", -1), j.get("I0", 0.0),
                                    j.get("step_cap", 0), None, j.get("level_dist"), j.get("grade", "entry"))
    return arr, keep


class Batch:
    """Many scenes traced in one persistent launch (rt_batch_*)."""

    def __init__(self, jobs, wg_waves=0, wgs_per_cu=0, tiles_per_pop=0, order=0, claims=None, tile_shape="rows",
                 stream=None):
        self._arr, self._keep = _batch_jobs(jobs)
        p = RtBatchParams()
        p.wg_waves, p.wgs_per_cu, p.tiles_per_pop, p.order = int(wg_waves), int(wgs_per_cu), int(tiles_per_pop), int(order)
        p.tile_shape = TILE_SHAPE[tile_shape] if isinstance(tile_shape, str) else int(tile_shape)
        p.d_claims = claims.data_ptr() if claims is not None else None
        self._claims = claims
        self._ws = _batch_workspace(len(jobs))
        h = _P()
        _check(lib().rt_batch_create(self._arr, len(jobs), ctypes.byref(p), self._ws.data_ptr(), self._ws.numel(),
                                     _stream(stream), ctypes.byref(h)))
        self.h = h

    def run(self, stream=None):
        _check(lib().rt_batch_run(self.h, _stream(stream)))

    def tiles(self):
        v = ctypes.c_int64(0)
        _check(lib().rt_batch_tiles(self.h, ctypes.byref(v)))
        return v.value

    def device_error(self, stream=None):
        e = RtDeviceErr()
        _check(lib().rt_batch_device_error(self.h, ctypes.byref(e), _stream(stream)))
        return int(e.step_cap_hits), int(e.first_ray)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.rt_batch_destroy(h)
            self.h = None


def _batch_workspace(n_jobs):
    import torch
    v = ctypes.c_size_t(0)
    _check(lib().rt_batch_workspace_bytes(int(n_jobs), ctypes.byref(v)))
    return torch.empty(v.value, dtype=torch.uint8, device="cuda")


def batch_autotune(jobs, reps=3, stream=None):
    """Fastest launch shape of the persistent kernel for these jobs: (params dict, ms per run)."""
    arr, keep = _batch_jobs(jobs)
    best = RtBatchParams()
    ms = ctypes.c_float(0)
    ws = _batch_workspace(len(jobs))
    _check(lib().rt_batch_autotune(arr, len(jobs), int(reps), ws.data_ptr(), ws.numel(), _stream(stream),
                                   ctypes.byref(best), ctypes.byref(ms)))
    del keep
    shape = {v: k for k, v in TILE_SHAPE.items()}[best.tile_shape]
    return {"wg_waves": best.wg_waves, "wgs_per_cu": best.wgs_per_cu, "tiles_per_pop": best.tiles_per_pop,
            "tile_shape": shape}, ms.value


class Graph:
    """Captures the work issued on a (non-default) stream and replays it (rt_graph_*)."""

    def __init__(self, stream):
        self.stream = stream
        self.h = None

    def __enter__(self):
        _check(lib().rt_graph_begin(_stream(self.stream)))
        return self

    def __exit__(self, exc_type, exc, tb):
        h = _P()
        st = lib().rt_graph_end(_stream(self.stream), ctypes.byref(h))
        if exc_type is None:
            _check(st)
            self.h = h
        return False

    def replay(self):
        _check(lib().rt_graph_launch(self.h, _stream(self.stream)))

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.rt_graph_destroy(h)
            self.h = None


# ------------------------------------------------------------ radiance cache
RAW = 12  # training row: pos 3, dir 3, wavelength offset, 4 level statistics, weight


def nrc_num_params():
    n = ctypes.c_int32(0)
    _check(lib().rt_nrc_num_params(ctypes.byref(n)))
    return n.value


class Nrc:
    """The neural radiance cache (rt_nrc_*): training rows are float32 [n][12]."""

    def __init__(self, max_batch=65536, freq_max=64.0, seed=0, stream=None):
        import torch
        self.torch = torch
        d = RtNrcDesc()
        d.max_batch, d.freq_max, d.seed = int(max_batch), float(freq_max), int(seed)
        self.desc = d
        v = ctypes.c_size_t(0)
        _check(lib().rt_nrc_workspace_bytes(ctypes.byref(d), ctypes.byref(v)))
        self._ws = torch.empty(v.value, dtype=torch.uint8, device="cuda")
        h = _P()
        _check(lib().rt_nrc_create(ctypes.byref(d), self._ws.data_ptr(), v.value, _stream(stream), ctypes.byref(h)))
        self.h = h
        self.n_params = nrc_num_params()

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.rt_nrc_destroy(h)
            self.h = None

    def get_weights(self, stream=None):
        w = np.zeros(self.n_params, np.float32)
        _check(lib().rt_nrc_get_weights(self.h, _np_ptr(w), _stream(stream)))
        return w

    def set_weights(self, w, stream=None):
        w = np.ascontiguousarray(w, np.float32)
        assert w.size == self.n_params
        _check(lib().rt_nrc_set_weights(self.h, _np_ptr(w), _stream(stream)))

    def get_state(self, stream=None):
        """Training state: dict of FP32 weights w, Adam moments m and v (host arrays) and the step count."""
        w, m, v = (np.zeros(self.n_params, np.float32) for _ in range(3))
        st = ctypes.c_int32(0)
        _check(lib().rt_nrc_get_state(self.h, _np_ptr(w), _np_ptr(m), _np_ptr(v), ctypes.byref(st), _stream(stream)))
        return {"w": w, "m": m, "v": v, "step": int(st.value)}

    def set_state(self, state, stream=None):
        w, m, v = (np.ascontiguousarray(state[k], np.float32) for k in ("w", "m", "v"))
        assert w.size == m.size == v.size == self.n_params
        _check(lib().rt_nrc_set_state(self.h, _np_ptr(w), _np_ptr(m), _np_ptr(v), int(state["step"]),
                                      _stream(stream)))

    def save_checkpoint(self, path):
        """Writes the training state to an .npz file (plain arrays, no pickled objects)."""
        st = self.get_state()
        np.savez(path, w=st["w"], m=st["m"], v=st["v"], step=np.array([st["step"]], np.int64))

    def load_checkpoint(self, path, stream=None):
        with np.load(path, allow_pickle=False) as z:
            self.set_state({"w": z["w"], "m": z["m"], "v": z["v"], "step": int(z["step"][0])}, stream)

    def _dev(self, a, dt=None):
        torch = self.torch
        t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
        return t.to(device="cuda", dtype=dt or torch.float32).contiguous()

    def train(self, raw, target, steps, batch, lr=1e-3, stream=None):
        r, t = self._dev(raw), self._dev(target)
        assert r.shape[-1] == RAW and t.numel() == r.shape[0]
        _check(lib().rt_nrc_train(self.h, r.data_ptr(), t.data_ptr(), int(r.shape[0]), int(steps), int(batch),
                                  float(lr), _stream(stream)))

    def loss(self, stream=None):
        v = ctypes.c_float(0)
        _check(lib().rt_nrc_loss(self.h, ctypes.byref(v), _stream(stream)))
        return v.value

    def gradients(self, raw, target, stream=None):
        r, t = self._dev(raw), self._dev(target)
        g = self.torch.zeros(self.n_params, dtype=self.torch.float32, device="cuda")
        _check(lib().rt_nrc_gradients(self.h, r.data_ptr(), t.data_ptr(), int(r.shape[0]), g.data_ptr(),
                                      _stream(stream)))
        return g

    def predict(self, raw, stream=None):
        r = self._dev(raw)
        y = self.torch.empty(r.shape[0], dtype=self.torch.float32, device="cuda")
        _check(lib().rt_nrc_predict(self.h, r.data_ptr(), int(r.shape[0]), y.data_ptr(), _stream(stream)))
        return y

    def pack(self, scene, tr, raw, target, row0, stream=None):
        """Training rows from a generation-mode truncated trace `tr` (Scene.trace_truncated output)."""
        _check(lib().rt_nrc_pack(scene.h, tr["dirs"].data_ptr(), int(tr["dirs"].shape[0]), int(tr["n_probes"]),
                                 tr["feat"].data_ptr(), tr["fstat"].data_ptr(), tr["I_far"].data_ptr(),
                                 raw.data_ptr(), target.data_ptr(), int(row0), _stream(stream)))

    def compose(self, scene, tr, out=None, stream=None):
        """I = I_near + T_near exp(10 y) over a truncated trace."""
        if out is None:
            out = self.torch.empty_like(tr["I_near"])
        _check(lib().rt_nrc_compose(self.h, scene.h, tr["dirs"].data_ptr(), int(tr["dirs"].shape[0]),
                                    int(tr["n_probes"]), tr["feat"].data_ptr(), tr["fstat"].data_ptr(),
                                    tr["I_near"].data_ptr(), tr["T_near"].data_ptr(), out.data_ptr(),
                                    _stream(stream)))
        return out

    def validate(self, scene, tr, thresh, fallback, count=None, stream=None):
        """Held-out check of a generation-mode trace: (prediction, relative error); flags
        fallback[block] for blocks whose queries exceed thresh and counts the checks per block
        (count: device int32/uint32 [n_blocks], optional)."""
        pred = self.torch.empty_like(tr["I_near"])
        err = self.torch.empty_like(tr["I_near"])
        _check(lib().rt_nrc_validate(self.h, scene.h, tr["dirs"].data_ptr(), int(tr["dirs"].shape[0]),
                                     int(tr["n_probes"]), tr["feat"].data_ptr(), tr["fstat"].data_ptr(),
                                     tr["I_near"].data_ptr(), tr["T_near"].data_ptr(), tr["I_far"].data_ptr(),
                                     float(thresh), pred.data_ptr(), fallback.data_ptr(),
                                     count.data_ptr() if count is not None else None, err.data_ptr(),
                                     _stream(stream)))
        return pred, err

    @staticmethod
    def fallback_unverified(scene, count, min_queries, fallback, stream=None):
        """Flags the blocks with fewer than min_queries held-out checks (rt_nrc_fallback_unverified)."""
        _check(lib().rt_nrc_fallback_unverified(scene.h, count.data_ptr(), int(min_queries), fallback.data_ptr(),
                                                _stream(stream)))


def nrc_workspace_bytes(max_batch=65536, freq_max=64.0, seed=0):
    """Device bytes a cache with this maximum batch holds (host only)."""
    d = RtNrcDesc()
    d.max_batch, d.freq_max, d.seed = int(max_batch), float(freq_max), int(seed)
    v = ctypes.c_size_t(0)
    _check(lib().rt_nrc_workspace_bytes(ctypes.byref(d), ctypes.byref(v)))
    return v.value
