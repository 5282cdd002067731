#!/usr/bin/env python
"""Formal-solution benchmark on one MI355X.

Workload (default): 2D 1024^2 grid, 16^2 bricks (40 % active), two Gaussian
lines + continuum with a +-30 km/s velocity field handled by velocity
interpolation (one node grid per quadrant of directions), 4-level VLM mip
chain, 64 directions from every active voxel, 256 wavelengths in batches of
8.  The headline setting (CFG2_HEADLINE) is the fastest one measured whose
p99.9 relative intensity error against the FP64 dense Classic march is below
5e-3; the configuration's literal reading (IoD threshold 1e-2 with the thin
bypass) is reported beside it with its error.

One step = for every wavelength batch: build (MIP-0 values, mip chain,
VLM levels, velocity-node values, packed states) + trace (HDDA march of all
rays, distance-graded levels following the paper's cascade caps).  Inputs
are resident in HBM before timing; the output I[batch][dir][lam][probe]
(27.5 GB) is written for every batch.

Reported (one JSON line):
  value           dense-equivalent Gsegments/s of the timed VLM+HDDA path:
                  (MIP-0 cells, empty ones included, crossed by the same rays)
                  x wavelengths / step time;
  raw_gseg_s      segment updates actually applied per second;
  error           p99.9 (and the paper's percentile set) of the relative
                  intensity error against the FP64 dense Classic oracle on a
                  seeded ray sample, and whether it meets the 5e-3 bar;
  comparators     DenseClassic and SparseClassic (exact line profiles in every
                  MIP-0 cell of the full grid / of the active bricks),
                  velocity interpolation at MIP 0, the headline with FP16 /
                  BF16 node records, Core and Voigt with mips, the literal
                  setting, angle-integrated output: time per batch over every
                  fourth batch, speedup and error on the same sample;
  pareto          those settings ordered by time, with their errors;
  roofline        the march kernel's binding roof (VALU issue or DRAM bytes,
                  from the committed rocprofv3 counters of these sources) and
                  its compulsory HBM bytes per launch / mean launch time (HIP
                  events on the launch stream) vs 8 TB/s;
  cpu_baseline    the FP64 oracle timed on the host's cores on the ray sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "formal-solution Gsegments/s: dense vs VLM+HDDA vs NRC; p99.9 rel err vs FP64"
HBM_PEAK = 8.0e12  # B/s
CPU_SHARE = 16  # host cores allotted to one GPU's job
VALU_ISSUE_PEAK = 256 * 2.4e9  # wave64 VALU instructions per second: 256 CUs x 1 per clock (4 SIMD16, non-packed)
MARCH_SOURCES = ("march.hip", "common.h", "profile.h")
NRC_SOURCES = ("nrc.hip", "scene_impl.h", "common.h")


def march_source_hash(sources=MARCH_SOURCES):
    """SHA-256 over the sources the march kernels (or the given ones) are compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2511_08498_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters(name, setting=None, sources=MARCH_SOURCES):
    """Counter summary profiles/<name>.json if it was taken on the current sources of its kernel (and, when
    given, the same workload setting), else None."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        c = json.load(fh)
    if c.get("source_sha256", c.get("march_source_sha256")) != march_source_hash(sources):
        return None
    if setting is not None and c.get("setting") != setting:
        return None
    return c


def march_roofline(kernel, setting, compulsory_bytes, mean_launch_ms, streamed_bps, seglam_launch, counters_name):
    """Roofline of the march kernel of one launch.

    The binding roof comes from the committed rocprofv3 counter summary (taken on the same sources and
    setting): VALU wave-instructions issued per launch against 256 CUs x 1 per clock, and DRAM bytes per
    launch (FETCH_SIZE and WRITE_SIZE scaled by a copy kernel) against 8 TB/s; the larger fraction is the
    binding one.  The HBM side's algorithmic bytes are the compulsory ones: every stored value of the batch
    read once and the output written once.  The streamed-byte model (every segment reading its records from
    memory) is reported beside them: rays of a wave share cells through L1/L2, so it is not DRAM traffic."""
    t = mean_launch_ms / 1e3
    streamed = {"bytes_per_seg_lam": streamed_bps, "seg_lam_per_launch": seglam_launch,
                "gbs": streamed_bps * seglam_launch / t / 1e9}
    hbm = {"bound": "hbm", "achieved": compulsory_bytes / t / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
           "frac": compulsory_bytes / t / HBM_PEAK, "traffic": None, "algorithmic_bytes_per_launch": compulsory_bytes}
    cnt = measured_counters(counters_name, setting)
    roof = dict(hbm)
    if cnt is not None:
        hbm["traffic"] = cnt["hbm_bytes_per_launch"]
        hbm["traffic_gbs"] = cnt["hbm_bytes_per_launch"] / t / 1e9
        hbm["traffic_frac"] = cnt["hbm_bytes_per_launch"] / t / HBM_PEAK
        valu_rate = cnt["valu_insts_per_launch"] / t
        if valu_rate / VALU_ISSUE_PEAK >= hbm["traffic_frac"]:
            roof = {"bound": "alu", "achieved": valu_rate / 1e9, "peak": VALU_ISSUE_PEAK / 1e9,
                    "unit": "G VALU wave-instructions/s", "frac": valu_rate / VALU_ISSUE_PEAK,
                    "traffic": cnt["hbm_bytes_per_launch"],
                    "valu_insts_per_launch": cnt["valu_insts_per_launch"],
                    "lane_efficiency": cnt.get("valu_lane_efficiency")}
        else:
            roof = dict(hbm)
        roof["counters"] = "profiles/%s.json" % counters_name
    else:
        roof["note"] = "no counter summary on these sources: traffic and the VALU roof are not known"
    roof.update({"kernel": kernel, "mean_launch_ms": mean_launch_ms, "hbm": hbm, "streamed_model": streamed})
    return roof


def log(*a):
    print(*a, file=sys.stderr, flush=True)


STORAGE_T = {"f32": "float", "bf16": "__hip_bfloat16", "f16": "__half"}


def bytes_per_seg_lam(emission, storage, dim, lam_batch=8):
    s = 4 if storage == "f32" else 2
    if emission == "static":
        return 2 * s
    if emission == "velinterp":
        return 4 * s + (dim + 2) * 4.0 / lam_batch
    return 2 * 4.0 / lam_batch  # cav: parameters per segment shared by the batch (ALU bound)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg2",
                    choices=["cfg2", "cfg3", "cfg4", "cfg5", "matrix", "prefilter", "nrc_forward", "nrc_train"],
                    help="cfg2: 2D velocity interpolation (default, the headline line); cfg3: 3D Core and Voigt "
                         "per storage dtype; cfg4: 48-scene batched vs sequential; cfg5: radiance cache on cfg3; "
                         "matrix: the paper's method matrix on a prominence-like 2D scene; prefilter: box-filtered "
                         "vs prefiltered merged cells (Sect. 5.1) on cfg2's scene with the lines at rest; "
                         "nrc_forward: the cache network's fused forward kernel on 2^22 dense rows; nrc_train: its "
                         "training steps (forward, backward, Adam) at the cache's batch of 2^14 rows")
    ap.add_argument("--emission", default="velinterp", choices=["velinterp", "static", "cav"])
    ap.add_argument("--n-v", type=int, default=None, help="velocity nodes per orthant (default: cfg2 headline 41, "
                                                           "else 21)")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"],
                    help="cfg2: storage of the velocity-node / value records (FP32 accumulation in every case)")
    ap.add_argument("--iod", type=float, default=None, help="IoD threshold T (default: cfg2 headline 6e-4, matrix 1, "
                                                             "else 1e-2)")
    ap.add_argument("--avg", default="linear", choices=["log", "linear"], help="stored level values: arithmetic "
                    "(box filter, default) or geometric mean of the children")
    ap.add_argument("--tau-thin", type=float, default=None, help="thin bypass threshold on a cell's optical side "
                                                                  "(default: cfg2 headline 0, else 0.25)")
    ap.add_argument("--grade-scale", type=float, default=None, help="multiplies the cascade level distances "
                                                                     "(default: cfg2 headline 16, else 1)")
    ap.add_argument("--iod-frame", default=None, choices=["rest", "core"],
                    help="velocity interpolation: level test with lines at rest (the paper) or core-closest")
    ap.add_argument("--no-grading", action="store_true", help="plain VLM (no distance-graded cap)")
    ap.add_argument("--grade", default="path", choices=["entry", "path"],
                    help="distance-graded cap taken along the path (the cascade intervals' caps) or at each "
                         "block's entry")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--sample-seconds", type=float, default=15.0)
    ap.add_argument("--batches", type=int, default=0,
                    help="profiling only: trace the first N wavelength batches per step (0 = all)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="profiling only: first run a device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--ladder", action="store_true", help="cfg2: error of other settings on the sampled rays")
    ap.add_argument("--pairs", type=int, default=8192, help="cfg3/cfg5: oracle sample size (probe, direction pairs)")
    ap.add_argument("--dtypes", default="f32,bf16,f16", help="cfg3: storage dtypes to time")
    ap.add_argument("--nrc-steps", type=int, default=3000, help="cfg5: Adam steps")
    ap.add_argument("--nrc-freq", type=float, default=0.0, help="cfg5: highest encoding frequency (0: grid side / 2)")
    ap.add_argument("--nrc-lr", type=float, default=1e-3, help="cfg5: Adam learning rate")
    ap.add_argument("--nrc-train-probes", type=int, default=1024, help="cfg5: training probes per wavelength batch")
    ap.add_argument("--nrc-held-probes", type=int, default=1024, help="cfg5: held-out probes per wavelength batch "
                                                                         "(x 32 directions x 16 batches = 2^19 rays)")
    ap.add_argument("--nrc-min-checks", type=int, default=2, help="cfg5: held-out rays a block needs to use the cache")
    ap.add_argument("--scenes", type=int, default=0, help="cfg4: first N scenes only (0 = all 48)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU (--gpus %d requested): rays are independent given the scene, and the "
              "path would shard by wavelength batch with no exchange." % args.gpus)
        sys.exit(2)
    if args.workload != "cfg2":
        # cfg2 and cfg3 take their headline settings (CFG2_HEADLINE, CFG3_HEADLINE) for what is not given; the
        # method matrix mirrors the deployment of Sect. 4.1 (IoD threshold 1); elsewhere the configurations' own
        # reading
        dflt = {"iod": 1.0 if args.workload == "matrix" else 1e-2, "n_v": 21, "tau_thin": 0.25, "grade_scale": 1.0,
                "iod_frame": "rest"}
        if args.workload in ("cfg3", "cfg5"):  # cfg5 runs on cfg3's scene
            dflt.update(CFG3_HEADLINE)
        for k, v in dflt.items():
            if getattr(args, k) is None:
                setattr(args, k, v)
    if args.workload == "cfg3":
        return bench_cfg3(args)
    if args.workload == "cfg4":
        return bench_cfg4(args)
    if args.workload == "cfg5":
        return bench_cfg5(args)
    if args.workload == "matrix":
        return bench_matrix(args)
    if args.workload == "prefilter":
        return bench_prefilter(args)
    if args.workload == "nrc_forward":
        return bench_nrc_forward(args)
    if args.workload == "nrc_train":
        return bench_nrc_train(args)
    return bench_cfg2(args)


def copy_probe(args, torch, dev):
    """Profiling only: device-to-device copies of a known size, whose FETCH_SIZE / WRITE_SIZE counters scale the
    march kernels' counters to DRAM bytes."""
    if not args.copy_probe_mb:
        return
    src = torch.ones(args.copy_probe_mb * 2 ** 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy probe: %d MiB read + %d MiB written per copy, 3 copies" % (args.copy_probe_mb, args.copy_probe_mb))
    del src, dst


def host_cpu_info():
    """Host cores the oracle may use: this process's CPU affinity (nproc), capped at the CPU share one GPU's job
    is given on the GPU host; all host cores and the CPU model are recorded beside it."""
    import platform
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    # one GPU's job on the GPU host is allotted CPU_SHARE cores, whatever the affinity mask shows
    return {"nproc": usable, "host_cpus": os.cpu_count(), "cpu_model": model, "cpu_share": CPU_SHARE,
            "threads": min(usable, CPU_SHARE)}


# cfg2 settings.  The headline is the fastest measured setting whose p99.9 relative error against the FP64
# dense Classic march stays below 4e-3, a 20 % margin under the 5e-3 bar (differently sampled runs move a
# setting's p99.9 by up to about 5 %; the accuracy/speed sweep is in the design notes); "as stated" is the
# configuration's literal reading (IoD threshold 1e-2 with the thin bypass of Sect. 2.2, the rest-frame level
# test of Sect. 3.1, 21 nodes per quadrant as in Sect. 4.1), which is about ten times faster than the dense
# march and about fourteen times over the bar.
CFG2_HEADLINE = {"n_v": 41, "iod": 6e-4, "iod_frame": "core", "tau_thin": 0.0, "grade_scale": 16.0}
HEADLINE_MARGIN_BAR = 4e-3
CFG2_AS_STATED = {"n_v": 21, "iod": 1e-2, "iod_frame": "rest", "tau_thin": 0.25, "grade_scale": 1.0}
ACCURACY_BAR = 5e-3


def _cfg2_setting_text(st, emission="velinterp", storage="f32"):
    return ("%s (n_v=%d per orthant), %s storage, VLM T=%g, level test %s frame, thin bypass %g, cascade-graded "
            "levels x%g (cap taken along the path)" % (emission, st["n_v"], storage.upper(), st["iod"],
                                                       st["iod_frame"], st["tau_thin"], st["grade_scale"]))


def bench_cfg2(args):

    import numpy as np
    import torch

    import paper_2511_08498_amd as rt
    from synth import make_cfg2

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    hs = dict(CFG2_HEADLINE)
    for k, v in (("n_v", args.n_v), ("iod", args.iod), ("iod_frame", args.iod_frame), ("tau_thin", args.tau_thin),
                 ("grade_scale", args.grade_scale)):
        if v is not None:
            hs[k] = v
    t_gen = time.time()
    sc = make_cfg2()
    log("scene generated in %.1fs" % (time.time() - t_gen))
    n_lam = sc["lam"].size
    nb_lam = n_lam // 8
    if args.batches:
        nb_lam = min(nb_lam, args.batches)
        n_lam = 8 * nb_lam
    spread = list(range(2, nb_lam, 4)) or [0]  # comparator timing: every fourth batch across both lines
    copy_probe(args, torch, dev)
    dirs = torch.from_numpy(sc["dirs"]).to(dev)
    n_dir = dirs.shape[0]

    def lds(st):
        return None if args.no_grading else [v * st["grade_scale"] for v in rt.CASCADE_LEVEL_DIST]

    def bkw(st, storage="f32"):
        return dict(iod_threshold=st["iod"], avg_mode=args.avg, tau_thin=st["tau_thin"], iod_frame=st["iod_frame"],
                    storage=storage, velocity_grid_warn=0)

    level_dist = lds(hs)
    scene = rt.Scene.from_dict(sc, emission=args.emission, n_v=hs["n_v"])
    n_probes = scene.info["n_probes"]
    I_all = torch.empty((nb_lam, n_dir, 8, n_probes), dtype=torch.float32, device=dev)
    log("scene: %d active bricks, %d probes, output %.1f GB, headline: %s" % (
        scene.info["n_active"], n_probes, I_all.numel() * 4 / 1e9, _cfg2_setting_text(hs, args.emission, args.storage)))
    stream = torch.cuda.current_stream()
    ev = []

    def step(record=False, stats=None):
        for b in range(nb_lam):
            scene.build(8 * b, 8 * b + 8, **bkw(hs, args.storage))
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            scene.trace(dirs, mode="vlm", level_dist=level_dist, grade=args.grade, out=I_all[b], stats=stats)
            if record:
                e1.record(stream)
                ev.append((e0, e1))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(record=True)
        log("timed step done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / max(args.steps, 1)
    trace_ms = [a.elapsed_time(b) for a, b in ev]
    mean_trace_ms = float(np.mean(trace_ms))
    log("step %.1f ms; mean trace launch %.2f ms" % (ms_step, mean_trace_ms))

    # ---- segment counts (untimed pass with device counters)
    stats = torch.zeros(5, dtype=torch.int64, device=dev)
    step(stats=stats)
    torch.cuda.synchronize()
    segs_step = int(stats[0].item())
    lane_util = (int(stats[0].item()) + int(stats[2].item())) / max(64 * int(stats[4].item()), 1)
    seglam_step = segs_step * 8
    dense_scene = rt.Scene.from_dict(sc, emission="static", dense=True)
    probes_vox = torch.from_numpy(scene.probe_voxels()).to(dev)
    dense_scene.build(0, 8)
    dstats = torch.zeros(5, dtype=torch.int64, device=dev)
    tmp = torch.empty((n_dir, 8, n_probes), dtype=torch.float32, device=dev)
    dense_scene.trace(dirs, probes=probes_vox, mode="level0", out=tmp, stats=dstats)
    torch.cuda.synchronize()
    dense_cells = int(dstats[0].item())  # per wavelength
    dense_seglam_step = dense_cells * n_lam
    del dense_scene
    value = dense_seglam_step / (ms_step / 1e3) / 1e9
    raw = seglam_step / (ms_step / 1e3) / 1e9

    # ---- roofline of the march kernel
    bps = bytes_per_seg_lam(args.emission, args.storage, sc["dim"])
    seglam_launch = seglam_step / nb_lam
    # compulsory bytes of one launch: every stored node record of the batch (all direction classes and
    # levels) and the velocity-grid records read once, the output written once
    inf = scene.info
    s_b = 4 if args.storage == "f32" else 2
    n_cells = inf["n_active"] * inf["cells_per_brick"]
    compulsory = (2 ** sc["dim"] * n_cells * (hs["n_v"] * 8 * 2 * s_b + 16)) if args.emission == "velinterp" \
        else n_cells * 8 * 2 * s_b
    compulsory += n_dir * 8 * n_probes * 4
    kernel = ("k_trace<2, VisVelinterp<2, %s>>" % STORAGE_T[args.storage]) if args.emission == "velinterp" \
        else "k_trace"
    roofline = march_roofline(kernel, _cfg2_setting_text(hs, args.emission, args.storage), compulsory,
                              mean_trace_ms, bps, seglam_launch, "counters_%s_cfg2" % args.emission)

    out = {"metric": METRIC, "value": value, "unit": "Gsegments/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
           "config": {"workload": (
               "2D 1024^2, 16^2 bricks, 40%% active, 2 Gaussian lines + continuum, |v| <= 30 km/s, %s, 4-level mip "
               "chain, %s means, 64 dirs, 256 lambda (32 batches of 8), all %d probes" % (
                   _cfg2_setting_text(hs, args.emission, args.storage), args.avg, n_probes)),
                      "value_kind": "dense-equivalent segment-wavelength updates per second"},
           "accuracy_bar": ACCURACY_BAR,
           "raw_gseg_s": raw, "seg_lam_per_step": seglam_step, "dense_seg_lam_per_step": dense_seglam_step,
           "lane_utilisation": lane_util,
           "roofline": roofline}

    # ---- comparators, timed on every fourth batch (both lines, wings and cores)
    def time_setting(scn, build_kw, trace_kw, probes=None):
        scn.build(8 * spread[0], 8 * spread[0] + 8, **build_kw)
        scn.trace(dirs, probes=probes, out=tmp, **trace_kw)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for b in spread:
            scn.build(8 * b, 8 * b + 8, **build_kw)
            scn.trace(dirs, probes=probes, out=tmp, **trace_kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - ta) * 1e3 / len(spread)

    cmp = {}
    settings = {}  # name -> (scene, build kwargs, trace kwargs): error evaluated below on the sampled rays
    headline_ms_batch = ms_step / nb_lam
    if not args.no_compare:
        dc = rt.Scene.from_dict(sc, emission="cav", dense=True)
        cmp["dense_classic"] = {"ms_per_batch": time_setting(dc, {}, dict(mode="level0"), probes=probes_vox),
                                "note": "exact line profiles in every MIP-0 cell of the full grid (GPU)"}
        del dc
        dense_ms = cmp["dense_classic"]["ms_per_batch"]
        cav = rt.Scene.from_dict(sc, emission="cav")
        kw = (dict(velocity_grid_warn=0), dict(mode="level0"))
        cmp["sparse_classic"] = {"ms_per_batch": time_setting(cav, *kw),
                                 "note": "exact line profiles in every MIP-0 cell of the active bricks"}
        settings["sparse_classic"] = (cav,) + kw
        kw = (bkw(hs), dict(mode="level0"))
        cmp["sparse_velinterp"] = {"ms_per_batch": time_setting(scene, *kw),
                                   "note": "velocity interpolation at MIP 0 (no merging), same nodes"}
        settings["sparse_velinterp"] = (scene,) + kw
        for dt in ("f16", "bf16"):
            kw = (bkw(hs, dt), dict(mode="vlm", level_dist=level_dist, grade=args.grade))
            cmp["headline_%s_nodes" % dt] = {"ms_per_batch": time_setting(scene, *kw),
                                             "note": "the headline setting with %s velocity-node records "
                                                     "(32 B instead of 64 B per node)" % dt.upper()}
            settings["headline_%s_nodes" % dt] = (scene,) + kw
        kw = (bkw(hs), dict(mode="vlm", level_dist=level_dist, grade=args.grade))
        cmp["headline_spread_batches"] = {"ms_per_batch": time_setting(scene, *kw),
                                          "note": "the headline setting timed like the comparators"}
        # Core and Voigt with mips at the headline's level-test settings
        kw = (dict(iod_threshold=hs["iod"], avg_mode=args.avg, tau_thin=hs["tau_thin"]),
              dict(mode="vlm", level_dist=level_dist, grade=args.grade))
        cmp["cav_mips_headline_levels"] = {"ms_per_batch": time_setting(cav, *kw),
                                           "note": "Core and Voigt (Sect. 3.2) with the headline's level test"}
        settings["cav_mips_headline_levels"] = (cav,) + kw
        # the configuration as stated (T = 1e-2, thin bypass, rest frame, 21 nodes per quadrant)
        ss = CFG2_AS_STATED
        scene_st = rt.Scene.from_dict(sc, emission=args.emission, n_v=ss["n_v"])
        kw = (bkw(ss), dict(mode="vlm", level_dist=lds(ss), grade=args.grade))
        cmp["as_stated"] = {"ms_per_batch": time_setting(scene_st, *kw),
                            "setting": _cfg2_setting_text(ss, args.emission)}
        settings["as_stated"] = (scene_st,) + kw
        # angle-integrated output (mean intensity J + diagonal operator) instead of I per direction
        jbuf = torch.empty((8, n_probes), dtype=torch.float32, device=dev)
        pbuf = torch.empty_like(jbuf)
        scene.build(8 * spread[0], 8 * spread[0] + 8, **bkw(hs))
        scene.trace_j(dirs, mode="vlm", level_dist=level_dist, grade=args.grade, J=jbuf, psi=pbuf)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for b in spread:
            scene.build(8 * b, 8 * b + 8, **bkw(hs))
            scene.trace_j(dirs, mode="vlm", level_dist=level_dist, grade=args.grade, J=jbuf, psi=pbuf)
        torch.cuda.synchronize()
        jms = (time.perf_counter() - ta) * 1e3 / len(spread)
        cmp["vlm_j_output"] = {"ms_per_batch": jms,
                               "vs_i_output": cmp["headline_spread_batches"]["ms_per_batch"] / jms,
                               "note": "same march; J and psi [8][probes] instead of I [64 dirs][8][probes]"}
        for k2, v in cmp.items():
            if "ms_per_batch" in v:
                v["speedup_vs_dense_classic"] = dense_ms / v["ms_per_batch"]
        out["speedup_vs_dense_classic"] = dense_ms / headline_ms_batch
        log("comparators timed: " + ", ".join("%s %.1f ms" % (k2, v["ms_per_batch"]) for k2, v in cmp.items()))
        out["comparators"] = cmp

    # ---- accuracy and CPU baseline on a seeded ray sample
    if not args.no_cpu_baseline:
        import oracle as orc
        rng = np.random.default_rng(2025)
        probes = scene.probe_voxels()
        cpu = host_cpu_info()
        nthreads = cpu["threads"]

        def oracle_run(npairs, lam_idx):
            k = rng.choice(probes.size, npairs, replace=False)
            d = rng.integers(0, n_dir, npairs).astype(np.int32)
            s = orc.Scene(sc, lam_idx=lam_idx)
            ta = time.perf_counter()
            ref, nseg = orc.march(s, orc.CLASSIC, None, probes[k], d, n_threads=nthreads, want_nseg=True)
            return k, d, ref, int(nseg.sum()), time.perf_counter() - ta

        lam_all = list(range(n_lam))
        # calibrate on 512 pairs, then size the sample to about --sample-seconds of CPU time
        _, _, _, ns_cal, dt_cal = oracle_run(512, lam_all)
        rate = ns_cal * n_lam / max(dt_cal, 1e-3)
        npairs = int(min(probes.size, max(512, 512 * args.sample_seconds / max(dt_cal, 1e-3))))
        k, d, ref, nseg, dt = oracle_run(npairs, lam_all)
        cpu_rate = nseg * n_lam / dt
        out["cpu_baseline"] = {"value": cpu_rate / 1e9, "unit": "Gsegments/s", "cores": nthreads, "kind": "oracle",
                               "sample": "%d seeded (probe, direction) pairs x %d wavelengths, FP64 dense Classic "
                                         "march (exact line profiles), %.1f s" % (npairs, n_lam, dt),
                               "calibration_rate_gseg_s": rate / 1e9, **cpu}
        log("oracle: %d pairs in %.1f s on %d threads" % (npairs, dt, nthreads))
        dd = torch.from_numpy(d).long().to(dev)
        kk = torch.from_numpy(k).long().to(dev)
        got = I_all[:, dd, :, kk].reshape(len(k), n_lam).cpu().numpy()  # [pair][lam]
        err = orc.rel_err_stats(got, ref)
        out["error"] = {"vs": "FP64 dense Classic oracle", "n": err["n"],
                        **{k2: err[k2] for k2 in err if k2.startswith("p")}}
        out["meets_accuracy_bar"] = bool(err["p99.9"] <= ACCURACY_BAR)
        if settings:
            errs = run_ladder(torch, np, [(n, s_, b_, t_) for n, (s_, b_, t_) in settings.items()], {}, {},
                              dirs, probes[k], d, ref, nb_lam)
            for n, e in errs.items():
                out["comparators"][n]["error_vs_fp64_classic"] = e
            pareto = [{"name": "headline", "ms_per_batch": headline_ms_batch,
                       "speedup_vs_dense_classic": out.get("speedup_vs_dense_classic"), "p99.9": err["p99.9"]}]
            for n, v in out["comparators"].items():
                if "error_vs_fp64_classic" in v:
                    pareto.append({"name": n, "ms_per_batch": v["ms_per_batch"],
                                   "speedup_vs_dense_classic": v["speedup_vs_dense_classic"],
                                   "p99.9": v["error_vs_fp64_classic"]["p99.9"]})
            for p_ in pareto:
                p_["meets_bar"] = bool(p_["p99.9"] <= ACCURACY_BAR)
            out["pareto"] = sorted(pareto, key=lambda q: q["ms_per_batch"])
        if args.ladder:
            out["accuracy_ladder"] = accuracy_ladder(args, rt, torch, np, sc, scene, hs, dirs, probes[k], d, ref,
                                                     nb_lam, time_setting)
    print(json.dumps(out), flush=True)


def accuracy_ladder(args, rt, torch, np, sc, scene, hs, dirs, probe_vox, d, ref, nb_lam, time_setting):
    """cfg2: error against the FP64 oracle and time per batch of settings around the headline (the
    accuracy/speed sweep behind the headline's choice), on the same sampled rays."""
    def bk(st, **kw):
        b = dict(iod_threshold=st["iod"], avg_mode=args.avg, tau_thin=st["tau_thin"], iod_frame=st["iod_frame"],
                 storage=args.storage, velocity_grid_warn=0)
        b.update(kw)
        return b

    def tk(scale, **kw):
        t = dict(mode="vlm", level_dist=[v * scale for v in rt.CASCADE_LEVEL_DIST], grade=args.grade)
        t.update(kw)
        return t

    g = hs["grade_scale"]
    settings = [("as benchmarked", scene, bk(hs), tk(g)),
                ("sparse MIP 0 (no merging)", scene, bk(hs), tk(g, mode="level0")),
                ("grading x%g" % (g / 2), scene, bk(hs), tk(g / 2)),
                ("grading x%g" % (g / 4), scene, bk(hs), tk(g / 4)),
                ("T / 2", scene, bk(hs, iod_threshold=hs["iod"] / 2), tk(g)),
                ("T / 4", scene, bk(hs, iod_threshold=hs["iod"] / 4), tk(g)),
                ("T x1.5", scene, bk(hs, iod_threshold=1.5 * hs["iod"]), tk(g)),
                ("T x1.5, grading x%g" % (g * 0.75), scene, bk(hs, iod_threshold=1.5 * hs["iod"]), tk(g * 0.75)),
                ("T x2", scene, bk(hs, iod_threshold=2 * hs["iod"]), tk(g)),
                ("T / 2, grading x%g" % (g / 2), scene, bk(hs, iod_threshold=hs["iod"] / 2), tk(g / 2)),
                ("T = 1e-2", scene, bk(hs, iod_threshold=1e-2), tk(g)),
                ("rest-frame level test", scene, bk(hs, iod_frame="rest"), tk(g)),
                ("thin bypass 0.25", scene, bk(hs, tau_thin=0.25), tk(g)),
                ("levels <= 1", scene, bk(hs), tk(g, max_level=1)),
                ("plain VLM (no distance grading)", scene, bk(hs), tk(g, level_dist=None)),
                ("FP16 node records", scene, bk(hs, storage="f16"), tk(g)),
                ("FP16 node records, T x1.5", scene, bk(hs, storage="f16", iod_threshold=1.5 * hs["iod"]), tk(g))]
    res = run_ladder(torch, np, settings, {}, {}, dirs, probe_vox, d, ref, nb_lam)
    for name, scn, b, t in settings:
        res[name]["ms_per_batch"] = time_setting(scn, b, t)
    scene_paper = rt.Scene.from_dict(sc, emission=args.emission, n_v=21)
    more = [("21 nodes per orthant, sparse MIP 0", scene_paper, bk(hs), tk(g, mode="level0")),
            ("21 nodes per orthant", scene_paper, bk(hs), tk(g))]
    res.update(run_ladder(torch, np, more, {}, {}, dirs, probe_vox, d, ref, nb_lam))
    for name, scn, b, t in more:
        res[name]["ms_per_batch"] = time_setting(scn, b, t)
    del scene_paper
    scene61 = rt.Scene.from_dict(sc, emission=args.emission, n_v=61)
    more = [("61 nodes per orthant, sparse MIP 0", scene61, bk(hs), tk(g, mode="level0")),
            ("61 nodes per orthant", scene61, bk(hs), tk(g)),
            ("61 nodes per orthant, T x1.5", scene61, bk(hs, iod_threshold=1.5 * hs["iod"]), tk(g))]
    res.update(run_ladder(torch, np, more, {}, {}, dirs, probe_vox, d, ref, nb_lam))
    for name, scn, b, t in more:
        res[name]["ms_per_batch"] = time_setting(scn, b, t)
    for v in res.values():
        v["meets_bar"] = bool(v["p99.9"] <= ACCURACY_BAR)
    return res


def run_ladder(torch, np, settings, base_build, base_trace, dirs, probe_vox, d, ref, nb_lam):
    """Each setting is traced only from the sampled probes (all directions); the sampled direction is picked."""
    dev = dirs.device
    pk = torch.from_numpy(np.ascontiguousarray(probe_vox)).to(dev)
    dd = torch.from_numpy(d).long().to(dev)
    ar = torch.arange(len(d), device=dev)
    res = {}
    for name, scn, bkw, tkw in settings:
        got = np.zeros((len(d), nb_lam * 8))
        for b in range(nb_lam):
            scn.build(8 * b, 8 * b + 8, **dict(base_build, **bkw))
            I = scn.trace(dirs, probes=pk, **dict(base_trace, **tkw))
            got[:, 8 * b:8 * b + 8] = I[dd, :, ar].cpu().numpy()
        res[name] = {k2: v for k2, v in _err(got, ref).items() if k2 in ("p100", "p99.9", "p99", "p50")}
        log("ladder %-40s p99.9 %.3e" % (name, res[name]["p99.9"]))
    return res


# ----------------------------------------------------------------------------- shared helpers
def _env():
    import numpy as np
    import torch

    import paper_2511_08498_amd as rt
    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    return np, torch, rt, dev


def _oracle_classic(sc, probe_vox, k, d, lam_idx, n_threads):
    """FP64 dense Classic march (the oracle) on (probe, direction) pairs: ref [pair][lam], seg-lam, seconds."""
    import oracle as orc
    s = orc.Scene(sc, lam_idx=lam_idx)
    ta = time.perf_counter()
    ref, nseg = orc.march(s, orc.CLASSIC, None, probe_vox[k], d, n_threads=n_threads, want_nseg=True)
    return ref, int(nseg.sum()) * len(lam_idx), time.perf_counter() - ta


def _grading(args):
    """workload text for the level cap along the ray"""
    if args.no_grading:
        return "plain VLM"
    scale = "" if args.grade_scale == 1.0 else " x%g" % args.grade_scale
    return "cascade-graded levels (cap taken %s)%s" % (
        "along the path" if args.grade == "path" else "at block entry", scale)


def _err(got, ref):
    import oracle as orc
    e = orc.rel_err_stats(got, ref)
    return {k2: e[k2] for k2 in e if k2.startswith("p") or k2 in ("n", "n_ref_zero_mismatch")}


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


# ----------------------------------------------------------------------------- cfg3
# The cfg3 headline is, like cfg2's, the fastest setting measured under the 5e-3 bar; on this scene (a dense
# chromosphere slab with steep vertical gradients, filaments in near-empty fill) the bar leaves almost no cell
# merged, so the headline runs at the speed of the exact sparse march.  The configuration's literal reading
# (T = 1e-2 with the thin bypass) is reported beside it.
CFG3_HEADLINE = {"iod": 3e-4, "tau_thin": 0.0, "grade_scale": 16.0}
CFG3_AS_STATED = {"iod": 1e-2, "tau_thin": 0.25, "grade_scale": 1.0}


def bench_cfg3(args):
    """3D 256^3 Core-and-Voigt scene at the headline setting, storage FP32 / BF16 / FP16: time per full solve
    (16 batches), march-kernel roofline, error of each dtype against the FP64 dense Classic oracle; the literal
    setting and the exact sparse march beside it (pareto)."""
    np, torch, rt, dev = _env()
    from synth import make_cfg3
    tg = time.time()
    sc = make_cfg3()
    log("cfg3 scene generated in %.1fs (%d active bricks)" % (time.time() - tg, int(sc["block_active"].sum())))
    copy_probe(args, torch, dev)
    nb = sc["lam"].size // 8
    if args.batches:
        nb = min(nb, args.batches)
    dirs = torch.from_numpy(sc["dirs"]).to(dev)
    n_dir = dirs.shape[0]
    level_dist = None if args.no_grading else [v * args.grade_scale for v in rt.CASCADE_LEVEL_DIST]
    scene = rt.Scene.from_dict(sc, emission="cav")
    n_probes = scene.info["n_probes"]
    probe_vox = scene.probe_voxels()
    out = torch.empty((n_dir, 8, n_probes), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(2026)
    k = rng.choice(n_probes, min(args.pairs, n_probes), replace=False)
    d = rng.integers(0, n_dir, k.size).astype(np.int32)
    kk, dd = torch.from_numpy(k).long().to(dev), torch.from_numpy(d).long().to(dev)
    stream = torch.cuda.current_stream()
    res = {}
    for dt in args.dtypes.split(","):
        got = torch.empty((k.size, nb * 8), dtype=torch.float32, device=dev)
        evs = []

        def solve(record=False, gather=False):
            for b in range(nb):
                scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin, storage=dt)
                if record:
                    e0, e1 = _events(torch)
                    e0.record(stream)
                scene.trace(dirs, mode="vlm", level_dist=level_dist, grade=args.grade, out=out)
                if record:
                    e1.record(stream)
                    evs.append((e0, e1))
                if gather:
                    got[:, 8 * b:8 * b + 8] = out[dd, :, kk]

        for _ in range(args.warmup):
            solve()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(args.steps):
            solve(record=True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - ta) * 1e3 / max(args.steps, 1)
        solve(gather=True)
        torch.cuda.synchronize()
        res[dt] = {"ms_per_solve": ms, "mean_trace_ms": float(np.mean([a.elapsed_time(b) for a, b in evs])),
                   "got": got.cpu().numpy()}
        log("cfg3 %s: %.1f ms per solve, trace %.2f ms" % (dt, ms, res[dt]["mean_trace_ms"]))
    # segment counts: levels come from the FP64 chain of the MIP-0 values, not from the storage dtype
    stats = torch.zeros(5, dtype=torch.int64, device=dev)
    for b in range(nb):
        scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin)
        scene.trace(dirs, mode="vlm", level_dist=level_dist, grade=args.grade, out=out, stats=stats)
    torch.cuda.synchronize()
    seglam = int(stats[0].item()) * 8
    if args.no_compare and args.no_cpu_baseline:  # profiling runs: the timed solves only
        log("cfg3: %d seg-lambda per solve" % seglam)
        return
    # dense comparator: Core and Voigt at MIP 0 on the full grid (every brick stored), one batch
    dense = rt.Scene.from_dict(sc, emission="cav", dense=True)
    pv = torch.from_numpy(probe_vox).to(dev)
    dstats = torch.zeros(5, dtype=torch.int64, device=dev)
    dense.build(0, 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin)
    dense.trace(dirs, probes=pv, mode="level0", out=out)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    dense.build(0, 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin)
    dense.trace(dirs, probes=pv, mode="level0", out=out, stats=dstats)
    torch.cuda.synchronize()
    dense_ms_batch = (time.perf_counter() - ta) * 1e3
    dense_cells = int(dstats[0].item())
    del dense
    torch.cuda.empty_cache()
    cpu = host_cpu_info()
    nthreads = cpu["threads"]
    ref, cpu_seglam, cpu_s = _oracle_classic(sc, probe_vox, k, d, list(range(nb * 8)), nthreads)
    log("cfg3 oracle: %d pairs x %d lambda in %.1fs" % (k.size, nb * 8, cpu_s))
    dense_seglam = dense_cells * 8 * nb
    ladder = None
    if args.ladder:
        base = dict(iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin)
        settings = [("as benchmarked (f32)", scene, {}, {}),
                    ("sparse MIP 0 (no merging)", scene, {}, {"mode": "level0"}),
                    ("levels <= 1", scene, {}, {"max_level": 1}),
                    ("levels <= 2", scene, {}, {"max_level": 2}),
                    ("plain VLM (no distance grading)", scene, {}, {"level_dist": None}),
                    ("no thin bypass", scene, {"tau_thin": 0.0}, {}),
                    ("no thin bypass, log means", scene, {"tau_thin": 0.0, "avg_mode": "log"}, {}),
                    ("log means", scene, {"avg_mode": "log"}, {}),
                    ("no thin bypass, T=1e-3", scene, {"tau_thin": 0.0, "iod_threshold": 1e-3}, {}),
                    ("no thin bypass, levels <= 2", scene, {"tau_thin": 0.0}, {"max_level": 2})]
        ladder = run_ladder(torch, np, settings, base, dict(mode="vlm", level_dist=level_dist, grade=args.grade),
                            dirs, probe_vox[k], d,
                            ref, nb)
    # pareto: the literal setting and the exact sparse march (Core and Voigt at MIP 0), timed on every fourth batch
    spread = list(range(1, nb, 4)) or [0]

    def time_setting(bkw, tkw):
        scene.build(8 * spread[0], 8 * spread[0] + 8, **bkw)
        scene.trace(dirs, out=out, **tkw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in spread:
            scene.build(8 * b, 8 * b + 8, **bkw)
            scene.trace(dirs, out=out, **tkw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / len(spread)

    st_ = CFG3_AS_STATED
    psets = [("as_stated", dict(iod_threshold=st_["iod"], avg_mode=args.avg, tau_thin=st_["tau_thin"]),
              dict(mode="vlm", level_dist=[v * st_["grade_scale"] for v in rt.CASCADE_LEVEL_DIST], grade=args.grade)),
             ("sparse_classic", dict(iod_threshold=args.iod), dict(mode="level0")),
             ("headline_f32", dict(iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin),
              dict(mode="vlm", level_dist=level_dist, grade=args.grade))]
    perr = run_ladder(torch, np, [(n_, scene, b_, t_) for n_, b_, t_ in psets], {}, {}, dirs, probe_vox[k], d, ref,
                      nb)
    pareto = []
    for n_, b_, t_ in psets:
        ms_b = time_setting(b_, t_)
        pareto.append({"name": n_, "ms_per_batch": ms_b, "speedup_vs_dense_classic": dense_ms_batch / ms_b,
                       "p99.9": perr[n_]["p99.9"], "meets_bar": bool(perr[n_]["p99.9"] <= ACCURACY_BAR)})
    pareto.sort(key=lambda q: q["ms_per_batch"])
    out_line = {"workload": "cfg3", "accuracy_ladder": ladder, "accuracy_bar": ACCURACY_BAR, "pareto": pareto,
                "as_stated": "T=%g, thin bypass %g, cascade grading x%g" % (
                    st_["iod"], st_["tau_thin"], st_["grade_scale"]),
                "config": {
        "workload": "3D 256^3, 8^3 bricks, %d active (25%%), slab + %d loops, 2 Voigt lines (Core and Voigt) + "
                    "grey continuum, |v| <= 30 km/s, 4-level VLM T=%g, thin bypass %g, %s, 32 Fibonacci directions, "
                    "%d lambda (%d batches of 8), all %d probes" % (
                        int(sc["block_active"].sum()), int(sc["n_loops"]), args.iod, args.tau_thin,
                        _grading(args), nb * 8, nb, n_probes)},
        "seg_lam_per_solve": seglam, "dense_seg_lam_per_solve": dense_seglam,
        "dense_classic_gpu": {"ms_per_batch": dense_ms_batch, "ms_per_solve_extrapolated": dense_ms_batch * nb},
        "cpu_baseline": {**cpu, "value": cpu_seglam / cpu_s / 1e9, "unit": "Gsegments/s", "cores": nthreads,
                         "kind": "oracle", "sample": "%d seeded (probe, direction) pairs x %d wavelengths, FP64 "
                                                     "dense Classic (exact Voigt), %.1f s" % (k.size, nb * 8, cpu_s)},
        "dtypes": {}}
    for dt, r in res.items():
        bps = bytes_per_seg_lam("cav", dt, 3)
        out_line["dtypes"][dt] = {
            "ms_per_solve": r["ms_per_solve"], "mean_trace_ms": r["mean_trace_ms"],
            "raw_gseg_s": seglam / (r["ms_per_solve"] / 1e3) / 1e9,
            "dense_equiv_gseg_s": dense_seglam / (r["ms_per_solve"] / 1e3) / 1e9,
            "speedup_vs_dense_classic": dense_ms_batch * nb / r["ms_per_solve"],
            "trace_bytes_per_seg_lam": bps,
            "trace_hbm_frac_streamed": bps * seglam / nb / (r["mean_trace_ms"] / 1e3) / HBM_PEAK,
            "error_vs_fp64_classic": _err(r["got"], ref)}
        out_line["dtypes"][dt]["meets_accuracy_bar"] = bool(
            out_line["dtypes"][dt]["error_vs_fp64_classic"]["p99.9"] <= ACCURACY_BAR)
    if "f32" in res:
        for dt in res:
            if dt != "f32":
                out_line["dtypes"][dt]["speedup_vs_f32"] = res["f32"]["ms_per_solve"] / res[dt]["ms_per_solve"]
                out_line["dtypes"][dt]["error_vs_gpu_f32"] = _err(res[dt]["got"], res["f32"]["got"].astype(np.float64))
    if "f32" in res:
        cnt = measured_counters("counters_cav_cfg3", "cfg3 headline f32")
        if cnt is not None:
            # counts and launch time from the same profiled run (batches 0-3), as fractions of the peaks
            t_ = cnt["mean_launch_ms_kernel_trace"] / 1e3
            out_line["roofline"] = {
                "bound": "alu", "achieved": cnt["valu_insts_per_launch"] / t_ / 1e9,
                "peak": VALU_ISSUE_PEAK / 1e9, "unit": "G VALU wave-instructions/s",
                "frac": cnt["valu_insts_per_launch"] / t_ / VALU_ISSUE_PEAK, "traffic": cnt["hbm_bytes_per_launch"],
                "hbm_traffic_frac": cnt["hbm_bytes_per_launch"] / t_ / HBM_PEAK,
                "kernel": "k_trace<3, VisCav<3, float, AccPlain, 2>>", "counters": "profiles/counters_cav_cfg3.json",
                "mean_launch_ms": cnt["mean_launch_ms_kernel_trace"]}
    print(json.dumps(out_line), flush=True)


# ----------------------------------------------------------------------------- prefiltering
def bench_prefilter(args):
    """cfg2's scene with every line at rest, stored as static emission: VLM with box-filtered merged cells against
    VLM with prefiltered merged cells (Sect. 5.1) on the same level maps, for several level settings.  Error against
    the FP64 dense march of the same static emission (MIP-0 values at rest, every cell at MIP 0) on a seeded ray
    sample; time per batch over every fourth batch."""
    np, torch, rt, dev = _env()
    import oracle as orc
    from synth import make_cfg2
    sc = make_cfg2()
    nb = sc["lam"].size // 8
    if args.batches:
        nb = min(nb, args.batches)
    spread = list(range(2, nb, 4)) or [0]
    dirs = torch.from_numpy(sc["dirs"]).to(dev)
    n_dir = dirs.shape[0]
    box = rt.Scene.from_dict(sc, emission="static")
    pf = rt.Scene.from_dict(sc, emission="prefilter")
    n_probes = box.info["n_probes"]
    probes = box.probe_voxels()
    rng = np.random.default_rng(2027)
    k = rng.choice(probes.size, min(args.pairs, probes.size), replace=False)
    d = rng.integers(0, n_dir, k.size).astype(np.int32)
    cpu = host_cpu_info()
    ta = time.perf_counter()
    ref = np.zeros((k.size, nb * 8))
    lv0 = np.zeros(sc["block_active"].size, np.int8)
    for b in range(nb):
        s = orc.Scene(sc, lam_idx=list(range(8 * b, 8 * b + 8)))
        st_e = np.zeros((8, s.level_total))
        st_c = np.zeros((8, s.level_total))
        for il in range(8):
            st_e[il, :s.nvox], st_c[il, :s.nvox] = orc.lines_mip0(s, il, 0)
        s.set_static_levels(st_e, st_c)
        ref[:, 8 * b:8 * b + 8] = orc.march(s, orc.STATIC, lv0, probes[k], d, n_threads=cpu["threads"])
    log("prefilter: oracle reference (%d pairs x %d lambda) in %.1f s" % (k.size, nb * 8, time.perf_counter() - ta))
    tmp = torch.empty((n_dir, 8, n_probes), dtype=torch.float32, device=dev)

    def time_setting(scn, bkw, tkw):
        scn.build(8 * spread[0], 8 * spread[0] + 8, **bkw)
        scn.trace(dirs, out=tmp, **tkw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in spread:
            scn.build(8 * b, 8 * b + 8, **bkw)
            scn.trace(dirs, out=tmp, **tkw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / len(spread)

    settings = [("MIP 0 (no merging)", box, dict(iod_threshold=1e-2), dict(mode="level0"))]
    for T, thin, g in ((1e-2, 0.25, 1.0), (1e-2, 0.0, 4.0), (1e-3, 0.0, 4.0), (3e-4, 0.0, 16.0)):
        ld = [v * g for v in rt.CASCADE_LEVEL_DIST]
        for name, scn in (("box", box), ("prefiltered", pf)):
            settings.append(("%s T=%g thin %g grading x%g" % (name, T, thin, g), scn,
                             dict(iod_threshold=T, tau_thin=thin), dict(mode="vlm", level_dist=ld, grade="path")))
    errs = run_ladder(torch, np, settings, {}, {}, dirs, probes[k], d, ref, nb)
    for name, scn, b_, t_ in settings:
        errs[name]["ms_per_batch"] = time_setting(scn, b_, t_)
        errs[name]["meets_bar"] = bool(errs[name]["p99.9"] <= ACCURACY_BAR)
        log("prefilter: %-45s %.2f ms p99.9 %.3e" % (name, errs[name]["ms_per_batch"], errs[name]["p99.9"]))
    out = {"workload": "prefilter", "config": {
        "workload": "cfg2's scene (2D 1024^2, 16^2 bricks, 40%% active) with both lines at rest, static emission, "
                    "4-level mip chain, 64 dirs, %d lambda, all %d probes; merged cells box-filtered (Sect. 2.1) or "
                    "prefiltered (Sect. 5.1) on the same level maps" % (nb * 8, n_probes)},
        "error_vs": "FP64 dense march of the same static emission (every cell at MIP 0), %d seeded (probe, direction) "
                    "pairs" % k.size,
        "settings": errs, "cpu": cpu}
    print(json.dumps(out), flush=True)


# ----------------------------------------------------------------------------- cfg4
def bench_cfg4(args):
    """48 uneven scenes (2D 64^2-1024^2, 3D 64^3-192^3, 2-5 levels, 16-64 directions, 64-256
    wavelengths), BF16 storage: sequential per-scene launches vs one persistent batched launch per
    wavelength-batch wave (eager and graph-replayed), with the autotuned launch shape."""
    np, torch, rt, dev = _env()
    from synth import cfg4_specs, make_cfg4_scene
    specs = cfg4_specs()
    if args.scenes:
        specs = specs[:args.scenes]
    level_dist = None if args.no_grading else [v * args.grade_scale for v in rt.CASCADE_LEVEL_DIST]
    items = []
    tg = time.time()
    for i, sp in enumerate(specs):
        sc = make_cfg4_scene(sp)
        s = rt.Scene.from_dict(sc, emission="static")
        dirs = torch.from_numpy(sc["dirs"]).to(dev)
        out = torch.empty((dirs.shape[0], 8, s.info["n_probes"]), dtype=torch.float32, device=dev)
        items.append({"spec": sp, "scene": s, "dirs": dirs, "out": out, "nb": sp["n_lam"] // 8})
        del sc
        if i % 8 == 7:
            log("cfg4: %d scenes resident (%.0fs)" % (i + 1, time.time() - tg))
    waves = max(it["nb"] for it in items)
    if args.batches:
        waves = min(waves, args.batches)

    def build_wave(b, stream=None):
        for it in items:
            if it["nb"] > b:
                it["scene"].build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                                   storage="bf16", stream=stream)

    def sequential(stats=None, tag="sequential"):
        for b in range(waves):
            build_wave(b)
            for it in items:
                if it["nb"] > b:
                    it["scene"].trace(it["dirs"], mode="vlm", level_dist=level_dist, grade=args.grade, out=it["out"],
                                      stats=stats)
            if b % 8 == 7:
                torch.cuda.synchronize()
                log("cfg4 %s: wave %d/%d" % (tag, b + 1, waves))

    def jobs(part):
        return [{"scene": items[i]["scene"], "dirs": items[i]["dirs"], "out": items[i]["out"],
                 "level_dist": level_dist, "grade": args.grade} for i in part]

    parts = sorted({tuple(i for i, it in enumerate(items) if it["nb"] > b) for b in range(waves)}, key=len,
                   reverse=True)
    build_wave(0)
    best, tune_ms = rt.batch_autotune(jobs(parts[0]), reps=2)
    log("cfg4 autotune: %s (%.2f ms)" % (best, tune_ms))
    batches = {p: rt.Batch(jobs(p), **best) for p in parts}
    stream = torch.cuda.current_stream()

    def part_of(b):
        return tuple(i for i, it in enumerate(items) if it["nb"] > b)

    run_ev = []

    def batched(record=False, st=None, tag="batched"):
        for b in range(waves):
            build_wave(b, stream=st)
            if record:
                e0, e1 = _events(torch)
                e0.record(stream)
            batches[part_of(b)].run(st)
            if record:
                e1.record(stream)
                run_ev.append((e0, e1))
            if st is None and b % 8 == 7:
                torch.cuda.synchronize()
                log("cfg4 %s: wave %d/%d" % (tag, b + 1, waves))

    # correctness: wave 0 batched == sequential, bit for bit
    build_wave(0)
    for it in items:
        it["scene"].trace(it["dirs"], mode="vlm", level_dist=level_dist, grade=args.grade, out=it["out"])
    ref0 = [it["out"].clone() for it in items]
    for it in items:
        it["out"].fill_(-1.0)
    batches[part_of(0)].run()
    torch.cuda.synchronize()
    identical = all(torch.equal(r, it["out"]) for r, it in zip(ref0, items))
    del ref0
    log("cfg4 wave 0: batched == sequential bit for bit: %s" % identical)
    # timing (each phase: one untimed pass, then --steps timed passes)
    sequential(tag="sequential warm-up")
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(args.steps):
        sequential()
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - ta) * 1e3 / args.steps
    log("cfg4 sequential: %.1f ms per solve" % ms_seq)
    batched(tag="batched warm-up")
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(args.steps):
        batched(record=True)
    torch.cuda.synchronize()
    ms_bat = (time.perf_counter() - ta) * 1e3 / args.steps
    run_ms = [a.elapsed_time(b) for a, b in run_ev]
    log("cfg4 batched: %.1f ms per solve" % ms_bat)
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with rt.Graph(side) as g:
            batched(st=side)
        g.replay()
        side.synchronize()
        log("cfg4 graph captured and replayed once")
        ta = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
            side.synchronize()
            log("cfg4 graph replay done")
        ms_graph = (time.perf_counter() - ta) * 1e3 / args.steps
    torch.cuda.synchronize()
    log("cfg4 graph: %.1f ms per solve" % ms_graph)
    stats = torch.zeros(5, dtype=torch.int64, device=dev)
    sequential(stats=stats, tag="counting")
    torch.cuda.synchronize()
    seglam = int(stats[0].item()) * 8
    n2 = sum(1 for it in items if it["spec"]["dim"] == 2)
    out_line = {"workload": "cfg4", "config": {
        "workload": "%d scenes (%d 2D 64^2-1024^2 with 16^2 bricks, %d 3D 64^3-192^3 with 8^3 bricks), 2-5 level "
                    "VLM T=%g, %s, static Gaussian line + continuum, 16-64 directions, 64-256 wavelengths, BF16 "
                    "storage, all probes" % (len(items), n2, len(items) - n2, args.iod,
                                             _grading(args))},
        "waves": waves, "seg_lam_per_solve": seglam, "batched_equals_sequential": identical,
        "autotuned": best, "autotune_ms": tune_ms,
        "sequential": {"ms_per_solve": ms_seq, "raw_gseg_s": seglam / ms_seq / 1e6},
        "batched_eager": {"ms_per_solve": ms_bat, "raw_gseg_s": seglam / ms_bat / 1e6,
                          "mean_persistent_launch_ms": float(np.mean(run_ms)),
                          "sum_persistent_launch_ms": float(np.sum(run_ms)) / args.steps},
        "batched_graph": {"ms_per_solve": ms_graph, "raw_gseg_s": seglam / ms_graph / 1e6},
        "speedup_batched_vs_sequential": ms_seq / ms_bat, "speedup_graph_vs_sequential": ms_seq / ms_graph}
    print(json.dumps(out_line), flush=True)


# ----------------------------------------------------------------------------- cfg5
def bench_cfg5(args):
    """Radiance cache on the cfg3 scene (BF16 storage): generation of training rows from truncated
    full marches, Adam training, held-out check and fallback map, then the timed truncated march +
    cache against the plain FP32 and BF16 marches; errors against the FP64 oracle (gain test: the
    same truncation without the cache)."""
    np, torch, rt, dev = _env()
    from synth import make_cfg3
    T_TRUNC, THRESH = 32.0, 5e-3
    tg = time.time()
    sc = make_cfg3()
    log("cfg5 scene generated in %.1fs" % (time.time() - tg))
    nb = sc["lam"].size // 8
    if args.batches:
        nb = min(nb, args.batches)
    dirs = torch.from_numpy(sc["dirs"]).to(dev)
    n_dir = dirs.shape[0]
    level_dist = None if args.no_grading else [v * args.grade_scale for v in rt.CASCADE_LEVEL_DIST]
    scene = rt.Scene.from_dict(sc, emission="cav")
    n_probes = scene.info["n_probes"]
    probe_vox = scene.probe_voxels()
    rng = np.random.default_rng(5)
    ptr, phd = args.nrc_train_probes, args.nrc_held_probes
    sel = [rng.choice(n_probes, ptr + phd, replace=False) for _ in range(nb)]
    tr_probes = [torch.from_numpy(probe_vox[s_[:ptr]]).to(dev) for s_ in sel]
    hd_probes = [torch.from_numpy(probe_vox[s_[ptr:]]).to(dev) for s_ in sel]
    rows_b = n_dir * 8 * ptr
    raw = torch.zeros((nb * rows_b, 12), dtype=torch.float32, device=dev)
    tgt = torch.zeros(nb * rows_b, dtype=torch.float32, device=dev)
    freq = args.nrc_freq if args.nrc_freq > 0 else sc["n"][0] / 2.0
    nn = rt.Nrc(max_batch=2 ** 14, freq_max=freq, seed=5)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for b in range(nb):
        scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin, storage="bf16")
        tr = scene.trace_truncated(dirs, T_TRUNC, gen=True, probes=tr_probes[b], level_dist=level_dist,
                                   grade=args.grade)
        nn.pack(scene, tr, raw, tgt, b * rows_b)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - ta
    q_frac_train = float(raw[:, 11].mean().item())
    log("cfg5 generation: %d rows in %.2fs (query fraction %.3f)" % (raw.shape[0], gen_s, q_frac_train))
    ta = time.perf_counter()
    nn.train(raw, tgt, steps=1, batch=2 ** 14, lr=args.nrc_lr)
    loss0 = nn.loss()
    done = 1
    while done < args.nrc_steps:
        n = min(500, args.nrc_steps - done)
        nn.train(raw, tgt, steps=n, batch=2 ** 14, lr=args.nrc_lr)
        done += n
        log("cfg5 training: %d steps, loss %.3e" % (done, nn.loss()))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - ta
    loss1 = nn.loss()
    # held-out check -> one fallback map per wavelength batch: a block uses the cache in a batch only where its
    # held-out queries (at least --nrc-min-checks rays) all pass the threshold, so a line core where the near field
    # is thick can use the cache while its wings fall back, and no block uses it unchecked
    fbs = [torch.zeros(scene.info["n_blocks"], dtype=torch.uint8, device=dev) for _ in range(nb)]
    held_err = []
    for b in range(nb):
        fb = fbs[b]
        cnt = torch.zeros(scene.info["n_blocks"], dtype=torch.int32, device=dev)
        scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin, storage="bf16")
        tr = scene.trace_truncated(dirs, T_TRUNC, gen=True, probes=hd_probes[b], level_dist=level_dist,
                                   grade=args.grade)
        _, err = nn.validate(scene, tr, THRESH, fb, count=cnt)
        nn.fallback_unverified(scene, cnt, 8 * args.nrc_min_checks, fb)
        q = (tr["feat"][..., 3] > 0)[:, None, :].expand_as(err)
        held_err.append(err[q].cpu().numpy())
    torch.cuda.synchronize()
    held_err = np.concatenate(held_err) if held_err else np.zeros(1)
    act = torch.from_numpy(scene.active_blocks().astype(np.int64)).to(dev)
    n_flag = float(np.mean([int(f[act].sum().item()) for f in fbs]))  # active blocks falling back, per batch
    log("cfg5 held-out: median %.3e p99.9 %.3e; %.1f blocks flagged per batch" % (
        np.median(held_err), np.percentile(held_err, 99.9, method="higher"), n_flag))
    # timed solves on all probes
    kk_np = rng.choice(n_probes, min(args.pairs, n_probes), replace=False)
    d_np = rng.integers(0, n_dir, kk_np.size).astype(np.int32)
    kk, dd = torch.from_numpy(kk_np).long().to(dev), torch.from_numpy(d_np).long().to(dev)
    out = torch.empty((n_dir, 8, n_probes), dtype=torch.float32, device=dev)
    outc = torch.empty_like(out)
    stream = torch.cuda.current_stream()

    def plain(dt, gather=None):
        for b in range(nb):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin, storage=dt)
            scene.trace(dirs, mode="vlm", level_dist=level_dist, grade=args.grade, out=out)
            if gather is not None:
                gather[:, 8 * b:8 * b + 8] = out[dd, :, kk]

    nrc_ev = []

    def cached(gather=None, gather_cut=None, fallback=fbs, record=False):
        qsum = 0
        for b in range(nb):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin, storage="bf16")
            if record:
                e0, e1 = _events(torch)
                e0.record(stream)
            tr = scene.trace_truncated(dirs, T_TRUNC, gen=False, fallback=None if fallback is None else fallback[b],
                                       level_dist=level_dist, grade=args.grade)
            if record:
                e1.record(stream)
            nn.compose(scene, tr, out=outc)
            if record:
                e2 = torch.cuda.Event(enable_timing=True)
                e2.record(stream)
                nrc_ev.append((e0, e1, e2))
            if gather is not None:
                gather[:, 8 * b:8 * b + 8] = outc[dd, :, kk]
                gather_cut[:, 8 * b:8 * b + 8] = tr["I_near"][dd, :, kk]
                qsum += int((tr["feat"][..., 3] > 0).sum().item())
            del tr
        return qsum

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    ms_f32 = timed(lambda: plain("f32"))
    ms_bf16 = timed(lambda: plain("bf16"))
    ms_nrc = timed(lambda: cached(record=True))
    tr_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in nrc_ev]))
    comp_ms = float(np.mean([b.elapsed_time(c) for _, b, c in nrc_ev]))
    log("cfg5 solve ms: plain f32 %.1f, plain bf16 %.1f, cache %.1f (trace %.2f + compose %.2f per batch)" % (
        ms_f32, ms_bf16, ms_nrc, tr_ms, comp_ms))
    g_f32 = torch.empty((kk.numel(), nb * 8), device=dev)
    g_bf16, g_nrc, g_cut, g_nrc0, g_cut0 = (torch.empty_like(g_f32) for _ in range(5))
    plain("f32", g_f32)
    plain("bf16", g_bf16)
    queries = cached(g_nrc, g_cut)
    queries0 = cached(g_nrc0, g_cut0, fallback=None)
    torch.cuda.synchronize()
    # the accuracy/speed trade of the held-out threshold: fallback maps at looser thresholds, each timed over
    # one full solve (after one warm-up) and measured on the same sampled pairs
    sweep = []
    for thr in (5e-2, 2e-1, 1.0):
        fbt = [torch.zeros(scene.info["n_blocks"], dtype=torch.uint8, device=dev) for _ in range(nb)]
        for b in range(nb):
            cnt = torch.zeros(scene.info["n_blocks"], dtype=torch.int32, device=dev)
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                        storage="bf16")
            tr = scene.trace_truncated(dirs, T_TRUNC, gen=True, probes=hd_probes[b], level_dist=level_dist,
                                       grade=args.grade)
            nn.validate(scene, tr, thr, fbt[b], count=cnt)
            nn.fallback_unverified(scene, cnt, 8 * args.nrc_min_checks, fbt[b])
            del tr
        cached(fallback=fbt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cached(fallback=fbt)
        torch.cuda.synchronize()
        ms_t = (time.perf_counter() - t0) * 1e3
        g_t, g_tc = torch.empty_like(g_f32), torch.empty_like(g_f32)
        q_t = cached(g_t, g_tc, fallback=fbt)
        sweep.append({"held_out_thresh": thr, "ms_per_solve": ms_t, "speedup_vs_plain_f32": ms_f32 / ms_t,
                      "fallback_block_frac": float(np.mean([int(f[act].sum().item()) for f in fbt])) / int(act.numel()),
                      "query_ray_frac": q_t / (n_dir * n_probes * nb), "I": g_t.cpu().numpy()})
        log("cfg5 threshold %g: %.1f ms per solve (%.2fx plain), %.1f %% of blocks fall back" % (
            thr, ms_t, ms_f32 / ms_t, 100 * sweep[-1]["fallback_block_frac"]))
    torch.cuda.synchronize()
    cpu = host_cpu_info()
    nthreads = cpu["threads"]
    ref, cpu_seglam, cpu_s = _oracle_classic(sc, probe_vox, kk_np, d_np, list(range(nb * 8)), nthreads)
    f32_np = g_f32.cpu().numpy().astype(np.float64)
    rays = n_dir * n_probes
    out_line = {"workload": "cfg5", "config": {
        "workload": "radiance cache on the 3D 256^3 Core-and-Voigt scene (%d active bricks), BF16 storage, "
                    "truncation at path %g, %d lambda, 32 directions, all %d probes; %d training rows, %d held-out "
                    "probes per batch; MLP 256-4x64 SiLU-1 BF16 MFMA, frequencies up to %g, Adam lr %g batch 16384, "
                    "%d steps" % (int(sc["block_active"].sum()), T_TRUNC, nb * 8, n_probes, raw.shape[0], phd, freq,
                                  args.nrc_lr, args.nrc_steps)},
        "timing_ms_per_solve": {"plain_f32": ms_f32, "plain_bf16": ms_bf16, "cache": ms_nrc,
                                "cache_trace_per_batch": tr_ms, "cache_compose_per_batch": comp_ms},
        "speedup_cache_vs_plain_f32": ms_f32 / ms_nrc, "speedup_cache_vs_plain_bf16": ms_bf16 / ms_nrc,
        "speedup_bf16_vs_f32": ms_f32 / ms_bf16,
        "generation_s": gen_s, "training_s": train_s, "loss_first": loss0, "loss_last": loss1,
        "held_out_rel_err": {"n": int(held_err.size), "p50": float(np.median(held_err)),
                             "p99": float(np.percentile(held_err, 99, method="higher")),
                             "p99.9": float(np.percentile(held_err, 99.9, method="higher"))},
        "fallback_active_blocks_per_batch": n_flag, "fallback_block_frac": n_flag / int(act.numel()),
        "query_ray_frac": queries / (rays * nb), "query_ray_frac_without_fallback": queries0 / (rays * nb),
        "error_vs_fp64_classic": {"plain_f32": _err(f32_np, ref), "plain_bf16": _err(g_bf16.cpu().numpy(), ref),
                                  "cache": _err(g_nrc.cpu().numpy(), ref),
                                  "truncated_no_cache": _err(g_cut.cpu().numpy(), ref),
                                  "cache_without_fallback": _err(g_nrc0.cpu().numpy(), ref),
                                  "truncated_no_cache_no_fallback": _err(g_cut0.cpu().numpy(), ref)},
        "held_out_threshold_sweep": [{**{k: v for k, v in w.items() if k != "I"}, "error_vs_fp64_classic": _err(w["I"], ref)}
                                     for w in sweep],
        "error_vs_gpu_plain_f32": {"plain_bf16": _err(g_bf16.cpu().numpy(), f32_np),
                                   "cache": _err(g_nrc.cpu().numpy(), f32_np),
                                   "truncated_no_cache": _err(g_cut.cpu().numpy(), f32_np)},
        "cpu_baseline": {**cpu, "value": cpu_seglam / cpu_s / 1e9, "unit": "Gsegments/s", "cores": nthreads,
                         "kind": "oracle", "sample": "%d pairs x %d wavelengths, FP64 dense Classic, %.1f s" % (
                             kk_np.size, nb * 8, cpu_s)}}
    # the network kernel's roofline on dense rows (`--workload nrc_forward`): in the compose pass above most
    # rows fall back and are copied, so its dispatch times the copies, not the MLP
    cnt = measured_counters("counters_nrc_forward_dense", sources=NRC_SOURCES)
    if cnt is not None:
        out_line["roofline_nrc_forward"] = {
            "bound": "mfma", "achieved": cnt["achieved_tflops"], "peak": 2500.0, "unit": "TFLOP/s",
            "frac": cnt["mfma_frac_of_peak"], "mfma_busy_frac": cnt["mfma_busy_frac"],
            "valu_issue_frac": cnt["valu_issue_frac"], "rows": "2^22 dense rows (bench.py --workload nrc_forward)",
            "counters": "profiles/counters_nrc_forward_dense.json"}
    print(json.dumps(out_line), flush=True)


# ----------------------------------------------------------------------------- cache network forward
NRC_FLOP_PER_ROW = 2 * (256 * 64 + 3 * 64 * 64 + 64)


def bench_nrc_forward(args):
    """The cache network's fused forward kernel alone (rt_nrc_predict) on 2^22 dense training-form rows:
    every 16-row tile holds queries, so the MLP's MFMA rate is measured without the compose pass's
    fallback copies.  Seeded uniform features in the ranges the packed rows take (positions, directions,
    wavelength offset and level statistics in [-1, 1]); the network is the library's seeded initialisation."""
    import numpy as np
    import torch
    import paper_2511_08498_amd as rt
    rt.lib()
    dev = torch.device("cuda")
    n = 1 << 22
    g = torch.Generator(device="cpu").manual_seed(7)
    raw = (torch.rand((n, 12), generator=g) * 2.0 - 1.0).to(dev)
    raw[:, 11] = 1.0
    nn = rt.Nrc(max_batch=2 ** 14, freq_max=128.0, seed=5)
    stream = torch.cuda.current_stream()
    for _ in range(max(args.warmup, 1)):
        nn.predict(raw)
    torch.cuda.synchronize()
    ms = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        y = nn.predict(raw)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = float(np.mean(ms)) / 1e3
    assert torch.isfinite(y).all().item()
    tflops = n * NRC_FLOP_PER_ROW / t / 1e12
    line = {"workload": "nrc_forward",
            "config": {"workload": "cache network 256-4x64 SiLU-1, BF16 MFMA, fused Fourier encoding (frequencies "
                                   "up to 128), 4194304 dense rows per launch"},
            "ms_per_launch": float(np.mean(ms)), "launches": args.steps, "rows_per_s": n / t,
            "roofline": {"bound": "mfma", "achieved": tflops, "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": tflops / 2500.0, "flop_per_row": NRC_FLOP_PER_ROW}}
    cnt = measured_counters("counters_nrc_forward_dense", sources=NRC_SOURCES)
    if cnt is not None:
        line["roofline"].update({"mfma_busy_frac": cnt["mfma_busy_frac"], "valu_issue_frac": cnt["valu_issue_frac"],
                                 "counters": "profiles/counters_nrc_forward_dense.json"})
    log("nrc forward: %.3f ms per launch, %.3g rows/s, %.1f TFLOP/s (%.1f %% of the BF16 dense peak)" % (
        t * 1e3, n / t, tflops, 100 * tflops / 2500.0))
    print(json.dumps(line), flush=True)


# training step: the forward with saved activations, and on the matrix cores per row the weight gradients of the
# four hidden layers (2 x (256 x 64 + 3 x 64 x 64)) and the activation gradients below the top three
# (2 x 3 x 64 x 64); the output layer's gradients are column sums on the vector units
NRC_TRAIN_FLOP_PER_ROW = NRC_FLOP_PER_ROW + 2 * (256 * 64 + 3 * 64 * 64) + 2 * 3 * 64 * 64


def bench_nrc_train(args):
    """Training steps of the cache network (rt_nrc_train: the fused forward writing its activations, the
    split-K MFMA backward, Adam) at the cache's batch of 2^14 rows drawn from 2^20 seeded rows: time per step,
    rows and MFMA-shaped FLOP per second.  Seeded uniform features as in nrc_forward, targets a smooth
    function of them (the time does not depend on the values)."""
    import numpy as np
    import torch
    import paper_2511_08498_amd as rt
    rt.lib()
    dev = torch.device("cuda")
    n, batch = 1 << 20, 1 << 14
    g = torch.Generator(device="cpu").manual_seed(11)
    raw = (torch.rand((n, 12), generator=g) * 2.0 - 1.0)
    raw[:, 11] = 1.0
    tgt = (0.3 * torch.sin(3.0 * raw[:, 0]) * torch.cos(2.0 * raw[:, 1]) + 0.1 * raw[:, 6]).to(dev)
    raw = raw.to(dev)
    nn = rt.Nrc(max_batch=batch, freq_max=128.0, seed=5)
    stream = torch.cuda.current_stream()
    steps = 50
    nn.train(raw, tgt, steps=max(args.warmup, 1) * steps, batch=batch, lr=1e-3)
    torch.cuda.synchronize()
    loss0 = nn.loss()
    ms = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        nn.train(raw, tgt, steps=steps, batch=batch, lr=1e-3)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1) / steps)
    loss1 = nn.loss()
    assert np.isfinite(loss1)
    t = float(np.mean(ms)) / 1e3
    tflops = batch * NRC_TRAIN_FLOP_PER_ROW / t / 1e12
    line = {"workload": "nrc_train",
            "config": {"workload": "cache network 256-4x64 SiLU-1 training: BF16 MFMA forward + split-K MFMA "
                                   "backward + Adam (FP32 master weights), 16384 rows per step from 1048576"},
            "ms_per_step": float(np.mean(ms)), "steps_timed": args.steps * steps, "rows_per_s": batch / t,
            "loss_after_warmup": loss0, "loss_end": loss1,
            "roofline": {"bound": "mfma", "achieved": tflops, "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": tflops / 2500.0, "flop_per_row": NRC_TRAIN_FLOP_PER_ROW}}
    cnt = measured_counters("counters_nrc_train", sources=NRC_SOURCES)
    if cnt is not None:
        line["roofline"]["counters"] = "profiles/counters_nrc_train.json"
        line["roofline"]["per_kernel"] = cnt["per_kernel"]
    log("nrc train: %.3f ms per step of %d rows, %.3g rows/s, %.2f TFLOP/s (%.2f %% of the BF16 dense peak)" % (
        t * 1e3, batch, batch / t, tflops, 100 * tflops / 2500.0))
    print(json.dumps(line), flush=True)


# ----------------------------------------------------------------------------- method matrix
def bench_matrix(args):
    """{Dense, Sparse} x {Classic, VelInterp, CaV} x {-, Mips} on the prominence-like 2D scene (512 x 768,
    16^2 bricks, ~58 % active, two Voigt lines, shear flow): time per full solve (16 wavelength batches),
    updates applied, and error against the FP64 dense Classic oracle on the same sampled rays.  Classic is
    the exact per-voxel line evaluation, which is what Core and Voigt computes at MIP 0, so Classic and CaV
    at MIP 0 are one method here; dense methods trace the same (active-voxel) probes."""
    np, torch, rt, dev = _env()
    from synth import make_prominence
    sc = make_prominence()
    nb = sc["lam"].size // 8
    if args.batches:
        nb = min(nb, args.batches)
    dirs = torch.from_numpy(sc["dirs"]).to(dev)
    n_dir = dirs.shape[0]
    level_dist = None if args.no_grading else [v * args.grade_scale for v in rt.CASCADE_LEVEL_DIST]
    sparse_cav = rt.Scene.from_dict(sc, emission="cav")
    probe_vox = sparse_cav.probe_voxels()
    pv = torch.from_numpy(probe_vox).to(dev)
    n_probes = probe_vox.size
    rng = np.random.default_rng(77)
    k = rng.choice(n_probes, min(args.pairs, n_probes), replace=False)
    d = rng.integers(0, n_dir, k.size).astype(np.int32)
    kk, dd = torch.from_numpy(k).long().to(dev), torch.from_numpy(d).long().to(dev)
    scenes = {"dense_cav": rt.Scene.from_dict(sc, emission="cav", dense=True), "sparse_cav": sparse_cav,
              "sparse_velinterp": rt.Scene.from_dict(sc, emission="velinterp", n_v=args.n_v)}
    methods = [("DenseClassic", "dense_cav", "level0"), ("SparseClassic", "sparse_cav", "level0"),
               ("SparseVelInterp", "sparse_velinterp", "level0"), ("DenseCavMips", "dense_cav", "vlm"),
               ("SparseCavMips", "sparse_cav", "vlm"), ("SparseVelInterpMips", "sparse_velinterp", "vlm")]
    out = torch.empty((n_dir, 8, n_probes), dtype=torch.float32, device=dev)
    bkw = dict(iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin)
    res = {}
    for name, key, mode in methods:
        scn = scenes[key]
        probes = None if key.startswith("sparse") else pv

        def solve(stats=None, gather=None):
            for b in range(nb):
                scn.build(8 * b, 8 * b + 8, **bkw)
                scn.trace(dirs, probes=probes, mode=mode, level_dist=level_dist if mode == "vlm" else None,
                          grade=args.grade, out=out,
                          stats=stats)
                if gather is not None:
                    gather[:, 8 * b:8 * b + 8] = out[dd, :, kk]

        solve()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(args.steps):
            solve()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - ta) * 1e3 / args.steps
        stats = torch.zeros(5, dtype=torch.int64, device=dev)
        got = torch.empty((k.size, nb * 8), dtype=torch.float32, device=dev)
        solve(stats=stats, gather=got)
        torch.cuda.synchronize()
        res[name] = {"ms_per_solve": ms, "seg_lam_per_solve": int(stats[0].item()) * 8, "got": got.cpu().numpy()}
        log("matrix %-20s %.1f ms per solve" % (name, ms))
    cpu = host_cpu_info()
    nthreads = cpu["threads"]
    ref, cpu_seglam, cpu_s = _oracle_classic(sc, probe_vox, k, d, list(range(nb * 8)), nthreads)
    base = res["DenseClassic"]["ms_per_solve"]
    table = {}
    for name, r in res.items():
        table[name] = {"ms_per_solve": r["ms_per_solve"], "speedup_vs_dense_classic": base / r["ms_per_solve"],
                       "raw_gseg_s": r["seg_lam_per_solve"] / (r["ms_per_solve"] / 1e3) / 1e9,
                       "error_vs_fp64_classic": _err(r["got"], ref)}
    line = {"workload": "matrix", "config": {
        "workload": "2D 512 x 768 prominence-like sheet, 16^2 bricks, %d of %d active, 2 Voigt lines + grey "
                    "continuum, shear flow |v| <= 30 km/s, %d directions, %d lambda (%d batches), VLM T=%g, %s; "
                    "velocity interpolation n_v=%d; all %d active-voxel probes" % (
                        int(sc["block_active"].sum()), sc["block_active"].size, n_dir, nb * 8, nb, args.iod,
                        _grading(args), args.n_v, n_probes)},
        "methods": table,
        "cpu_baseline": {**cpu, "value": cpu_seglam / cpu_s / 1e9, "unit": "Gsegments/s", "cores": nthreads,
                         "kind": "oracle", "sample": "%d pairs x %d wavelengths, FP64 dense Classic, %.1f s" % (
                             k.size, nb * 8, cpu_s)}}
    print(json.dumps(line), flush=True)

if __name__ == "__main__":
    main()
