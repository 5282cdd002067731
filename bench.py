#!/usr/bin/env python
"""Formal-solution benchmark on one MI355X.

Workload (default): 2D 1024^2 grid, 16^2 bricks (40 % active), two Gaussian
lines + continuum with a +-30 km/s velocity field handled by velocity
interpolation (21 nodes), 4-level VLM mip chain with IoD threshold 1e-2 and
the paper's thin bypass, 64 directions from every active voxel, 256
wavelengths in batches of 8.

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
  comparators     DenseClassic (exact line profile in every MIP-0 cell of
                  the full grid) and SparseVelInterp (HDDA at MIP 0), timed
                  over a subset of batches;
  error           p99.9 (and the paper's percentile set) of the relative
                  intensity error against the FP64 dense Classic oracle on a
                  seeded ray sample;
  roofline        the march kernel's algorithmic bytes per launch / its mean
                  launch time (HIP events on the launch stream) vs 8 TB/s;
  cpu_baseline    the FP64 oracle timed on the host on the same ray sample.
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
VALU_ISSUE_PEAK = 256 * 2.4e9  # wave64 VALU instructions per second: 256 CUs x 1 per clock (4 SIMD16, non-packed)
MARCH_SOURCES = ("march.hip", "common.h", "profile.h")


def march_source_hash():
    """SHA-256 over the sources the march kernels are compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in MARCH_SOURCES:
        with open(os.path.join(ROOT, "paper_2511_08498_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters(name):
    """Counter summary profiles/<name>.json if it was taken on the current march sources, else None."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        c = json.load(fh)
    return c if c.get("march_source_sha256") == march_source_hash() else None


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
    ap.add_argument("--workload", default="cfg2", choices=["cfg2", "cfg3", "cfg4", "cfg5", "matrix"],
                    help="cfg2: 2D velocity interpolation (default, the headline line); cfg3: 3D Core and Voigt "
                         "per storage dtype; cfg4: 48-scene batched vs sequential; cfg5: radiance cache on cfg3; "
                         "matrix: the paper's method matrix on a prominence-like 2D scene")
    ap.add_argument("--emission", default="velinterp", choices=["velinterp", "static", "cav"])
    ap.add_argument("--n-v", type=int, default=21)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"],
                    help="cfg2: storage of the velocity-node / value records (FP32 accumulation in every case)")
    ap.add_argument("--iod", type=float, default=None, help="IoD threshold T (default 1 for matrix, else 1e-2)")
    ap.add_argument("--avg", default="linear", choices=["log", "linear"], help="stored level values: arithmetic "
                    "(box filter, default) or geometric mean of the children")
    ap.add_argument("--tau-thin", type=float, default=0.25, help="thin bypass threshold on a cell's optical side")
    ap.add_argument("--grade-scale", type=float, default=1.0, help="multiplies the cascade level distances")
    ap.add_argument("--iod-frame", default="rest", choices=["rest", "core"],
                    help="velocity interpolation: level test with lines at rest (the paper) or core-closest")
    ap.add_argument("--no-grading", action="store_true", help="plain VLM (no distance-graded cap)")
    ap.add_argument("--grade", default="path", choices=["entry", "path"],
                    help="distance-graded cap taken along the path (the cascade intervals' caps) or at each "
                         "block's entry")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--compare-batches", type=int, default=4)
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
    ap.add_argument("--nrc-held-probes", type=int, default=128, help="cfg5: held-out probes per wavelength batch")
    ap.add_argument("--scenes", type=int, default=0, help="cfg4: first N scenes only (0 = all 48)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU (--gpus %d requested): rays are independent given the scene, and the "
              "path would shard by wavelength batch with no exchange." % args.gpus)
        sys.exit(2)
    if args.iod is None:
        # the method matrix mirrors the deployment of Sect. 4.1 (IoD threshold 1); elsewhere 1e-2
        args.iod = 1.0 if args.workload == "matrix" else 1e-2
    if args.workload == "cfg3":
        return bench_cfg3(args)
    if args.workload == "cfg4":
        return bench_cfg4(args)
    if args.workload == "cfg5":
        return bench_cfg5(args)
    if args.workload == "matrix":
        return bench_matrix(args)
    return bench_cfg2(args)


def bench_cfg2(args):

    import numpy as np
    import torch

    import paper_2511_08498_amd as rt
    from synth import make_cfg2

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.time()
    sc = make_cfg2()
    log("scene generated in %.1fs" % (time.time() - t_gen))
    n_lam = sc["lam"].size
    nb_lam = n_lam // 8
    if args.batches:
        nb_lam = min(nb_lam, args.batches)
        n_lam = 8 * nb_lam
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb * 2 ** 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d MiB read + %d MiB written per copy, 3 copies" % (args.copy_probe_mb, args.copy_probe_mb))
        del src, dst
    dirs = torch.from_numpy(sc["dirs"]).to(dev)
    n_dir = dirs.shape[0]
    level_dist = None if args.no_grading else [v * args.grade_scale for v in rt.CASCADE_LEVEL_DIST]
    scene = rt.Scene.from_dict(sc, emission=args.emission, n_v=args.n_v)
    n_probes = scene.info["n_probes"]
    I_all = torch.empty((nb_lam, n_dir, 8, n_probes), dtype=torch.float32, device=dev)
    log("scene: %d active bricks, %d probes, output %.1f GB" % (scene.info["n_active"], n_probes,
                                                               I_all.numel() * 4 / 1e9))
    stream = torch.cuda.current_stream()
    ev = []

    def step(record=False, stats=None):
        for b in range(nb_lam):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                        iod_frame=args.iod_frame, storage=args.storage)
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
    achieved = bps * seglam_launch / (mean_trace_ms / 1e3)
    # measured DRAM bytes and VALU issue per launch from the committed rocprofv3 counter summary,
    # only while it matches the kernel sources (else null)
    cnt = measured_counters("counters_%s_cfg2" % args.emission) if args.n_v == 21 and args.storage == "f32" else None
    traffic = None
    valu = None
    if cnt is not None:
        traffic = cnt["hbm_bytes_per_launch"]
        valu = {"valu_insts_per_launch": cnt["valu_insts_per_launch"],
                "issue_frac": cnt["valu_insts_per_launch"] / (VALU_ISSUE_PEAK * mean_trace_ms / 1e3),
                "measured_hbm_gbs": traffic / (mean_trace_ms * 1e6)}
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": traffic, "valu": valu,
                "kernel": ("k_trace<2, VisVelinterp<2, %s>>" % STORAGE_T[args.storage]) if args.emission == "velinterp"
                else "k_trace",
                "bytes_per_seg_lam": bps, "seg_lam_per_launch": seglam_launch,
                "mean_launch_ms": mean_trace_ms}

    out = {"metric": METRIC, "value": value, "unit": "Gsegments/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
           "config": {"workload": (
               "2D 1024^2, 16^2 bricks, 40%% active, 2 Gaussian lines + continuum, |v| <= 30 km/s, %s (n_v=%d), "
               "%s storage, 4-level VLM T=%g, %s means, thin %g, level test %s frame, %s, 64 dirs, 256 lambda "
               "(32 batches of 8), all %d probes" % (args.emission, args.n_v, args.storage.upper(), args.iod, args.avg,
                                                     args.tau_thin, args.iod_frame, _grading(args), n_probes)),
                      "value_kind": "dense-equivalent segment-wavelength updates per second"},
           "raw_gseg_s": raw, "seg_lam_per_step": seglam_step, "dense_seg_lam_per_step": dense_seglam_step,
           "lane_utilisation": lane_util,
           "roofline": roofline}

    # ---- comparators
    if not args.no_compare:
        cmp = {}
        nbc = min(args.compare_batches, nb_lam)
        dc = rt.Scene.from_dict(sc, emission="cav", dense=True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for b in range(nbc):
            dc.build(8 * b, 8 * b + 8, iod_threshold=args.iod)
            dc.trace(dirs, probes=probes_vox, mode="level0", out=tmp)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        cmp["dense_classic"] = {"gseg_s": dense_cells * 8 * nbc / (tb - ta) / 1e9,
                                "ms_per_batch": (tb - ta) * 1e3 / nbc}
        del dc
        torch.cuda.synchronize()
        ta = time.perf_counter()
        sp_stats = torch.zeros(5, dtype=torch.int64, device=dev)
        for b in range(nbc):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                        iod_frame=args.iod_frame)
            scene.trace(dirs, mode="level0", out=tmp)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for b in range(nbc):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                        iod_frame=args.iod_frame)
            scene.trace(dirs, mode="level0", out=tmp, stats=sp_stats)
        torch.cuda.synchronize()
        cmp["sparse_" + args.emission] = {"gseg_s": dense_cells * 8 * nbc / (tb - ta) / 1e9,
                                          "raw_gseg_s": int(sp_stats[0].item()) * 8 / (tb - ta) / 1e9,
                                          "ms_per_batch": (tb - ta) * 1e3 / nbc}
        vlm_ms_batch = ms_step / nb_lam
        cmp["speedup_vs_dense_classic"] = cmp["dense_classic"]["ms_per_batch"] / vlm_ms_batch
        # angle-integrated output (mean intensity J + diagonal operator) instead of I per direction
        jbuf = torch.empty((8, n_probes), dtype=torch.float32, device=dev)
        pbuf = torch.empty_like(jbuf)
        for b in range(nbc):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                        iod_frame=args.iod_frame)
            scene.trace_j(dirs, mode="vlm", level_dist=level_dist, grade=args.grade, J=jbuf, psi=pbuf)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for b in range(nbc):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                        iod_frame=args.iod_frame)
            scene.trace_j(dirs, mode="vlm", level_dist=level_dist, grade=args.grade, J=jbuf, psi=pbuf)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        cmp["vlm_j_output"] = {"ms_per_batch": (tb - ta) * 1e3 / nbc,
                               "speedup_vs_i_output": vlm_ms_batch / ((tb - ta) * 1e3 / nbc),
                               "note": "same march; J and psi [8][probes] instead of I [64 dirs][8][probes]"}
        # radiance intervals: the same rays split at the cascade interval ends 1.5 * 4^c, each interval
        # with its cascade's maximum MIP level, I and T written per interval (what a merge consumes)
        ends, caps = [0.0, 1.5, 6.0, 24.0, 96.0, float("inf")], [0, 0, 1, 2, 3]
        ibufs = [(torch.empty_like(tmp), torch.empty_like(tmp)) for _ in caps]
        iv_stats = torch.zeros(5, dtype=torch.int64, device=dev)

        def intervals(stats=None):
            for c in range(len(caps)):
                scene.trace_interval(dirs, ends[c], ends[c + 1], mode="vlm", max_level=caps[c], out=ibufs[c][0],
                                     out_T=ibufs[c][1], stats=stats)
        for b in range(nbc):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                        iod_frame=args.iod_frame)
            intervals()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for b in range(nbc):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                        iod_frame=args.iod_frame)
            intervals()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for b in range(nbc):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                        iod_frame=args.iod_frame)
            intervals(stats=iv_stats)
        torch.cuda.synchronize()
        cmp["cascade_intervals"] = {"ms_per_batch": (tb - ta) * 1e3 / nbc,
                                    "raw_gseg_s": int(iv_stats[0].item()) * 8 / (tb - ta) / 1e9,
                                    "vs_whole_ray_vlm": vlm_ms_batch / ((tb - ta) * 1e3 / nbc),
                                    "intervals": [[ends[c], ends[c + 1], caps[c]] for c in range(len(caps))],
                                    "note": "same rays split at 1.5 * 4^c, per-cascade MIP caps, I and T of "
                                            "every interval written"}
        del ibufs
        if args.emission == "velinterp":
            # the accuracy-preserving setting: no merging, 81 velocity nodes (error filled in below)
            scene81 = rt.Scene.from_dict(sc, emission="velinterp", n_v=81)
            kw81 = dict(iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin)
            for b in range(nbc):
                scene81.build(8 * b, 8 * b + 8, **kw81)
                scene81.trace(dirs, mode="level0", out=tmp)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for b in range(nbc):
                scene81.build(8 * b, 8 * b + 8, **kw81)
                scene81.trace(dirs, mode="level0", out=tmp)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            cmp["sparse_velinterp_nv81"] = {"gseg_s": dense_cells * 8 * nbc / (tb - ta) / 1e9,
                                            "ms_per_batch": (tb - ta) * 1e3 / nbc,
                                            "speedup_vs_dense_classic":
                                                cmp["dense_classic"]["ms_per_batch"] / ((tb - ta) * 1e3 / nbc)}
            # the same VLM march with the node records stored in FP32 / BF16 / FP16, timed on the same
            # batches (error filled in below)
            node_t = {}
            for dt in ("f32", "bf16", "f16"):
                kwd = dict(iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin,
                           iod_frame=args.iod_frame, storage=dt)
                for b in range(nbc):
                    scene.build(8 * b, 8 * b + 8, **kwd)
                    scene.trace(dirs, mode="vlm", level_dist=level_dist, grade=args.grade, out=tmp)
                torch.cuda.synchronize()
                evd = []
                ta = time.perf_counter()
                for b in range(nbc):
                    scene.build(8 * b, 8 * b + 8, **kwd)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    scene.trace(dirs, mode="vlm", level_dist=level_dist, grade=args.grade, out=tmp)
                    e1.record(stream)
                    evd.append((e0, e1))
                torch.cuda.synchronize()
                tb = time.perf_counter()
                node_t[dt] = ((tb - ta) * 1e3 / nbc, float(np.mean([a.elapsed_time(b2) for a, b2 in evd])))
            for dt, (ms_b, lms) in node_t.items():
                cmp["vlm_%s_nodes" % dt] = {
                    "ms_per_batch": ms_b, "mean_launch_ms": lms,
                    "step_speedup_vs_f32": node_t["f32"][0] / ms_b, "launch_speedup_vs_f32": node_t["f32"][1] / lms,
                    "note": "batches 0-%d, build + VLM trace; node records %d B per segment" % (
                        nbc - 1, 128 if dt == "f32" else 64)}
        out["comparators"] = cmp

    # ---- accuracy and CPU baseline on a seeded ray sample
    if not args.no_cpu_baseline:
        import oracle as orc
        rng = np.random.default_rng(2025)
        probes = scene.probe_voxels()
        ncores = os.cpu_count() or 1
        nthreads = min(ncores, 16)

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
                                         "march (exact line profiles), %.1f s" % (npairs, n_lam, dt)}
        dd = torch.from_numpy(d).long().to(dev)
        kk = torch.from_numpy(k).long().to(dev)
        got = I_all[:, dd, :, kk].reshape(len(k), n_lam).cpu().numpy()  # [pair][lam]
        err = orc.rel_err_stats(got, ref)
        out["error"] = {"vs": "FP64 dense Classic oracle", "n": err["n"],
                        **{k2: err[k2] for k2 in err if k2.startswith("p")}}
        out["cpu_baseline"]["calibration_rate_gseg_s"] = rate / 1e9
        if "comparators" in out and "sparse_velinterp_nv81" in out["comparators"]:
            e81 = run_ladder(torch, np, [("sparse MIP 0, n_v=81", scene81, {}, {"mode": "level0"})],
                             dict(iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin), {},
                             dirs, probes[k], d, ref, nb_lam)
            out["comparators"]["sparse_velinterp_nv81"]["error_vs_fp64_classic"] = e81["sparse MIP 0, n_v=81"]
            base_b = dict(iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin, iod_frame=args.iod_frame)
            for dt in ("f32", "bf16", "f16"):
                key = "vlm_%s_nodes" % dt
                if key in out["comparators"]:
                    e = run_ladder(torch, np, [(key, scene, {"storage": dt}, {})], base_b,
                                   dict(mode="vlm", level_dist=level_dist, grade=args.grade), dirs, probes[k], d, ref,
                                   nb_lam)
                    out["comparators"][key]["error_vs_fp64_classic"] = e[key]
        if args.ladder:
            out["accuracy_ladder"] = accuracy_ladder(args, rt, torch, np, sc, scene, dirs, probes[k], d, ref, nb_lam,
                                                     level_dist)
    print(json.dumps(out), flush=True)


def accuracy_ladder(args, rt, torch, np, sc, scene, dirs, probe_vox, d, ref, nb_lam, level_dist):
    """cfg2: error against the FP64 oracle of other settings on the same sampled rays."""
    base = dict(iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin, iod_frame=args.iod_frame,
                storage=args.storage)
    scene81 = rt.Scene.from_dict(sc, emission=args.emission, n_v=81)
    ld4 = [v * 4 for v in rt.CASCADE_LEVEL_DIST]
    settings = [("as benchmarked", scene, {}, {}),
                ("sparse MIP 0 (no merging)", scene, {}, {"mode": "level0"}),
                ("levels <= 1", scene, {}, {"max_level": 1}),
                ("levels <= 2", scene, {}, {"max_level": 2}),
                ("plain VLM (no distance grading)", scene, {}, {"level_dist": None}),
                ("no thin bypass", scene, {"tau_thin": 0.0}, {}),
                ("core-closest level test", scene, {"iod_frame": "core"}, {}),
                ("core-closest level test, T=1e-3", scene, {"iod_frame": "core", "iod_threshold": 1e-3}, {}),
                ("n_v=81", scene81, {}, {}),
                ("n_v=81, sparse MIP 0", scene81, {}, {"mode": "level0"}),
                ("n_v=81, levels <= 1", scene81, {}, {"max_level": 1}),
                ("n_v=81, levels <= 2", scene81, {}, {"max_level": 2}),
                ("n_v=81, grading x4", scene81, {}, {"level_dist": ld4}),
                ("n_v=81, core-closest, levels <= 2", scene81, {"iod_frame": "core"}, {"max_level": 2}),
                ("n_v=81, core-closest, grading x4", scene81, {"iod_frame": "core"}, {"level_dist": ld4})]
    return run_ladder(torch, np, settings, base, dict(mode="vlm", level_dist=level_dist, grade=args.grade), dirs,
                      probe_vox, d, ref,
                      nb_lam)


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
def bench_cfg3(args):
    """3D 256^3 Core-and-Voigt scene, storage FP32 / BF16 / FP16: time per full solve (16 batches),
    march-kernel roofline, error of each dtype against the FP64 dense Classic oracle."""
    np, torch, rt, dev = _env()
    from synth import make_cfg3
    tg = time.time()
    sc = make_cfg3()
    log("cfg3 scene generated in %.1fs (%d active bricks)" % (time.time() - tg, int(sc["block_active"].sum())))
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
    nthreads = min(os.cpu_count() or 1, 16)
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
    out_line = {"workload": "cfg3", "accuracy_ladder": ladder, "config": {
        "workload": "3D 256^3, 8^3 bricks, %d active (25%%), slab + %d loops, 2 Voigt lines (Core and Voigt) + "
                    "grey continuum, |v| <= 30 km/s, 4-level VLM T=%g, %s, 32 Fibonacci directions, %d lambda "
                    "(%d batches of 8), all %d probes" % (
                        int(sc["block_active"].sum()), int(sc["n_loops"]), args.iod,
                        _grading(args), nb * 8, nb, n_probes)},
        "seg_lam_per_solve": seglam, "dense_seg_lam_per_solve": dense_seglam,
        "dense_classic_gpu": {"ms_per_batch": dense_ms_batch, "ms_per_solve_extrapolated": dense_ms_batch * nb},
        "cpu_baseline": {"value": cpu_seglam / cpu_s / 1e9, "unit": "Gsegments/s", "cores": nthreads,
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
    if "f32" in res:
        for dt in res:
            if dt != "f32":
                out_line["dtypes"][dt]["speedup_vs_f32"] = res["f32"]["ms_per_solve"] / res[dt]["ms_per_solve"]
                out_line["dtypes"][dt]["error_vs_gpu_f32"] = _err(res[dt]["got"], res["f32"]["got"].astype(np.float64))
    print(json.dumps(out_line), flush=True)


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
    # held-out check -> fallback map
    fb = torch.zeros(scene.info["n_blocks"], dtype=torch.uint8, device=dev)
    held_err = []
    for b in range(nb):
        scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin, storage="bf16")
        tr = scene.trace_truncated(dirs, T_TRUNC, gen=True, probes=hd_probes[b], level_dist=level_dist,
                                   grade=args.grade)
        _, err = nn.validate(scene, tr, THRESH, fb)
        q = (tr["feat"][..., 3] > 0)[:, None, :].expand_as(err)
        held_err.append(err[q].cpu().numpy())
    torch.cuda.synchronize()
    held_err = np.concatenate(held_err) if held_err else np.zeros(1)
    n_flag = int(fb.sum().item())
    log("cfg5 held-out: median %.3e p99.9 %.3e; %d blocks flagged" % (
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

    def cached(gather=None, gather_cut=None, fallback=fb, record=False):
        qsum = 0
        for b in range(nb):
            scene.build(8 * b, 8 * b + 8, iod_threshold=args.iod, avg_mode=args.avg, tau_thin=args.tau_thin, storage="bf16")
            if record:
                e0, e1 = _events(torch)
                e0.record(stream)
            tr = scene.trace_truncated(dirs, T_TRUNC, gen=False, fallback=fallback, level_dist=level_dist,
                                       grade=args.grade)
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
    nthreads = min(os.cpu_count() or 1, 16)
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
        "fallback_blocks": n_flag, "fallback_block_frac": n_flag / int(sc["block_active"].sum()),
        "query_ray_frac": queries / (rays * nb), "query_ray_frac_without_fallback": queries0 / (rays * nb),
        "error_vs_fp64_classic": {"plain_f32": _err(f32_np, ref), "plain_bf16": _err(g_bf16.cpu().numpy(), ref),
                                  "cache": _err(g_nrc.cpu().numpy(), ref),
                                  "truncated_no_cache": _err(g_cut.cpu().numpy(), ref),
                                  "cache_without_fallback": _err(g_nrc0.cpu().numpy(), ref),
                                  "truncated_no_cache_no_fallback": _err(g_cut0.cpu().numpy(), ref)},
        "error_vs_gpu_plain_f32": {"plain_bf16": _err(g_bf16.cpu().numpy(), f32_np),
                                   "cache": _err(g_nrc.cpu().numpy(), f32_np),
                                   "truncated_no_cache": _err(g_cut.cpu().numpy(), f32_np)},
        "cpu_baseline": {"value": cpu_seglam / cpu_s / 1e9, "unit": "Gsegments/s", "cores": nthreads,
                         "kind": "oracle", "sample": "%d pairs x %d wavelengths, FP64 dense Classic, %.1f s" % (
                             kk_np.size, nb * 8, cpu_s)}}
    print(json.dumps(out_line), flush=True)


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
    nthreads = min(os.cpu_count() or 1, 16)
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
        "cpu_baseline": {"value": cpu_seglam / cpu_s / 1e9, "unit": "Gsegments/s", "cores": nthreads,
                         "kind": "oracle", "sample": "%d pairs x %d wavelengths, FP64 dense Classic, %.1f s" % (
                             k.size, nb * 8, cpu_s)}}
    print(json.dumps(line), flush=True)

if __name__ == "__main__":
    main()
