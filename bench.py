"""Benchmark of the 2D-LUT hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--rows all|none|c1,c3,c4,c5,g1,g4,sweep,dims,u1,p1]

Headline (`value`): svdlut_apply on one 3840x2160 float32 frame (33x33 LUTs at rank 8,
reconstruction fused, 480x270 spatial map), in Mpix/s, inputs resident in HBM.  Each timed
step is one launch; four disjoint buffer sets rotate so that the 256 MB Infinity Cache
cannot serve a step from the previous one.  `roofline.achieved` is the algorithmic bytes of
one launch over the back-to-back step time.  The other hot-path rows are timed in the same
run, before the headline, and reported under "rows".  Prints ONE JSON line.

    python bench.py --summarize-trace DIR --steps K --warmup W --command "..."
    python bench.py --summarize-traffic FETCH_DIR WRITE_DIR --command "cmd1 ;; cmd2"

turn rocprofv3 CSV output of `bench.py --rows none` runs into the summaries under profiles/
that the bench line cites (no GPU needed).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
N_ROT = 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 500 warm-up launches (about 30 ms at 4K): the first ~300 launches after the GPU has been
    # idle run up to 15 % slower while its clocks ramp to the sustained-load state
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--rows", default="all", help="extra rows to time: all, none, or a list of c1,c3,c4,c5,g1,g4,sweep,dims,u1,p1")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the oracle CPU baseline (0: skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run device-to-device copies of one 4K fp32 frame (99.5 MB), the reference "
                         "kernel that calibrates HBM byte counters in a profiler run")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="no GPU: summarise a rocprofv3 --kernel-trace CSV run of `bench.py --rows none` "
                         "(same --steps/--warmup) into profiles/apply_4k_fp32_kernel_trace.json")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU: summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "`bench.py --rows none --copy-probe` into profiles/apply_4k_fp32_traffic.json")
    ap.add_argument("--summarize-mfma", nargs=2, metavar=("TRACE_DIR", "PMC_DIR"),
                    help="no GPU: MFMA utilisation of the generator GEMMs from a --kernel-trace run and a --pmc "
                         "run of `bench.py --rows c5` into profiles/generator_mfma_counters.json")
    ap.add_argument("--command", default="", help="the profiler command recorded in a summary")
    return ap.parse_args()


def event_time(fn, steps, warmup, torch):
    """Average ms per call of fn(i) over `steps` calls, timed with HIP events on the current stream."""
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        fn(i)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


KERNEL_SOURCES = ("paper_2508_16121_amd/csrc/lut_fwd.hip", "paper_2508_16121_amd/csrc/lut_common.h",
                  "paper_2508_16121_amd/csrc/internal.h", "paper_2508_16121_amd/csrc/api.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_4k_fp32_traffic.json")


def kernel_hash(sources=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


GEN_SOURCES = ("paper_2508_16121_amd/csrc/gen_common.h", "paper_2508_16121_amd/csrc/gen.hip")
MFMA_FILE = os.path.join(ROOT, "profiles", "generator_mfma_counters.json")
GEMM_KERNEL = "mfma_gemm_kernel"
# MFMA ops counters count in units of 512 flops (v_mfma_f32_16x16x32_bf16: 16384 flops = 32)
MOPS_FLOPS = 512


def mfma_counters():
    """Counter-based MFMA figures of the generator's GEMM kernels from the committed summary
    (or None when the generator sources changed since it was taken)."""
    try:
        with open(MFMA_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash(GEN_SOURCES):
        return None
    return {k: t[k] for k in ("gemm_tflops", "gemm_frac_of_bf16_peak", "mfma_busy_frac", "gemm_time_share")} | \
        {"source": os.path.relpath(MFMA_FILE, ROOT)}


TRACE_FILE = os.path.join(ROOT, "profiles", "apply_4k_fp32_kernel_trace.json")
HEADLINE_KERNEL = "apply_kernel<float, float, true, false, false, 4>"


def _current_summary(path):
    """A committed profile summary, or None when the kernel sources changed since it was taken."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    return t if t.get("kernel_hash") == kernel_hash() else None


def measured_traffic():
    """HBM bytes per launch of the 4K apply from the committed counter summary (or None)."""
    t = _current_summary(TRAFFIC_FILE)
    return t.get("bytes_per_launch") if t else None


def profiled_launch():
    """Mean duration of the timed 4K launches under rocprofv3 from the committed trace summary
    (or None)."""
    t = _current_summary(TRACE_FILE)
    if not t:
        return None
    return {"avg_ms": round(t["timed_avg_ns"] * 1e-6, 5), "source": os.path.relpath(TRACE_FILE, ROOT)}


def _csvs(d, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _kernel_rows(rows, name):
    """Dispatches of the headline kernel variant, in start order (one row per dispatch)."""
    sel = {}
    for r in rows:
        if name in r["Kernel_Name"]:
            sel.setdefault(int(r.get("Dispatch_Id", r.get("Correlation_Id", 0))), r)
    return [sel[k] for k in sorted(sel, key=lambda k: int(sel[k]["Start_Timestamp"]))]


def summarize_trace(args):
    rows = _kernel_rows(_csvs(args.summarize_trace, "kernel_trace.csv"), HEADLINE_KERNEL)
    dur = np.array([int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows], dtype=np.float64)
    # launch order of `bench.py --rows none`: warm-up, the back-to-back timed run, then the
    # event-pair run of the same number of launches
    w, k = args.warmup, args.steps
    if len(dur) < w + 2 * k:
        raise SystemExit(f"expected {w + 2 * k} dispatches of {HEADLINE_KERNEL}, found {len(dur)}")
    timed = dur[w:w + k]
    out = {"kernel": HEADLINE_KERNEL + " (svdlut_apply, 1x3x2160x3840 fp32, D=33 R=8, map 9x270x480 fp32)",
           "kernel_hash": kernel_hash(), "kernel_hash_sources": list(KERNEL_SOURCES),
           "dispatches": int(len(dur)), "warmup": w, "steps": k,
           "timed_avg_ns": round(float(timed.mean()), 1), "timed_median_ns": float(np.median(timed)),
           "timed_min_ns": float(timed.min()), "timed_max_ns": float(timed.max()),
           "all_avg_ns": round(float(dur.mean()), 1), "command": args.command}
    with open(TRACE_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def summarize_traffic(args):
    def per_dispatch(d, counter):
        rows = _csvs(d, "counter_collection.csv")
        acc = {}
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            key = (r["Kernel_Name"], int(r["Dispatch_Id"]))
            acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
        heads = {i: x for (n, i), x in acc.items() if HEADLINE_KERNEL in n}
        # the probe's device-to-device copies run after the last headline launch (the copies
        # before it upload the inputs from the host)
        last = max(heads)
        probe = [x for (n, i), x in acc.items() if "copyBuffer" in n and i > last]
        return float(np.mean(list(heads.values()))), float(np.mean(probe))
    fa, fc = per_dispatch(args.summarize_traffic[0], "FETCH_SIZE")
    wa, wc = per_dispatch(args.summarize_traffic[1], "WRITE_SIZE")
    frame = 2160 * 3840 * 3 * 4
    fs, ws = frame / 1024.0 / fc, frame / 1024.0 / wc
    rd, wr = int(fa * 1024 * fs), int(wa * 1024 * ws)
    out = {"kernel": HEADLINE_KERNEL + " (svdlut_apply, 1x3x2160x3840 fp32, D=33 R=8, map 9x270x480 fp32)",
           "kernel_hash": kernel_hash(), "kernel_hash_sources": list(KERNEL_SOURCES),
           "fetch_size_kib_per_dispatch": round(fa, 2), "write_size_kib_per_dispatch": round(wa, 2),
           "copy_probe": {"bytes_read": frame, "bytes_written": frame, "fetch_size_kib": round(fc, 2),
                          "write_size_kib": round(wc, 2)},
           "fetch_scale": round(fs, 5), "write_scale": round(ws, 5),
           "bytes_read_per_launch": rd, "bytes_written_per_launch": wr, "bytes_per_launch": rd + wr,
           "algorithmic_bytes_per_launch": HEADLINE_BYTES, "commands": args.command.split(" ;; ")}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def summarize_mfma(args):
    """MFMA utilisation of the generator GEMMs from a --kernel-trace run and a --pmc run
    (SQ_INSTS_VALU_MFMA_MOPS_BF16, SQ_VALU_MFMA_BUSY_CYCLES, SQ_BUSY_CU_CYCLES) of
    `bench.py --rows c5`."""
    trace_dir, pmc_dir = args.summarize_mfma
    stats = _csvs(trace_dir, "kernel_stats.csv")
    t_all = sum(float(r["TotalDurationNs"]) for r in stats)
    g = [r for r in stats if GEMM_KERNEL in r["Name"]]
    t_gemm = sum(float(r["TotalDurationNs"]) for r in g)
    calls = sum(int(r["Calls"]) for r in g)
    tot = {}
    for r in _csvs(pmc_dir, "counter_collection.csv"):
        if GEMM_KERNEL in r["Kernel_Name"]:
            tot[r["Counter_Name"]] = tot.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    flops = tot["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * MOPS_FLOPS
    tflops = flops / (t_gemm * 1e-9) / 1e12
    out = {"kernel": GEMM_KERNEL, "kernel_hash": kernel_hash(GEN_SOURCES), "kernel_hash_sources": list(GEN_SOURCES),
           "dispatches": calls, "gemm_time_ns": t_gemm, "gemm_time_share": round(t_gemm / t_all, 4),
           "counters": {k: v for k, v in sorted(tot.items())}, "mfma_flops": flops,
           "gemm_tflops": round(tflops, 3), "gemm_frac_of_bf16_peak": round(tflops / BF16_PEAK_TFLOPS, 5),
           "mfma_busy_frac": round(tot["SQ_VALU_MFMA_BUSY_CYCLES"] / tot["SQ_BUSY_CU_CYCLES"], 5),
           "commands": args.command.split(" ;; ")}
    with open(MFMA_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


HEADLINE_BYTES = 2160 * 3840 * 24 + 9 * 270 * 480 * 4 + 9 * 33 * 8 * 2 * 4 + 9 * 8 * 4


def launch_times(fn, steps, warmup, torch):
    """(ms per step, ms per event pair) over `steps` calls of a one-kernel fn(i), both with HIP
    events on the current stream (the stream the library launches on).  The first figure
    brackets the whole run of `steps` back-to-back calls and is the one every rate is computed
    from.  The second comes from a separate run in which every launch has its own event pair;
    the event packets add their own time (about 2 us per launch on this part), so it is an
    upper bound of the launch duration, reported only for reference."""
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        fn(i)
    e1.record()
    torch.cuda.synchronize()
    per_step = e0.elapsed_time(e1) / steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    for i in range(steps):
        ev[2 * i].record()
        fn(i)
        ev[2 * i + 1].record()
    torch.cuda.synchronize()
    per = sum(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(steps)) / steps
    return per_step, per


def roof(bytes_alg, ms):
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


_BAND = {}   # frame, LUTs and map shared with forked workers (copy-on-write)


def _oracle_band(rows_):
    """Worker: the oracle on rows [y0, y1) of the frame in _BAND."""
    from oracle import lut as ol
    y0, y1 = rows_
    x, T, m, W = _BAND["x"], _BAND["T"], _BAND["m"], _BAND["W"]
    ys = np.repeat(np.arange(y0, y1), W)
    xs = np.tile(np.arange(W), y1 - y0)
    ol.transform_at(x, T, m, ys, xs)
    return (y1 - y0) * W


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


# worker processes of the CPU baseline: every core of the affinity mask, but no more than the
# 16 cores a one-GPU machine grants a job (more processes would only time-slice the same cores)
CPU_SHARE = 16


def cpu_baseline(case, budget_s, c1):
    """The fp64 oracle on the same 4K frame, timed on the host: one process on row bands until
    about budget_s of work, and the same rows as bands over a process pool on every usable
    core, median of three runs; plus the oracle on the whole 256x256 frame of the plain config
    (median of three single-process runs).  Runs before the GPU is touched (the pool forks)."""
    import multiprocessing as mp
    from oracle import lut as ol
    x, U, s, V, m = case.x[0], case.U[0], case.s[0], case.V[0], case.smap[0]
    H, W = x.shape[1:]
    T = ol.reconstruct(U, s, V)
    _BAND.update(x=x, T=T, m=m, W=W)
    band = 64
    px, t_total, rows, y0 = 0, 0.0, 0, 0
    while t_total < budget_s and y0 < H:
        t = time.perf_counter()
        px += _oracle_band((y0, min(y0 + band, H)))
        t_total += time.perf_counter() - t
        rows += min(band, H - y0)
        y0 += band
    single = px / t_total / 1e6
    avail = len(os.sched_getaffinity(0))
    cores = max(1, min(CPU_SHARE, avail))
    # all cores: the rows the single-process run covered, split into bands over a fork pool
    jobs = [(r, min(r + band, rows)) for r in range(0, rows, band)]
    runs = []
    with mp.get_context("fork").Pool(cores) as pool:
        for _ in range(3):
            t = time.perf_counter()
            npx = sum(pool.map(_oracle_band, jobs, chunksize=1))
            runs.append(npx / (time.perf_counter() - t) / 1e6)
    multi = float(np.median(runs))
    # C1: the plain 256x256 frame, whole frame, one process (the full oracle: reconstruct + apply)
    c1_runs = []
    for _ in range(3):
        t = time.perf_counter()
        ol.apply(c1.x, c1.U, c1.s, c1.V, c1.smap)
        c1_runs.append(time.perf_counter() - t)
    c1_ms = float(np.median(c1_runs)) * 1e3
    model = _cpu_model()
    return {"value": round(multi, 3), "unit": "Mpix/s", "cores": cores, "kind": "oracle",
            "single_core_value": round(single, 3),
            "sample": f"{rows} of {H} rows of the {W}x{H} frame (fp64 NumPy oracle): one process "
                      f"{t_total:.1f} s; {cores} processes on 64-row bands ({avail} cores in the affinity "
                      f"mask), median of 3; {model}",
            "c1": {"workload": "oracle apply (reconstruct + transform), whole 256x256 frame, D=17 R=4, map 9x32x32",
                   "ms": round(c1_ms, 2), "mpix_s": round(256 * 256 / (c1_ms * 1e-3) / 1e6, 3), "cores": 1}}


def row_g1(svd, torch, synth, args):
    """4K frame with the paper's fused slicing: K = 6 bilateral grids of 3 planes, 17x17."""
    c, gr, gw, gb = synth.grid_case(43, 2160, 3840, 33, 8, 270, 480)
    sets = []
    for k in range(N_ROT):
        sets.append([torch.from_numpy(a).cuda() for a in (c.x, c.U, c.s, c.V, c.smap, gr, gw, gb)]
                    + [torch.empty_like(torch.from_numpy(c.x)).cuda()])
    torch.cuda.synchronize()

    def step(i):
        b = sets[i % N_ROT]
        svd.apply_grid(*b[:8], out=b[8])

    ms, ms_kernel = launch_times(step, args.steps, args.warmup, torch)
    npx = 2160 * 3840
    bytes_alg = npx * 24 + 9 * 270 * 480 * 4 + 9 * 33 * 8 * 2 * 4 + 9 * 8 * 4 + gr.nbytes + gw.nbytes + gb.nbytes
    return {"workload": "svdlut_apply_grid 1x3x2160x3840 fp32, D=33 R=8, map 9x270x480, K=6 grids x 3 planes 17x17",
            "ms": round(ms, 5), "event_pair_ms": round(ms_kernel, 5), "mpix_s": round(npx / (ms * 1e-3) / 1e6, 1),
            "roofline": roof(bytes_alg, ms)}


def row_u1(svd, torch, synth, args):
    """The paper's unfused original structure at 4K (slicing -> f_s -> 1x1 fusion -> 3D LUT, K = 6
    grids of 17x17, 33^3 3D LUTs) against the fused pass (svdlut_apply_grid) on the same frame."""
    c, gr, gw, gb = synth.grid_case(43, 2160, 3840, 33, 8, 270, 480)
    g = np.random.default_rng(49)
    K, D3 = 6, 33
    Wf = np.concatenate([np.eye(3, dtype=np.float32)[None], g.normal(0, 0.1, (1, 3, K)).astype(np.float32)], axis=2)
    bf = g.normal(0, 0.01, (1, 3)).astype(np.float32)
    T3 = g.normal(0.5, 0.1, (1, 3, D3, D3, D3)).astype(np.float32)
    sets = []
    for k in range(N_ROT):
        t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (c.x, gr, gw, gb, Wf, bf, T3)]
        ws = torch.empty(svd._lib.load().svdlut_unfused_workspace_size(1, 2160, 3840, K, D3) // 4 + 64, device="cuda")
        sets.append((t, ws, torch.empty_like(t[0])))
    torch.cuda.synchronize()

    def step(i):
        t, ws, y = sets[i % N_ROT]
        svd.unfused_apply(*t, out=y, ws=ws)

    steps = max(10, args.steps // 4)
    ms = event_time(step, steps, 3, torch)
    npx = 2160 * 3840
    per_px = 12 + 4 * K + (12 + 4 * K + 12) + (12 + 12)   # slicing, fusion, 3D LUT passes (B/px)
    return {"workload": "unfused original structure 1x3x2160x3840 fp32: slicing (K=6 grids 17x17) -> f_s -> "
                        "1x1 fusion -> 33^3 3D LUT, 4 kernels",
            "ms": round(ms, 4), "mpix_s": round(npx / (ms * 1e-3) / 1e6, 1), "bytes_per_px": per_px,
            "roofline": roof(npx * per_px, ms)}


def row_c1(svd, torch, synth, args):
    c = synth.plain_256()
    d = [torch.from_numpy(a).cuda() for a in (c.x, c.U, c.s, c.V, c.smap)]
    y = torch.empty_like(d[0])
    ms = event_time(lambda i: svd.apply(*d, out=y), args.steps, args.warmup, torch)
    # the same launches replayed from one HIP graph (20 applies per replay): the per-frame time
    # without the host-side call overhead that bounds the eager loop at this size
    n_in_graph = 20
    svd.apply(*d, out=y)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(n_in_graph):
            svd.apply(*d, out=y)
    ms_graph = event_time(lambda i: graph.replay(), max(5, args.steps // 10), 2, torch) / n_in_graph
    return {"workload": "svdlut_apply 1x3x256x256 fp32, D=17 R=4, map 9x32x32", "ms": round(ms, 5),
            "mpix_s": round(256 * 256 / (ms * 1e-3) / 1e6, 1), "graph_ms_per_frame": round(ms_graph, 5),
            "graph_mpix_s": round(256 * 256 / (ms_graph * 1e-3) / 1e6, 1)}


def row_c3(svd, torch, synth, args):
    images = synth.uneven_batch(64, workers=16)
    xf, mf, U, s, V, descs = synth.pack_uneven(images)
    del images
    npx = sum(d["H"] * d["W"] for d in descs)
    x = torch.from_numpy(xf).cuda().half()
    m = torch.from_numpy(mf).cuda().half()
    del xf, mf
    y = torch.empty_like(x)
    Ud, sd, Vd = (torch.from_numpy(a).cuda() for a in (U, s, V))
    plan = svd.Plan(descs, 33, 8, torch.float16, torch.float16)
    plan.autotune(x, y, Ud, sd, Vd, m)
    steps = max(5, args.steps // 10)
    ms = event_time(lambda i: plan.launch(x, y, Ud, sd, Vd, m), steps, 2, torch)
    views = []
    for b, d in enumerate(descs):
        H, W, h, w = d["H"], d["W"], d["h"], d["w"]
        views.append((x[d["x_off"]:d["x_off"] + 3 * H * W].view(1, 3, H, W), Ud[b:b + 1], sd[b:b + 1], Vd[b:b + 1],
                      m[d["map_off"]:d["map_off"] + 9 * h * w].view(1, 9, h, w),
                      y[d["y_off"]:d["y_off"] + 3 * H * W].view(1, 3, H, W)))

    def loop(i):
        for xv, u, ss, v, mv, yv in views:
            svd.apply(xv, u, ss, v, mv, out=yv)

    ms_loop = event_time(loop, steps, 2, torch)
    bytes_alg = npx * 12 + sum(9 * d["h"] * d["w"] * 2 for d in descs) + 64 * 9 * (2 * 33 * 8 + 8) * 4
    info = plan.info()
    return {"workload": f"64 uneven images ({npx / 1e6:.1f} Mpx; 480x640/1080x1920/2160x3840 bases, +-10% width), "
                        "fp16 storage, D=33 R=8, 1/8 maps, one graph-replayed persistent launch",
            "ms": round(ms, 4), "mpix_s": round(npx / (ms * 1e-3) / 1e6, 1), "roofline": roof(bytes_alg, ms),
            "loop_of_64_apply_ms": round(ms_loop, 4), "speedup_vs_loop": round(ms_loop / ms, 3),
            "plan": {k: info[k] for k in ("block", "grid", "blocks_per_cu", "tile_px", "px_per_lane", "tuned", "graph")}}


def row_c4(svd, torch, synth, args):
    c = synth.diff_batch()
    B, H, W = c.x.shape[0], c.x.shape[2], c.x.shape[3]
    npx = B * H * W
    sets = []
    for k in range(N_ROT):
        d = {a: torch.from_numpy(getattr(c, a)).cuda() for a in ("x", "U", "s", "V", "smap", "target")}
        d["y"] = torch.empty_like(d["x"])
        d["ws"] = svd.bwd_workspace(B, 33, "cuda")
        sets.append(d)

    def fwd(i):
        d = sets[i % N_ROT]
        svd.apply(d["x"], d["U"], d["s"], d["V"], d["smap"], out=d["y"])

    def fwd_bwd(i):
        d = sets[i % N_ROT]
        svd.apply(d["x"], d["U"], d["s"], d["V"], d["smap"], out=d["y"])
        _, dy = svd.loss(d["y"], d["target"], "l1")
        svd.apply_bwd(d["x"], dy, d["U"], d["s"], d["V"], d["smap"], ws=d["ws"])

    for d in sets:
        d["lws"] = svd.loss_bwd_workspace(B, 33, "cuda")

    def fused(i):
        d = sets[i % N_ROT]
        svd.apply_loss_bwd(d["x"], d["target"], d["U"], d["s"], d["V"], d["smap"], kind="l1", ws=d["lws"])

    steps = max(5, args.steps // 4)
    ms_f = event_time(fwd, steps, 3, torch)
    ms_fb = event_time(fwd_bwd, steps, 3, torch)
    ms_fused = event_time(fused, steps, 3, torch)
    # the same three passes in deterministic mode (dmap and dbias from per-workgroup partials)
    was = svd.deterministic()
    svd.deterministic(True)
    try:
        for d in sets:
            d["dws"] = svd.bwd_workspace(B, 33, "cuda", (H, W, c.smap.shape[2], c.smap.shape[3]))

        def fwd_bwd_det(i):
            d = sets[i % N_ROT]
            svd.apply(d["x"], d["U"], d["s"], d["V"], d["smap"], out=d["y"])
            _, dy = svd.loss(d["y"], d["target"], "l1")
            svd.apply_bwd(d["x"], dy, d["U"], d["s"], d["V"], d["smap"], ws=d["dws"])

        ms_fb_det = event_time(fwd_bwd_det, steps, 3, torch)
    finally:
        svd.deterministic(was)
    # algorithmic bytes: forward 24.56 B/px; loss 24 B/px (y, target read, dy written);
    # backward x 12 + dy 12 + dx 12 B/px plus the map and its gradient
    mapb = B * 9 * 64 * 64 * 4
    b_fwd = npx * 24 + mapb
    b_fb = b_fwd + npx * 36 + npx * 36 + 2 * mapb
    return {"workload": "16x3x512x512 fp32, D=33 R=8, map 9x64x64: apply + L1 loss + apply_bwd (dU ds dV dmap dx)",
            "fwd_ms": round(ms_f, 4), "fwd_bwd_ms": round(ms_fb, 4),
            "fwd_mpix_s": round(npx / (ms_f * 1e-3) / 1e6, 1), "fwd_bwd_mpix_s": round(npx / (ms_fb * 1e-3) / 1e6, 1),
            "fwd_roofline": roof(b_fwd, ms_f), "fwd_bwd_roofline": roof(b_fb, ms_fb),
            "fwd_bwd_deterministic_ms": round(ms_fb_det, 4),
            # the same step as one fused pass (svdlut_apply_loss_bwd): x, target in; dx out
            "fused_loss_bwd_ms": round(ms_fused, 4), "fused_mpix_s": round(npx / (ms_fused * 1e-3) / 1e6, 1),
            "fused_roofline": roof(npx * 36 + 2 * mapb, ms_fused)}


def row_g4(svd, torch, synth, args):
    """C4's differentiation batch with K = 6 bilateral grids of 17x17: forward + L1 + full backward."""
    c = synth.diff_batch()
    B, H, W = c.x.shape[0], c.x.shape[2], c.x.shape[3]
    npx = B * H * W
    gr, gw, gb = synth.grids(np.random.default_rng(47), B, 6, 17)
    sets = []
    for k in range(N_ROT):
        d = {a: torch.from_numpy(getattr(c, a)).cuda() for a in ("x", "U", "s", "V", "smap", "target")}
        d.update(gr=torch.from_numpy(gr).cuda(), gw=torch.from_numpy(gw).cuda(), gb=torch.from_numpy(gb).cuda())
        d["y"] = torch.empty_like(d["x"])
        d["ws"] = svd.grid_bwd_workspace(B, 33, 17, "cuda")
        sets.append(d)

    def fwd_bwd(i):
        d = sets[i % N_ROT]
        svd.apply_grid(d["x"], d["U"], d["s"], d["V"], d["smap"], d["gr"], d["gw"], d["gb"], out=d["y"])
        _, dy = svd.loss(d["y"], d["target"], "l1")
        svd.apply_grid_bwd(d["x"], dy, d["U"], d["s"], d["V"], d["smap"], d["gr"], d["gw"], ws=d["ws"])

    steps = max(5, args.steps // 4)
    ms_fb = event_time(fwd_bwd, steps, 3, torch)
    mapb = B * 9 * 64 * 64 * 4
    b_fb = npx * 24 + mapb + npx * 36 + npx * 36 + 2 * mapb + npx * 24   # + the grid pass's dx read/write
    return {"workload": "16x3x512x512 fp32, D=33 R=8, map 9x64x64, K=6 grids 17x17: apply_grid + L1 loss + "
                        "apply_grid_bwd (dU ds dV dmap dx dgrids dgw dgb)",
            "fwd_bwd_ms": round(ms_fb, 4), "fwd_bwd_mpix_s": round(npx / (ms_fb * 1e-3) / 1e6, 1),
            "fwd_bwd_roofline": roof(b_fb, ms_fb)}


def row_sweep(svd, torch, synth, args):
    """4K fp32 apply throughput across LUT sizes D in {17, 33} and ranks R in {1, 4, 8, 16}, and the
    rank-R truncation error of a dense LUT of the same size (Eckart-Young: the Frobenius error
    equals the norm of the dropped singular values)."""
    g = np.random.default_rng(48)
    xh = synth.image(g, 2160, 3840)[None]
    mh = synth.spatial_map(g, 1, 270, 480)
    # four disjoint buffer sets, as for the headline, so the 256 MB cache does not hold the frame
    bufs = [(torch.from_numpy(xh).cuda(), torch.from_numpy(mh).cuda(), torch.empty(1, 3, 2160, 3840, device="cuda"))
            for _ in range(N_ROT)]
    out = {}
    for D in (17, 33):
        A = g.uniform(-1, 1, (D, D))
        sig = np.linalg.svd(A, compute_uv=False)
        for R in (1, 4, 8, 16):
            U, s, V = (torch.from_numpy(a).cuda() for a in synth.factors(g, 1, D, R))

            def step(i):
                x, m, y = bufs[i % N_ROT]
                svd.apply(x, U, s, V, m, out=y)
            ms = event_time(step, max(10, args.steps // 4), 3, torch)
            out[f"D{D}_R{R}"] = {"ms": round(ms, 4), "mpix_s": round(2160 * 3840 / (ms * 1e-3) / 1e6, 1),
                                 "rel_frobenius_error": round(float(np.sqrt((sig[R:] ** 2).sum() / (sig ** 2).sum())), 5)}
    return {"workload": "svdlut_apply 1x3x2160x3840 fp32, map 9x270x480; D x R sweep", "points": out}


def row_dims(svd, torch, synth, args):
    """LUT dimension at the same 4K fp32 frame (D = 33): per-channel 1D LUTs, the 2D
    decomposition (R = 8) with scalar LUT weights (1x1 map) and with the 9x270x480 spatial map,
    and a dense 3D LUT.  Four rotating buffer sets, event timing."""
    g = np.random.default_rng(49)
    D, R, H, W = 33, 8, 2160, 3840
    xh = synth.image(g, H, W)[None]
    bufs = [(torch.from_numpy(xh).cuda(), torch.empty(1, 3, H, W, device="cuda")) for _ in range(N_ROT)]
    T1 = torch.from_numpy(g.normal(0, 1, (1, 3, D)).astype(np.float32)).cuda()
    T3 = torch.from_numpy(g.normal(0, 0.3, (1, 3, D, D, D)).astype(np.float32)).cuda()
    ws3 = torch.empty(svd._lib.load().svdlut_lut3d_workspace_size(1, D) // 4 + 64, device="cuda")
    U, s, V = (torch.from_numpy(a).cuda() for a in synth.factors(g, 1, D, R))
    m1 = torch.from_numpy(synth.spatial_map(g, 1, 1, 1)).cuda()
    mm = torch.from_numpy(synth.spatial_map(g, 1, 270, 480)).cuda()
    steps = max(10, args.steps // 4)
    cases = {
        "lut1d": (lambda i: svd.lut1d_apply(bufs[i % N_ROT][0], T1, out=bufs[i % N_ROT][1]), 3 * D),
        "lut2d_svd_scalar_weights": (lambda i: svd.apply(bufs[i % N_ROT][0], U, s, V, m1, out=bufs[i % N_ROT][1]),
                                     9 * (2 * D * R + R) + 9),
        "lut2d_svd_map": (lambda i: svd.apply(bufs[i % N_ROT][0], U, s, V, mm, out=bufs[i % N_ROT][1]),
                          9 * (2 * D * R + R)),
        "lut3d": (lambda i: svd.lut3d_apply(bufs[i % N_ROT][0], T3, out=bufs[i % N_ROT][1], ws=ws3), 3 * D ** 3),
    }
    out = {}
    for k, (fn, npar) in cases.items():
        ms = event_time(fn, steps, 3, torch)
        out[k] = {"ms": round(ms, 4), "mpix_s": round(H * W / (ms * 1e-3) / 1e6, 1), "lut_params": npar,
                  "gb_s_at_24_b_px": round(24 * H * W / (ms * 1e-3) / 1e9, 1)}
    return {"workload": "1x3x2160x3840 fp32, D=33: 1D LUTs vs 2D SVD (R=8) vs dense 3D LUT", "points": out}


def row_c5(svd, torch, synth, args):
    from paper_2508_16121_amd import generator as G
    g = np.random.default_rng(5)
    x8 = torch.from_numpy(np.concatenate([synth.image(g, 2160, 3840)[None]] * 8)).cuda()
    gen = G.Generator(33, 8, seed=0)
    y = torch.empty_like(x8)

    def infer(i):
        U, s, V, m = gen.forward(x8)
        svd.apply(x8, U, s, V, m, out=y)

    steps = max(5, args.steps // 10)
    ms_inf = event_time(infer, steps, 2, torch)
    ms_gen = event_time(lambda i: gen.forward(x8), steps, 2, torch)
    xb = torch.rand(16, 3, 256, 256, device="cuda")
    tb = torch.rand(16, 3, 256, 256, device="cuda")
    tr = G.Trainer(G.Generator(33, 8, seed=1), lr=1e-4)
    ms_train = event_time(lambda i: tr.step(xb, tb), max(10, args.steps // 2), 3, torch)
    macs = 0
    ch = (3, 16, 32, 64, 128, 128)
    for i in range(5):
        hw = 256 >> (i + 1)
        macs += hw * hw * ch[i + 1] * 9 * ch[i]
    macs += 32 * 32 * 9 * 9 * 64 + 128 * 9 * (2 * 33 * 8 + 8)
    tflops = 8 * 2 * macs / (ms_gen * 1e-3) / 1e12
    return {"workload": "generator: 8x 3840x2160 fp32 -> downsample 256 -> 5 conv (bf16 MFMA) + map head + FC, "
                        "then svdlut_apply at 4K; training step batch 16 at 256x256 (MSE, Adam lr 1e-4)",
            "infer_ms_per_batch8": round(ms_inf, 4), "infer_mpix_s": round(8 * 3840 * 2160 / (ms_inf * 1e-3) / 1e6, 1),
            "generator_fwd_ms_batch8": round(ms_gen, 4), "generator_mac_per_image": macs,
            "generator_tflops": round(tflops, 3), "mfma_frac_of_bf16_peak": round(tflops / BF16_PEAK_TFLOPS, 6),
            "train_step_ms_batch16": round(ms_train, 4), "train_steps_s": round(1000.0 / ms_train, 1),
            # the GEMM kernels under rocprofv3 counters (committed summary of this same row)
            "mfma_counters": mfma_counters()}


def row_p1(svd, torch, synth, args):
    """The paper's whole model at 4K: its generator (m = 8 backbone, four FC generators) then
    the fused slicing + 2D-LUT transform with scalar LUT weights and K = 6 grids."""
    from paper_2508_16121_amd import paper_model as PM
    g = np.random.default_rng(7)
    img = synth.image(g, 2160, 3840)[None]
    gen = PM.PaperGenerator(33, 8, 6, 17, seed=0)
    res = {"workload": "paper model (160,478 params): 3x2160x3840 fp32 -> downsample 256 -> 5 conv blocks (bf16 MFMA, "
                       "LeakyReLU, instance norm) -> pool -> 4 FC generators -> svdlut_apply_grid (K=6 grids 17x17, "
                       "1x1 LUT-weight map); training step batch 16 at 256x256 with dropout (MSE, Adam lr 1e-4)",
           "params": int(gen.n), "paper_v100_ms_4k": 1.38}
    steps = max(10, args.steps // 4)
    for B in (1, 8):
        x = torch.from_numpy(np.concatenate([img] * B)).cuda()
        y = torch.empty_like(x)
        box = {}

        def infer(i):
            o = gen.forward(x)
            box["o"] = o
            svd.apply_grid(x, o["U"], o["s"], o["V"], o["lut_w"], o["grids"], o["gw"], o["gb"], bias=o["lut_b"], out=y)

        ms = event_time(infer, steps, 3, torch)
        ms_gen = event_time(lambda i: gen.forward(x), steps, 3, torch)
        o = box["o"]
        ms_tr = event_time(lambda i: svd.apply_grid(x, o["U"], o["s"], o["V"], o["lut_w"], o["grids"], o["gw"],
                                                    o["gb"], bias=o["lut_b"], out=y), steps, 3, torch)
        enh = PM.PaperEnhancer(gen, B, 2160, 3840)
        ms_graph = event_time(lambda i: enh.graph.replay(), steps, 3, torch)
        res[f"b{B}"] = {"ms": round(ms, 4), "generator_ms": round(ms_gen, 4), "transform_ms": round(ms_tr, 4),
                        "mpix_s": round(B * 3840 * 2160 / (ms * 1e-3) / 1e6, 1), "graph_ms": round(ms_graph, 4),
                        "graph_mpix_s": round(B * 3840 * 2160 / (ms_graph * 1e-3) / 1e6, 1)}
        del enh
    xb = torch.rand(16, 3, 256, 256, device="cuda")
    tb = torch.rand(16, 3, 256, 256, device="cuda")
    tr = PM.PaperTrainer(PM.PaperGenerator(33, 8, 6, 17, seed=1), lr=1e-4)
    ms_train = event_time(lambda i: tr.step(xb, tb), max(10, args.steps // 2), 3, torch)
    res["train_step_ms_batch16"] = round(ms_train, 4)
    res["train_steps_s"] = round(1000.0 / ms_train, 1)
    return res


def main():
    args = parse()
    if args.summarize_trace:
        return summarize_trace(args)
    if args.summarize_traffic:
        return summarize_traffic(args)
    if args.summarize_mfma:
        return summarize_mfma(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import synth
    c2 = synth.frame_4k()                         # host inputs first, before the GPU is touched
    cpu = (cpu_baseline(c2, args.cpu_seconds, synth.plain_256()) if args.cpu_seconds > 0
           else None)                             # forks: before torch
    import torch
    import paper_2508_16121_amd as svd

    # The other rows run first: the headline's warm-up launches then find the GPU's clocks in
    # the state of sustained work rather than ramping up from idle.
    want = {"c1", "c3", "c4", "c5", "g1", "g4", "sweep", "dims", "u1", "p1"} if args.rows == "all" else (set() if args.rows == "none" else set(args.rows.split(",")))
    rows = {}
    for name, fn in (("c1", row_c1), ("c4", row_c4), ("c3", row_c3), ("c5", row_c5), ("g1", row_g1), ("g4", row_g4), ("sweep", row_sweep), ("dims", row_dims), ("u1", row_u1), ("p1", row_p1)):
        if name in want:
            rows[name] = fn(svd, torch, synth, args)
            print(f"row {name} done", file=sys.stderr, flush=True)

    B, H, W, D, R, h, w = c2.shape
    npx = H * W
    sets = []
    for k in range(N_ROT):
        sets.append(dict(x=torch.from_numpy(c2.x).cuda(), U=torch.from_numpy(c2.U).cuda(),
                         s=torch.from_numpy(c2.s).cuda(), V=torch.from_numpy(c2.V).cuda(),
                         m=torch.from_numpy(c2.smap).cuda(), y=torch.empty_like(torch.from_numpy(c2.x)).cuda()))
    torch.cuda.synchronize()

    def step(i):
        b = sets[i % N_ROT]
        svd.apply(b["x"], b["U"], b["s"], b["V"], b["m"], out=b["y"])

    ms, ms_pair = launch_times(step, args.steps, args.warmup, torch)
    bytes_alg = npx * (12 + 12) + 9 * h * w * 4 + 9 * D * R * 2 * 4 + 9 * R * 4
    assert bytes_alg == HEADLINE_BYTES
    out = {
        "metric": "Mpix/s of 2D-LUT apply at 4K (fwd, fwd+bwd, batched); % of HBM peak",
        "value": round(npx / (ms * 1e-3) / 1e6, 1), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "svdlut_apply 1x3x2160x3840 fp32, D=33 R=8, map 9x270x480 fp32, fused reconstruction",
                   "global_batch": 1, "pixels": npx},
        # every step is one launch of the kernel on the library's stream, so the back-to-back
        # step time is the launch duration the roofline is computed from
        "roofline": dict(roof(bytes_alg, ms), traffic=measured_traffic(), kernel=HEADLINE_KERNEL,
                         bytes_per_launch=bytes_alg, event_pair_ms=round(ms_pair, 5), rocprof=profiled_launch()),
    }
    if args.copy_probe:
        src = sets[0]["x"]
        dst = torch.empty_like(src)
        ms_copy = event_time(lambda i: dst.copy_(src), max(5, args.steps // 4), 2, torch)
        out["copy_probe"] = {"bytes_per_copy": 2 * src.numel() * 4, "ms": round(ms_copy, 5),
                             "gb_s": round(2 * src.numel() * 4 / (ms_copy * 1e-3) / 1e9, 1)}
    if rows:
        out["rows"] = rows
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
