#!/usr/bin/env python3
"""Benchmark of the probe update + probe query on one MI355X.

A step is one pass of the whole hot path over the 16x8x16-probe city (256
rays per probe, ~100k triangles, 8 point lights, 32 emissive quads): the
per-frame update (state step and compaction, ray directions, nearest-hit
traversal, shadow rays, hit shading with the previous frame's probes, blend
with hysteresis and border texels, state promotion) and the query of the
full 1920x1080 G-buffer against its result.  The timed steps answer each
frame's queries inside the next frame's probe-ray trace and shadow-ray
launches (irf_update_probes_query), which gives the same frames and the same query
results as running each frame and then its queries (that schedule is timed
too, `serial_ms_per_step`).  Inputs are synthetic and seeded; everything
is resident on the GPU before timing starts.

Prints one JSON line: the metric and its value (ms per city step), the
dominant kernel's roofline against the bound that binds it (DRAM bytes,
VALU instructions and matrix-core busy cycles per launch from committed
rocprofv3 counter summaries, valid while the kernel sources match them,
over the kernel's live duration), the oracle's CPU time, and the sections'
figures.

``python bench.py --summarize WORKLOAD CSV...`` turns rocprofv3 counter
CSVs of one workload into the committed summary that the roofline reads.
"""
import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "probe update ms/frame, Grays/s, queries/s; MFMA vs FP32 blend at stated error"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# MI355X: 256 compute units x 4 SIMDs, 2.4 GHz; a wave64 VALU instruction
# occupies a 16-lane SIMD for 4 cycles
SIMDS, CLOCK_GHZ = 1024, 2.4
VALU_PEAK_GINSTR = SIMDS * CLOCK_GHZ / 4.0
NODE_BYTES, TRI_BYTES, RAY_IO_BYTES = 64, 48, 32
COUNTER_FILES = {"city": os.path.join(ROOT, "profiles", "city-16x8x16-256rays_counters.md"),
                 "terrain": os.path.join(ROOT, "profiles", "terrain-4x32x16x32-192rays_counters.md")}
# kernel symbol -> bench key (longer names first: k_shadow_refill before
# k_shadow).  The hit shading runs as k_shade_direct when the shadow-ray
# launch computed the indirect terms (every frame with lights), else k_shade:
# one key, since a frame runs one of them
KERNEL_KEYS = (("k_shadow_refill", "shadow_refill"), ("k_shadow_count", "shadow_count"),
               ("k_shadow_query", "shadow_query"), ("k_shadow", "shadow"),
               ("k_trace_count", "trace_count"), ("k_trace_query", "trace_query"), ("k_trace", "trace"),
               ("k_shade_terms", "shade_terms"), ("k_shade_direct", "shade"), ("k_shade", "shade"),
               ("k_blend_mma", "blend_mma"), ("k_blend_f32", "blend_valu"),
               ("k_blend_backward", "blend_backward"), ("k_query_terms", "query_terms"), ("k_query", "query"),
               ("k_gather_pieces", "gather_pieces"), ("k_finish_pieces", "finish_pieces"),
               ("k_piece_offsets", "piece_offsets"), ("k_blend_norms", "blend_norms"), ("k_segments", "segments"),
               ("k_frame_begin", "frame_begin"), ("k_state_count", "state_count"),
               ("k_state_scatter", "state_scatter"), ("k_glossy", "glossy"))
# the sources of the frame and query kernels: a change to any of them voids
# the committed counter figures
KERNEL_SOURCES = ("device_common.h", "irf_internal.h", "kernels_frame.hip", "kernels_trace.hip",
                  "kernels_update.hip", "kernels_blend.hip")


def kernel_source_hash() -> str:
    """sha256 over the sources of the frame and query kernels."""
    import hashlib
    d = os.path.join(ROOT, "paper_2009_10796_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_key(name: str):
    base = name.split("(")[0].split("<")[0].split("::")[-1].strip()
    for sym, key in KERNEL_KEYS:
        if base == sym:
            return key
    if "copyBuffer" in name:
        return "copy"
    return None


def load_counters(workload: str) -> dict:
    """Per-launch hardware figures per kernel of a workload (DRAM bytes,
    VALU instructions, waves, matrix-core busy cycles) from the committed
    summary, if it was taken on the current kernel sources; else {}."""
    try:
        with open(COUNTER_FILES[workload]) as f:
            text = f.read()
    except (OSError, KeyError):
        return {}
    block = text.split("```json")[-1].split("```")[0] if "```json" in text else ""
    try:
        data = json.loads(block)
    except ValueError:
        return {}
    if data.get("kernel_source_sha256") != kernel_source_hash():
        return {}
    return data.get("per_launch", {})


def summarize(workload: str, paths) -> dict:
    """rocprofv3 counter-collection CSVs (any of FETCH_SIZE, WRITE_SIZE,
    SQ_INSTS_VALU, SQ_WAVES, SQ_VALU_MFMA_BUSY_CYCLES, ...) of one workload
    -> per kernel and launch: the mean of each counter over its dispatches.
    FETCH_SIZE and WRITE_SIZE (KiB) are scaled to bytes by the copy kernel of
    --copy-calibration (256 MiB read and written three times)."""
    import csv
    from collections import defaultdict
    per = defaultdict(lambda: defaultdict(lambda: defaultdict(float)))   # key -> counter -> dispatch -> value
    copy_grid = {}                                                      # copy dispatch -> grid size
    for path in paths:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                key = kernel_key(row.get("Kernel_Name", ""))
                if key is None:
                    continue
                d = (path, row.get("Dispatch_Id") or row.get("Correlation_Id"))
                per[key][row["Counter_Name"]][d] += float(row["Counter_Value"])
                if key == "copy":
                    copy_grid[d] = int(float(row.get("Grid_Size") or 0))
    # the calibration copies are the runtime copies of the largest grid (the
    # runtime's other copies are small staging and read-back transfers)
    big = max(copy_grid.values()) if copy_grid else 0
    cal = {d for d, g in copy_grid.items() if g == big}
    copy = {c: [v for d, v in ds.items() if d in cal] for c, ds in per.pop("copy", {}).items()}
    mean = {k: {c: sum(v.values()) / len(v) for c, v in cs.items()} for k, cs in per.items()}
    scale = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        if copy.get(c):
            scale[c] = (256 << 20) / (sum(copy[c]) / len(copy[c]) * 1024.0)
    out = {}
    for k, cs in mean.items():
        e = {}
        if "FETCH_SIZE" in cs and "FETCH_SIZE" in scale:
            e["fetch_bytes"] = cs["FETCH_SIZE"] * 1024.0 * scale["FETCH_SIZE"]
        if "WRITE_SIZE" in cs and "WRITE_SIZE" in scale:
            e["write_bytes"] = cs["WRITE_SIZE"] * 1024.0 * scale["WRITE_SIZE"]
        if "fetch_bytes" in e and "write_bytes" in e:
            e["dram_bytes"] = e["fetch_bytes"] + e["write_bytes"]
        for c, name in (("SQ_INSTS_VALU", "valu_insts"), ("SQ_WAVES", "waves"),
                        ("SQ_VALU_MFMA_BUSY_CYCLES", "mfma_busy_cycles"), ("SQ_INSTS_SALU", "salu_insts"),
                        ("SQ_INSTS_VMEM_RD", "vmem_rd_insts"), ("SQ_INSTS_LDS", "lds_insts")):
            if c in cs:
                e[name] = cs[c]
        out[k] = {n: round(v, 1) for n, v in e.items()}
    return {"workload": workload, "kernel_source_sha256": kernel_source_hash(), "copy_scale": scale,
            "per_launch": out}


def kernel_stats(paths) -> dict:
    """rocprofv3 --kernel-trace --stats CSVs -> per bench key: calls and
    average / min / max duration (us)."""
    import csv
    out = {}
    for path in paths:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                key = kernel_key(row["Name"])
                if key is None:
                    continue
                out[key] = {"calls": int(row["Calls"]), "avg_us": round(float(row["AverageNs"]) / 1e3, 2),
                            "min_us": round(float(row["MinNs"]) / 1e3, 2), "max_us": round(float(row["MaxNs"]) / 1e3, 2)}
    return out


def summary_markdown(workload: str, paths) -> str:
    """The committed form of a profile summary: kernel durations (from
    kernel_stats CSVs), a per-kernel counter table and the JSON block
    load_counters reads (from counter-collection CSVs)."""
    stats_paths = [p for p in paths if p.endswith("kernel_stats.csv")]
    d = summarize(workload, [p for p in paths if p not in stats_paths])
    ks = kernel_stats(stats_paths)
    d["kernel_trace_us"] = ks
    lines = []
    if ks:
        lines += ["| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
        for k, e in sorted(ks.items(), key=lambda kv: -kv[1]["avg_us"]):
            lines.append(f"| {k} | {e['calls']} | {e['avg_us']} | {e['min_us']} | {e['max_us']} |")
        lines.append("")
    rows = ["| kernel | DRAM MB / launch | fetch MB | write MB | waves | VALU instr / wave | MFMA busy cycles |",
            "|---|---|---|---|---|---|---|"]
    for k, e in sorted(d["per_launch"].items()):
        waves = e.get("waves")
        vpw = e["valu_insts"] / waves if waves and "valu_insts" in e else None
        mb = lambda x: f"{x / 1e6:.2f}" if x is not None else "-"
        rows.append(f"| {k} | {mb(e.get('dram_bytes'))} | {mb(e.get('fetch_bytes'))} | {mb(e.get('write_bytes'))} | "
                    f"{int(waves) if waves else '-'} | {f'{vpw:.0f}' if vpw else '-'} | "
                    f"{int(e['mfma_busy_cycles']) if e.get('mfma_busy_cycles') else '-'} |")
    return "\n".join([*lines, f"Counters per launch (mean over the kernel's dispatches); FETCH_SIZE / WRITE_SIZE "
                      f"(KiB) scaled to bytes by the calibration copy: {d['copy_scale']}.", "", *rows, "",
                      "```json", json.dumps(d, indent=1), "```"])


def quiet_gc() -> None:
    """Python's garbage collector off for the timed work: a full collection
    of this process (torch and the workloads: ~170k objects) takes ~37 ms on
    the host, and one landing inside a timed region stalls the GPU's queue
    for that long.  The objects so far are collected once and frozen, and no
    automatic collection runs until the bench ends (reference counting still
    frees everything that is not in a cycle)."""
    gc.collect()
    gc.freeze()
    gc.disable()


def binding_roofline(kernel: str, avg_us: float, counters: dict, extra: dict = None) -> dict:
    """The kernel's fractions of the MI355X limits that could bind it, from
    its per-launch counter figures over its live duration: DRAM bytes vs HBM
    (8 TB/s), VALU instruction issue vs 1024 SIMDs x 2.4 GHz / 4 cycles, and
    matrix-core busy cycles vs 1024 SIMDs x 2.4 GHz.  The roofline is the
    largest (the bound that binds); without counter figures for the current
    kernel sources every field is null."""
    c = counters.get(kernel, {})
    t = avg_us * 1e-6
    cyc = SIMDS * CLOCK_GHZ * 1e9 * t
    fr, ach = {}, {}
    if c.get("dram_bytes"):
        ach["hbm"] = c["dram_bytes"] / t / 1e9
        fr["hbm"] = ach["hbm"] / HBM_PEAK_GBS
    if c.get("valu_insts"):
        ach["alu"] = c["valu_insts"] / t / 1e9
        fr["alu"] = c["valu_insts"] * 4.0 / cyc
    if c.get("mfma_busy_cycles"):
        ach["mfma"] = c["mfma_busy_cycles"] / t / 1e9
        fr["mfma"] = c["mfma_busy_cycles"] / cyc
    out = {"kernel": kernel, "avg_us": round(avg_us, 2)}
    if not fr:
        out.update({"bound": None, "achieved": None, "peak": None, "unit": None, "frac": None, "traffic": None,
                    "fractions": {}})
    else:
        b = max(fr, key=fr.get)
        peak, unit = {"hbm": (HBM_PEAK_GBS, "GB/s"), "alu": (round(VALU_PEAK_GINSTR, 1), "G VALU instr/s"),
                      "mfma": (round(SIMDS * CLOCK_GHZ, 1), "G MFMA busy cycles/s")}[b]
        out.update({"bound": b, "achieved": round(ach[b], 1), "peak": peak, "unit": unit, "frac": round(fr[b], 4),
                    "traffic": int(c["dram_bytes"]) if c.get("dram_bytes") else None,
                    "fractions": {k: round(v, 4) for k, v in fr.items()}})
    if extra:
        out.update(extra)
    return out


def query_bytes(w, states):
    """Algorithmic bytes of the query pass: per point 36 B in + 12 B out,
    the 8 cage states (1 B each) and, per sampled probe, 4 irradiance texels
    (3 x 4 B) and 4 distance texels (2 x 4 B)."""
    d = w.volumes[0]
    q = w.queries
    u = (q.pos.astype(np.float64) - np.array(d.origin)) / np.array(d.spacing)
    cnt = np.array(d.counts)
    g = np.clip(np.floor(u), 0, cnt - 2).astype(np.int64)
    sampled = np.isin(states, [4, 5])
    n = np.zeros(len(u), np.int64)
    for c in range(8):
        cb = np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1])
        gg = g + cb
        idx = gg[:, 0] + cnt[0] * (gg[:, 1] + cnt[1] * gg[:, 2])
        n += sampled[idx]
    return int(len(u) * (36 + 12 + 8) + n.sum() * (4 * 12 + 4 * 8)), float(n.mean())


def cpu_baseline(w, n_frames=3):
    """The FP64 oracle on the host cores, same workload and step."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    oracle.classify(sc, ov, w.classify_rotations)
    oracle.update_frame(sc, w.lights, ov, w.frame_rotation(1), records=False)
    times = []
    q = w.queries
    for f in range(2, 2 + n_frames):
        t0 = time.perf_counter()
        oracle.update_frame(sc, w.lights, ov, w.frame_rotation(f), records=False)
        oracle.query(ov, q.pos, q.nrm, q.view)
        times.append(time.perf_counter() - t0)
    out = {"value": round(1e3 * float(np.median(times)), 3), "unit": "ms/frame", "cores": threads, "kind": "oracle",
           "sample": f"full step (update frame + {q.n} G-buffer queries), FP64, OpenMP, median of {n_frames} frames"}
    out.update(host_cpu())
    out["one_thread"] = cpu_one_thread()
    return out


def host_cpu() -> dict:
    """The host's CPU model, its logical CPU count and the CPUs this process
    may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


# The oracle's full step at one thread, in a child process (OpenMP fixes its
# thread count at start-up): warm-up frame, then three timed steps (update
# frame + G-buffer query), the median reported.
_ONE_THREAD_STEP = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle
from paper_2009_10796_amd import scenes as S
w = S.config1()
sc = oracle.Scene(w.scene)
ov = [oracle.Volume(d) for d in w.volumes]
oracle.classify(sc, ov, w.classify_rotations)
oracle.update_frame(sc, w.lights, ov, w.frame_rotation(1), records=False)
q = w.queries
upd, qry = [], []
for f in (2, 3, 4):
    t0 = time.perf_counter()
    oracle.update_frame(sc, w.lights, ov, w.frame_rotation(f), records=False)
    t1 = time.perf_counter()
    oracle.query(ov, q.pos, q.nrm, q.view)
    t2 = time.perf_counter()
    upd.append(t1 - t0)
    qry.append(t2 - t1)
tot = [a + b for a, b in zip(upd, qry)]
i = int(np.argsort(tot)[1])
print(json.dumps({"update_ms": 1e3 * upd[i], "query_ms": 1e3 * qry[i]}))
"""


def cpu_one_thread() -> dict:
    """The same step of the oracle on one host core (median of three steps)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", _ONE_THREAD_STEP, ROOT], env=env, capture_output=True, text=True,
                           timeout=900)
        d = json.loads(r.stdout.strip().splitlines()[-1])
    except Exception as e:   # reported, never fatal to the GPU figures
        return {"error": f"{type(e).__name__}: {e}"}
    return {"value": round(d["update_ms"] + d["query_ms"], 1), "unit": "ms/frame", "cores": 1,
            "update_ms": round(d["update_ms"], 1), "query_ms": round(d["query_ms"], 1)}


def _oracle_frame_as(oracle, sc, lights, vols, R, tri, vis):
    """The oracle's frame, run again with the GPU's hit and shadow decisions
    on the rays where they differ (rays the oracle flags as ones a float32
    tracer may decide otherwise); returns the number of such rays."""
    saved = oracle.copy_volumes(vols)
    rec = oracle.update_frame(sc, lights, vols, R)
    flip = (rec["tri"] != tri) | (rec["vis"] != vis)
    if flip.any():
        for v, p in zip(vols, saved):
            for a in ("irr", "dist", "irr_kappa", "dist_kappa", "states", "offsets"):
                getattr(v, a)[:] = getattr(p, a)
        oracle.update_frame(sc, lights, vols, R, force=(np.where(flip, 3, 0).astype(np.uint8), tri, vis))
    return int(flip.sum())


def blend_precision(w, irf, torch, timing_frames=6):
    """Every blend mode on the city against the FP64 oracle: after frames 1
    and 2 from the oracle's classification, the relative error (floor 1e-3 of
    the channel's largest value) of each atlas -- irradiance E (R, G, B),
    mean distance mu, mean squared distance mu2 -- as max and p99, and the
    blend kernel's time over further frames."""
    import copy
    import oracle
    sc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    oracle.classify(sc, ov, w.classify_rotations)
    states0 = ov[0].states.copy()
    res, substituted = {}, 0
    for i, (mode, f16) in enumerate((("f32", False), ("f32_valu", False), ("bf16", False), ("f16", False),
                                     ("bf16", True), ("f16", True))):
        ww = copy.deepcopy(w)
        for d in ww.volumes:
            d.blend, d.atlas_f16 = mode, f16
        ctx = irf.build_workload(ww, device=0)
        ctx.volumes[0].states.copy_(torch.from_numpy(states0))
        for f in (1, 2):
            ctx.update_probes(ww.frame_rotation(f))
            torch.cuda.synchronize()
            if i == 0:     # hits and shadow decisions do not depend on the blend
                rec = ctx.ray_records(0)
                substituted += _oracle_frame_as(oracle, sc, w.lights, ov, w.frame_rotation(f), rec["tri"], rec["vis"])
        gi = ctx.volumes[0].irradiance[..., :3].float().cpu().numpy().astype(np.float64)
        gd = ctx.volumes[0].distance.float().cpu().numpy().astype(np.float64)
        err = {}
        for name, g, o in (("E", gi, ov[0].irr), ("mu", gd[..., :1], ov[0].dist[..., :1]),
                           ("mu2", gd[..., 1:], ov[0].dist[..., 1:])):
            tau = 1e-3 * np.abs(o).reshape(-1, o.shape[-1]).max(0)
            rel = np.abs(g - o) / np.maximum(np.abs(o), tau)
            err[name] = {"max": float(rel.max()), "p99": float(np.quantile(rel, 0.99))}
        ctx.profile(True)
        ctx.profile_read(reset=True)
        for f in range(3, 3 + timing_frames):
            ctx.update_probes(ww.frame_rotation(f))
        torch.cuda.synchronize()
        prof = ctx.profile_read(reset=True)
        bk = [k for k in prof if k.startswith("blend")][0]
        key = mode + ("+f16atlas" if f16 else "")
        res[key] = {"blend_us": round(1e3 * prof[bk][1] / prof[bk][0], 2), "vs_fp64": err,
                    "meets_1e-3_irradiance": bool(err["E"]["max"] <= 1e-3)}
        ctx.close()
    res["oracle_substituted_rays"] = substituted
    return res


def terrain_batched(irf, torch, frames=60, oracle_step=True, drift=True, tuning=None):
    """The batching workload: four cascades of 32x16x32 probes (1, 2, 4, 8 m)
    over ~1.1M triangles of terrain and buildings, 192 rays, a sun moving
    1 degree per frame; launch shapes autotuned, the frame captured as a HIP
    graph and replayed for `frames` frames.  Also: per-kernel times of eager
    frames with their rooflines (terrain counter summary), the FP64 oracle's
    one-frame step from the GPU's frame-29 state (its CPU baseline), and the
    drift of float16 atlases from float32 ones over the same frames.
    `tuning`: launch shapes to apply instead of autotuning (for profiles of
    one configuration)."""
    from paper_2009_10796_amd import autotune, scenes as S
    w = S.config3()
    ctx = irf.build_workload(w, device=0)
    ctx.classify(w.classify_rotations)
    R = S.rotations(w.config, 400, start_frame=1)
    states0 = [v.states.clone() for v in ctx.volumes]
    # frames 1-2 converge the probes, then tune on later frames
    ctx.set_lights(S.sun_for_frame(0))
    for f in range(2):
        ctx.update_probes(R[f])
    if tuning is None:
        tuning = autotune.autotune(ctx, R[200:], frames_per_candidate=2)
    else:
        ctx.set_tuning(**tuning)

    def reset(c):
        for v, st in zip(c.volumes, states0):
            v.states.copy_(st)
            v.irradiance.zero_()
            v.distance.zero_()

    reset(ctx)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        g = ctx.capture_frame(s)
    times = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    active, before30 = [], None
    for f in range(frames):
        ctx.set_lights(S.sun_for_frame(f))
        if f == 29:
            before30 = [(v.irradiance[..., :3].float().cpu().numpy(), v.distance.float().cpu().numpy(),
                         v.states.cpu().numpy().copy()) for v in ctx.volumes]
        with torch.cuda.stream(s):
            ev0.record(s)
            g.launch(R[f])
            ev1.record(s)
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
        if f == 1:
            active = [int(np.isin(v.states.cpu().numpy(), [4, 5]).sum()) for v in ctx.volumes]
    stats = ctx.frame_stats()
    g.close()
    eager = []
    for f in range(frames, frames + 10):
        ctx.set_lights(S.sun_for_frame(f))
        torch.cuda.synchronize()
        ev0.record()
        ctx.update_probes(R[f])
        ev1.record()
        ev1.synchronize()
        eager.append(ev0.elapsed_time(ev1))
    ctx.profile(True)
    ctx.profile_read(reset=True)
    for f in range(frames + 10, frames + 20):
        ctx.set_lights(S.sun_for_frame(f))
        ctx.update_probes(R[f])
    torch.cuda.synchronize()
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    kern = {k: {"launches": n, "avg_us": round(1e3 * ms / max(1, n), 2)} for k, (n, ms) in prof.items()}
    counters = load_counters("terrain")
    rooflines = {k: binding_roofline(k, kern[k]["avg_us"], counters) for k in kern}
    dominant = max(kern, key=lambda k: kern[k]["avg_us"])
    steady = np.array(times[2:])
    prim, shad = stats["probe_rays"], stats["shadow_rays"]
    p50 = float(np.median(steady))
    out = {"workload": w.name, "triangles": int(w.scene.n_triangles), "frames": frames,
           "probes_per_cascade": int(w.volumes[0].n_probes), "active_per_cascade": active,
           "rays_per_frame": {"primary": int(prim), "shadow": int(shad)},
           "graph_ms_per_frame": {"p50": round(p50, 4), "p95": round(float(np.quantile(steady, 0.95)), 4),
                                  "first": round(times[0], 4)},
           "eager_ms_per_frame_p50": round(float(np.median(eager)), 4),
           "grays_per_s": round((prim + shad) / (p50 * 1e-3) / 1e9, 3),
           "tuning": tuning, "kernels_us": kern, "dominant_kernel": dominant, "kernel_rooflines": rooflines,
           "roofline": rooflines[dominant]}
    if drift:
        out["f16_atlas_drift"] = f16_drift(irf, torch, w, ctx, states0, R, frames, reset)
    ctx.close()
    if oracle_step and before30 is not None:
        out["cpu_baseline"] = oracle_one_frame(w, before30, R[30], S.sun_for_frame(30))
    return out


def f16_drift(irf, torch, w, ctx, states0, R, frames, reset):
    """The same frames with float16 atlases beside float32 ones (same tuning,
    eager): relative difference of the irradiance atlases (floor 1e-3 of the
    channel's largest value) at frames 1, 2, 10, 30 and 60 -- the storage
    rounding carried through the hysteresis."""
    import copy
    from paper_2009_10796_amd import scenes as S
    w16 = copy.deepcopy(w)
    for d in w16.volumes:
        d.atlas_f16 = True
    c16 = irf.build_workload(w16, device=0)
    c16.set_tuning(**ctx.get_tuning())
    reset(ctx)
    reset(c16)
    rows = {}
    for f in range(frames):
        L = S.sun_for_frame(f)
        for c in (ctx, c16):
            c.set_lights(L)
            c.update_probes(R[f])
        if f + 1 in (1, 2, 10, 30, 60):
            a = np.concatenate([v.irradiance[..., :3].float().cpu().numpy().ravel() for v in ctx.volumes])
            b = np.concatenate([v.irradiance[..., :3].float().cpu().numpy().ravel() for v in c16.volumes])
            tau = 1e-3 * np.abs(a).max()
            rel = np.abs(b.astype(np.float64) - a) / np.maximum(np.abs(a), tau)
            rows[f + 1] = {"max": float(rel.max()), "p99": float(np.quantile(rel, 0.99))}
    c16.close()
    return {"frames": list(rows), "irr_rel_max": [r["max"] for r in rows.values()],
            "irr_rel_p99": [r["p99"] for r in rows.values()]}


def oracle_one_frame(w, state, R, lights):
    """The FP64 oracle's frame 30 of the terrain from the GPU's atlases and
    states after frame 29 (the one-frame stepping of the parity test), timed
    on the host cores (scene and BVH build excluded)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sc = oracle.Scene(w.scene)
    ov = [oracle.Volume(d) for d in w.volumes]
    for o, (irr, dist, st) in zip(ov, state):
        o.irr[:] = irr
        o.dist[:] = dist
        o.states[:] = st
    t0 = time.perf_counter()
    oracle.update_frame(sc, lights, ov, R, records=False)
    ms = 1e3 * (time.perf_counter() - t0)
    out = {"value": round(ms, 1), "unit": "ms/frame", "cores": threads, "kind": "oracle",
           "sample": "one frame (frame 30 from the GPU's frame-29 atlases and states), FP64, OpenMP"}
    out.update(host_cpu())
    return out


def glossy_timing(irf, torch, reps=20):
    """Second-order glossy over the city's G-buffer at quarter resolution
    (every 4th pixel; mirror-reflective ground 0.3, buildings 0.1): mirror
    ray, its shadow rays and two probe lookups per point, after two update
    frames; median time over `reps`."""
    from paper_2009_10796_amd import scenes as S
    w = S.config1()
    spec = np.full((w.scene.albedo.shape[0], 3), 0.1, np.float32)
    spec[0] = 0.3
    w.scene.specular = spec
    ctx = irf.build_workload(w, device=0)
    ctx.classify(w.classify_rotations)
    for f in (1, 2):
        ctx.update_probes(w.frame_rotation(f))
    q = w.queries
    sel = np.arange(0, q.n, 4)
    pos, nrm, view = (torch.from_numpy(np.ascontiguousarray(a[sel])).cuda() for a in (q.pos, q.nrm, q.view))
    for _ in range(3):
        ctx.glossy(pos, nrm, view)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        ev0.record()
        ctx.glossy(pos, nrm, view)
        ev1.record()
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
    _, rec = ctx.glossy(pos, nrm, view, records=True)
    ctx.close()
    ms = float(np.median(times))
    n = int(len(sel))
    shadow = int(sum(bin(int(x)).count("1") for x in rec["vis"]))
    return {"workload": w.name + "-glossy-quarter-res", "points": n, "ms": round(ms, 4),
            "points_per_s": round(n / (ms * 1e-3), 1), "hits": int((rec["tri"] >= 0).sum()),
            "unblocked_shadow_rays": shadow}


def adjoint_timing(irf, torch, reps=10):
    """The differentiable frame at full size (city volume, 64 emissive quads,
    65,536 surface points): forward frame with its inputs saved, query,
    query backward, update backward; median times over `reps`."""
    from paper_2009_10796_amd import scenes as S
    w = S.config4()
    ctx = irf.build_workload(w, device=0)
    ctx.classify(w.classify_rotations)
    for f in (1, 2):
        ctx.update_probes(w.frame_rotation(f))
    q = w.queries
    pos, nrm, view = (torch.from_numpy(a).cuda() for a in (q.pos, q.nrm, q.view))
    target = torch.zeros((q.n, 3), device="cuda")
    st0 = [v.states.clone() for v in ctx.volumes]
    a0 = [(v.irradiance.clone(), v.distance.clone()) for v in ctx.volumes]
    V = ctx.volumes
    Gi = [torch.zeros(v.irradiance.shape, device="cuda") for v in V]
    Gd = [torch.zeros(v.distance.shape, device="cuda") for v in V]
    Pi = [torch.zeros_like(t) for t in Gi]
    Pd = [torch.zeros_like(t) for t in Gd]
    ge = torch.zeros((w.scene.emission.shape[0], 3), device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    rows = {"frame_saving_inputs": [], "query": [], "query_backward": [], "update_backward": [], "frame_plain": []}
    for mode in (True, False):
        ctx.set_differentiable(mode)
        for i in range(reps + 2):
            for v, s0, (a, b) in zip(V, st0, a0):
                v.states.copy_(s0)
                v.irradiance.copy_(a)
                v.distance.copy_(b)
            R = w.frame_rotation(3)
            ev[0].record()
            ctx.update_probes(R)
            ev[1].record()
            if not mode:
                ev[1].synchronize()
                if i >= 2:
                    rows["frame_plain"].append(ev[0].elapsed_time(ev[1]))
                continue
            E = ctx.query_irradiance(pos, nrm, view)
            ev[2].record()
            gE = (2.0 / E.numel()) * (E - target)
            for t in Gi + Gd + Pi + Pd + [ge]:
                t.zero_()
            ev[3].record()
            ctx.query_backward(pos, nrm, view, gE, Gi, Gd)
            ev[4].record()
            ctx.update_backward(Gi, Gd, Pi, Pd, ge)
            e5 = torch.cuda.Event(enable_timing=True)
            e5.record()
            e5.synchronize()
            if i >= 2:
                rows["frame_saving_inputs"].append(ev[0].elapsed_time(ev[1]))
                rows["query"].append(ev[1].elapsed_time(ev[2]))
                rows["query_backward"].append(ev[3].elapsed_time(ev[4]))
                rows["update_backward"].append(ev[4].elapsed_time(e5))
    ctx.set_differentiable(False)
    stats = ctx.frame_stats()
    ctx.close()
    med = {k: round(float(np.median(v)), 4) for k, v in rows.items()}
    return {"workload": w.name, "points": int(q.n), "emitter_parameters": 64 * 3,
            "texel_gradients": int(V[0].n_probes * (64 * 3 + 256 * 2)), "active_probes": int(stats["active_probes"]),
            "ms": med,
            "backward_ms": round(med["query_backward"] + med["update_backward"], 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-blend-variants", action="store_true")
    ap.add_argument("--no-terrain", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-glossy", action="store_true")
    ap.add_argument("--only", choices=["terrain", "adjoint", "glossy"],
                    help="run one secondary section alone and print its JSON (for per-section profiles)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 256 MiB device-to-device three times before timing (a known-size kernel for "
                         "scaling hardware byte counters)")
    ap.add_argument("--no-drift", action="store_true", help="terrain: skip the float16-atlas drift run")
    ap.add_argument("--tuning", help="terrain: JSON launch shapes to apply instead of autotuning")
    ap.add_argument("--summarize", nargs="+", metavar="ARG",
                    help="WORKLOAD CSV...: print the counter summary (markdown with a JSON block) of rocprofv3 "
                         "counter-collection CSVs of one workload (city or terrain); runs no GPU work")
    args = ap.parse_args()
    if args.summarize:
        print(summary_markdown(args.summarize[0], args.summarize[1:]))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; runs on several GPUs are not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2009_10796_amd import irf, scenes as S
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        quiet_gc()
        if args.only == "terrain":
            res = terrain_batched(irf, torch, oracle_step=not args.no_cpu_baseline, drift=not args.no_drift,
                                  tuning=json.loads(args.tuning) if args.tuning else None)
        else:
            res = {"adjoint": adjoint_timing, "glossy": glossy_timing}[args.only](irf, torch)
        print(json.dumps({"section": args.only, **res}), flush=True)
        return
    t_setup = time.perf_counter()
    w = S.config1()
    ctx = irf.build_workload(w, device=0)
    ctx.classify(w.classify_rotations)
    q = w.queries
    pos = torch.from_numpy(q.pos).cuda()
    nrm = torch.from_numpy(q.nrm).cuda()
    view = torch.from_numpy(q.view).cuda()
    out = torch.empty_like(pos)
    R = S.rotations(w.config, 1 + 4 * max(2, args.warmup) + 7 * args.steps, start_frame=1)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    print(f"[bench] setup {setup_s:.1f}s, {w.scene.n_triangles} triangles, {q.n} queries", file=sys.stderr, flush=True)
    quiet_gc()

    f = 0
    for _ in range(max(1, args.warmup)):
        ctx.update_probes(R[f])
        ctx.query_irradiance(pos, nrm, view, out)
        f += 1
    torch.cuda.synchronize()

    # the update frame replayed as a captured HIP graph (its only per-frame
    # input is the rotation) followed by the G-buffer query, one stream
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        graph = ctx.capture_frame(s)
        for _ in range(max(1, args.warmup)):     # replays warm up like the eager steps
            graph.launch(R[f])
            ctx.query_irradiance(pos, nrm, view, out)
            f += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        for _ in range(args.steps):
            graph.launch(R[f])
            ctx.query_irradiance(pos, nrm, view, out)
            f += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    graph.close()
    graph_ms = 1e3 * (t1 - t0) / args.steps

    # the fused steps (below) with the frame that answers the queries
    # captured as a graph (irf_graph_capture_query)
    with torch.cuda.stream(s):
        gq = ctx.capture_frame_query(pos, nrm, view, out, s)

        def graph_fused_steps(k):
            nonlocal f
            ctx.update_probes(R[f])
            f += 1
            for _ in range(k - 1):
                gq.launch(R[f])
                f += 1
            ctx.query_irradiance(pos, nrm, view, out)

        graph_fused_steps(max(2, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        graph_fused_steps(args.steps)
    torch.cuda.synchronize()
    graph_fused_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    gq.close()

    # the same steps with eager launches, no instrumentation: serial (each
    # frame, then its query) ...
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.update_probes(R[f])
        ctx.query_irradiance(pos, nrm, view, out)
        f += 1
    torch.cuda.synchronize()
    serial_ms = 1e3 * (time.perf_counter() - t0) / args.steps

    def fused_steps(k):
        # k frames and k queries with the same results as the serial steps:
        # the query of frame i runs inside frame i+1's trace and shadow-ray
        # launches (irf_update_probes_query), the last one on its own
        nonlocal f
        ctx.update_probes(R[f])
        f += 1
        for _ in range(k - 1):
            ctx.update_probes_query(R[f], pos, nrm, view, out)
            f += 1
        ctx.query_irradiance(pos, nrm, view, out)

    # ... and (the value) fused: the same frames and queries, each query
    # answered inside the next frame's traversal launches
    fused_steps(max(2, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fused_steps(args.steps)
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step (serial {serial_ms:.3f}, graph replay "
          f"{graph_ms:.3f}, fused graph replay {graph_fused_ms:.3f})", file=sys.stderr, flush=True)

    # per-kernel times: separate passes with the library's kernel timing,
    # serial (the update's and the query's own kernels) and fused
    def profiled(run):
        ctx.profile(True)
        ctx.profile_read(reset=True)
        run()
        torch.cuda.synchronize()
        pr = ctx.profile_read(reset=True)
        ctx.profile(False)
        return {k: {"launches": n, "avg_us": round(1e3 * ms / max(1, n), 2)} for k, (n, ms) in pr.items()}

    def serial_steps():
        nonlocal f
        for _ in range(args.steps):
            ctx.update_probes(R[f])
            ctx.query_irradiance(pos, nrm, view, out)
            f += 1

    kern = profiled(serial_steps)
    kern_fused = profiled(lambda: fused_steps(args.steps))
    stats = ctx.frame_stats()

    # the fused steps' own launches (the plain first frame and the last
    # query run once per pass)
    step_kernels = sorted(k for k, e in kern_fused.items() if e["launches"] >= args.steps - 1)
    for k in step_kernels:
        kern.setdefault(k, kern_fused[k])
    upd = [k for k in kern if k not in ("query", "trace_query", "shadow_query")]
    update_ms = sum(kern[k]["avg_us"] for k in upd) / 1e3
    query_ms = kern["query"]["avg_us"] / 1e3
    prim, shad = stats["probe_rays"], stats["shadow_rays"]
    trav = ctx.traversal_stats()
    states = ctx.volumes[0].states.cpu().numpy()
    qbytes, mean_sampled = query_bytes(w, states)

    counters = load_counters("city")
    sk = "shadow_refill" if "shadow_refill" in kern else "shadow"

    def fetch(kernel, nbytes):
        # node, triangle and texel fetches as if each came from HBM: served
        # by L2 and the Infinity Cache, so not a bound (context only)
        return {"fetch_bytes_per_launch": int(nbytes),
                "cache_served_fetch_GBps": round(nbytes / (kern[kernel]["avg_us"] * 1e-6) / 1e9, 1)}

    n_rays = w.volumes[0].rays_per_probe
    blend_flops = 2.0 * n_rays * (36 * 3 + 196 * 2) * stats["active_probes"]
    bk = [k for k in kern if k.startswith("blend")][0]
    extra = {
        "trace": fetch("trace", trav["probe_nodes"] * NODE_BYTES + trav["probe_tris"] * TRI_BYTES + prim * RAY_IO_BYTES),
        # compulsory: each point's position, normal and view in, irradiance
        # out, the states and the sampled probes' atlases once
        "query": dict(fetch("query", qbytes), compulsory_bytes_per_launch=int(
            q.n * 48 + states.size + np.isin(states, [4, 5]).sum() * (64 * 16 + 256 * 8))),
        sk: fetch(sk, trav["shadow_nodes"] * NODE_BYTES + trav["shadow_tris"] * TRI_BYTES
                  + shad * RAY_IO_BYTES) if sk in kern else {},
        bk: {"algorithmic_flops_per_launch": blend_flops,
             "fp32_matrix_frac": round(blend_flops / (kern[bk]["avg_us"] * 1e-6) / 1e12 / FP32_PEAK_TFLOPS, 4)},
    }
    # the fused launches: each traversal's own fetches and its share of the queries'
    share = ctx.get_tuning()["query_shadow"] / 1000.0
    if "trace_query" in kern:
        extra["trace_query"] = fetch("trace_query", trav["probe_nodes"] * NODE_BYTES + trav["probe_tris"] * TRI_BYTES
                                     + prim * RAY_IO_BYTES + (1.0 - share) * qbytes)
    if "shadow_query" in kern:
        extra["shadow_query"] = fetch("shadow_query", trav["shadow_nodes"] * NODE_BYTES + trav["shadow_tris"]
                                      * TRI_BYTES + shad * RAY_IO_BYTES + share * qbytes)
    rooflines = {k: binding_roofline(k, kern[k]["avg_us"], counters, extra.get(k)) for k in kern}
    # the dominant kernel of the timed (fused) step
    dominant = max(step_kernels, key=lambda k: kern[k]["avg_us"])
    roof = rooflines[dominant]
    line = {
        "metric": METRIC,
        "value": round(ms_step, 4),
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "query_shadow": ctx.get_tuning()["query_shadow"],
        "config": {"workload": w.name, "probes": int(w.volumes[0].n_probes), "active_probes": int(stats["active_probes"]),
                   "rays_per_probe": int(w.volumes[0].rays_per_probe), "triangles": int(w.scene.n_triangles),
                   "point_lights": 8, "queries": int(q.n), "blend": "f32", "atlas": "f32",
                   "launch": "eager, each frame's G-buffer query inside the next frame's trace and shadow "
                             "launches"},
        "serial_ms_per_step": round(serial_ms, 4),
        "graph_ms_per_step": round(graph_ms, 4),
        "graph_fused_ms_per_step": round(graph_fused_ms, 4),
        "update_ms": round(update_ms, 4),
        "query_ms": round(query_ms, 4),
        "rays": {"primary": int(prim), "shadow": int(shad), "total": int(prim + shad)},
        "grays_per_s": {"primary": round(prim / (kern["trace"]["avg_us"] * 1e-6) / 1e9, 3),
                        "shadow": round(shad / (kern.get(sk, {"avg_us": float("inf")})["avg_us"] * 1e-6) / 1e9, 3),
                        "total_update": round((prim + shad) / (update_ms * 1e-3) / 1e9, 3)},
        "queries_per_s": round(q.n / (query_ms * 1e-3), 1),
        "kernels_us": kern,
        "step_kernels": step_kernels,
        "dominant_kernel": dominant,
        "traversal": {k: int(v) for k, v in trav.items()},
        "kernel_rooflines": rooflines,
        "roofline": roof,
    }
    if not args.no_blend_variants:
        print("[bench] blend modes against the FP64 oracle ...", file=sys.stderr, flush=True)
        line["blend_variants"] = blend_precision(w, irf, torch)
    if not args.no_terrain:
        print("[bench] terrain (batched cascades) ...", file=sys.stderr, flush=True)
        line["batched"] = terrain_batched(irf, torch, oracle_step=not args.no_cpu_baseline, drift=not args.no_drift)
    if not args.no_glossy:
        print("[bench] second-order glossy ...", file=sys.stderr, flush=True)
        line["glossy"] = glossy_timing(irf, torch)
    if not args.no_adjoint:
        print("[bench] adjoint (differentiable frame) ...", file=sys.stderr, flush=True)
        line["adjoint"] = adjoint_timing(irf, torch)
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
