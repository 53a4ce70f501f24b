#!/usr/bin/env python3
"""Benchmark of the probe update + probe query on one MI355X.

A step is one pass of the whole hot path over the 16x8x16-probe city (256
rays per probe, ~100k triangles, 8 point lights, 32 emissive quads): the
per-frame update (state step and compaction, ray directions, nearest-hit
traversal, shadow rays, hit shading with the previous frame's probes, blend
with hysteresis and border texels, state promotion) followed by the query of
the full 1920x1080 G-buffer.  Inputs are synthetic and seeded; everything
is resident on the GPU before timing starts.

Prints one JSON line: the metric and its value (ms per city step), the
dominant kernel's roofline (algorithmic bytes or flops over its measured
duration, with DRAM traffic from committed counter figures while the kernel
sources match them), the oracle's CPU time, and the sections' figures.
"""
import argparse
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
NODE_BYTES, TRI_BYTES, RAY_IO_BYTES = 64, 48, 32
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "city-16x8x16-256rays_hbm_traffic.md")


def kernel_source_hash() -> str:
    """sha256 over the library's kernel sources (a change voids measured
    hardware byte counts)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2009_10796_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic() -> dict:
    """Per-launch DRAM bytes per kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a known-size copy), when it was
    taken on the current kernel sources; else {}."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
    except OSError:
        return {}
    block = text.split("```json")[-1].split("```")[0] if "```json" in text else ""
    try:
        data = json.loads(block)
    except ValueError:
        return {}
    if data.get("kernel_source_sha256") != kernel_source_hash():
        return {}
    return {k: int(v) for k, v in data.get("bytes_per_launch", {}).items()}


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


def blend_variants(w, R, frames, irf, torch):
    """Blend kernel time of every blend mode on the same workload and frames,
    and each mode's irradiance difference from the float32 matrix-core path
    (relative, floor 1e-3 of the channel maximum)."""
    import copy
    res, ref = {}, None
    for mode, f16 in (("f32", False), ("f32_valu", False), ("bf16", False), ("f16", False), ("bf16", True),
                      ("f16", True)):
        ww = copy.deepcopy(w)
        for d in ww.volumes:
            d.blend, d.atlas_f16 = mode, f16
        ctx = irf.build_workload(ww, device=0)
        ctx.classify(ww.classify_rotations)
        for f in range(frames):
            if f == frames - 3:
                torch.cuda.synchronize()
                ctx.profile(True)
                ctx.profile_read(reset=True)
            ctx.update_probes(R[f])
        torch.cuda.synchronize()
        prof = ctx.profile_read(reset=True)
        irr = ctx.volumes[0].irradiance[..., :3].float().cpu().numpy().astype(np.float64)
        bk = [k for k in prof if k.startswith("blend")][0]
        t_us = 1e3 * prof[bk][1] / prof[bk][0]
        key = mode + ("+f16atlas" if f16 else "")
        if ref is None:
            ref = irr
        t = 1e-3 * np.abs(ref).reshape(-1, 3).max(0)
        rel = np.abs(irr - ref) / np.maximum(np.abs(ref), t)
        res[key] = {"blend_us": round(t_us, 2), "irr_vs_f32_max": float(rel.max()),
                    "irr_vs_f32_p99": float(np.quantile(rel, 0.99))}
        ctx.close()
    return res


def terrain_batched(irf, torch, frames=60):
    """The batching workload: four cascades of 32x16x32 probes (1, 2, 4, 8 m)
    over ~1.1M triangles of terrain and buildings, 192 rays, a sun moving
    1 degree per frame; launch shapes autotuned, the frame captured as a HIP
    graph and replayed for `frames` frames."""
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
    tuning = autotune.autotune(ctx, R[200:], frames_per_candidate=2)
    for v, st in zip(ctx.volumes, states0):
        v.states.copy_(st)
        v.irradiance.zero_()
        v.distance.zero_()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        g = ctx.capture_frame(s)
    times = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    active = []
    for f in range(frames):
        ctx.set_lights(S.sun_for_frame(f))
        with torch.cuda.stream(s):
            ev0.record(s)
            g.launch(R[f])
            ev1.record(s)
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
        if f == 1:
            active = [int(np.isin(v.states.cpu().numpy(), [4, 5]).sum()) for v in ctx.volumes]
    stats = ctx.frame_stats()
    eager = []
    for f in range(frames, frames + 10):
        ctx.set_lights(S.sun_for_frame(f))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.update_probes(R[f])
        torch.cuda.synchronize()
        eager.append(1e3 * (time.perf_counter() - t0))
    g.close()
    ctx.close()
    steady = np.array(times[2:])
    prim, shad = stats["probe_rays"], stats["shadow_rays"]
    p50 = float(np.median(steady))
    return {"workload": w.name, "triangles": int(w.scene.n_triangles), "frames": frames,
            "probes_per_cascade": int(w.volumes[0].n_probes), "active_per_cascade": active,
            "rays_per_frame": {"primary": int(prim), "shadow": int(shad)},
            "graph_ms_per_frame": {"p50": round(p50, 4), "p95": round(float(np.quantile(steady, 0.95)), 4),
                                   "first": round(times[0], 4)},
            "eager_ms_per_frame_p50": round(float(np.median(eager)), 4),
            "grays_per_s": round((prim + shad) / (p50 * 1e-3) / 1e9, 3),
            "tuning": tuning}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; runs on several GPUs are not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2009_10796_amd import irf, scenes as S
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.only:
        fn = {"terrain": terrain_batched, "adjoint": adjoint_timing, "glossy": glossy_timing}[args.only]
        print(json.dumps({"section": args.only, **fn(irf, torch)}), flush=True)
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
    R = S.rotations(w.config, 1 + args.warmup + 3 * args.steps, start_frame=1)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    print(f"[bench] setup {setup_s:.1f}s, {w.scene.n_triangles} triangles, {q.n} queries", file=sys.stderr, flush=True)

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
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

    # timed (the value): the same steps with eager launches, no instrumentation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.update_probes(R[f])
        ctx.query_irradiance(pos, nrm, view, out)
        f += 1
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step (graph replay {graph_ms:.3f})", file=sys.stderr,
          flush=True)

    # per-kernel times: a separate pass with the library's kernel timing
    ctx.profile(True)
    ctx.profile_read(reset=True)
    for _ in range(args.steps):
        ctx.update_probes(R[f])
        ctx.query_irradiance(pos, nrm, view, out)
        f += 1
    torch.cuda.synchronize()
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    stats = ctx.frame_stats()

    kern = {k: {"launches": n, "avg_us": round(1e3 * ms / max(1, n), 2)} for k, (n, ms) in prof.items()}
    upd = [k for k in kern if k != "query"]
    update_ms = sum(kern[k]["avg_us"] for k in upd) / 1e3
    query_ms = kern["query"]["avg_us"] / 1e3
    prim, shad = stats["probe_rays"], stats["shadow_rays"]
    trav = ctx.traversal_stats()
    states = ctx.volumes[0].states.cpu().numpy()
    qbytes, mean_sampled = query_bytes(w, states)

    traffic = measured_traffic()

    def hbm(kernel, nbytes):
        gbs = nbytes / (kern[kernel]["avg_us"] * 1e-6) / 1e9
        return {"kernel": kernel, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic.get(kernel),
                "algorithmic_bytes_per_launch": int(nbytes)}

    rooflines = {
        "trace": hbm("trace", trav["probe_nodes"] * NODE_BYTES + trav["probe_tris"] * TRI_BYTES + prim * RAY_IO_BYTES),
        "query": hbm("query", qbytes),
    }
    if "shadow" in kern:
        rooflines["shadow"] = hbm("shadow", trav["shadow_nodes"] * NODE_BYTES + trav["shadow_tris"] * TRI_BYTES
                                  + shad * RAY_IO_BYTES)
    n_rays = w.volumes[0].rays_per_probe
    blend_flops = 2.0 * n_rays * (36 * 3 + 196 * 2) * stats["active_probes"]
    bk = [k for k in kern if k.startswith("blend")][0]
    tf = blend_flops / (kern[bk]["avg_us"] * 1e-6) / 1e12
    rooflines["blend"] = {"kernel": bk, "bound": "mfma" if bk == "blend_mma" else "alu", "achieved": round(tf, 3),
                          "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / FP32_PEAK_TFLOPS, 4),
                          "traffic": traffic.get(bk), "algorithmic_flops_per_launch": blend_flops}
    dominant = max(kern, key=lambda k: kern[k]["avg_us"])
    roof = rooflines.get(dominant if not dominant.startswith("blend") else "blend")
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
        "config": {"workload": w.name, "probes": int(w.volumes[0].n_probes), "active_probes": int(stats["active_probes"]),
                   "rays_per_probe": int(w.volumes[0].rays_per_probe), "triangles": int(w.scene.n_triangles),
                   "point_lights": 8, "queries": int(q.n), "blend": "f32", "atlas": "f32",
                   "launch": "eager"},
        "graph_ms_per_step": round(graph_ms, 4),
        "update_ms": round(update_ms, 4),
        "query_ms": round(query_ms, 4),
        "rays": {"primary": int(prim), "shadow": int(shad), "total": int(prim + shad)},
        "grays_per_s": {"primary": round(prim / (kern["trace"]["avg_us"] * 1e-6) / 1e9, 3),
                        "shadow": round(shad / (kern.get("shadow", {"avg_us": float("inf")})["avg_us"] * 1e-6) / 1e9, 3),
                        "total_update": round((prim + shad) / (update_ms * 1e-3) / 1e9, 3)},
        "queries_per_s": round(q.n / (query_ms * 1e-3), 1),
        "kernels_us": kern,
        "dominant_kernel": dominant,
        "traversal": {k: int(v) for k, v in trav.items()},
        "kernel_rooflines": rooflines,
        "roofline": roof,
    }
    if not args.no_blend_variants:
        print("[bench] blend variants ...", file=sys.stderr, flush=True)
        line["blend_variants"] = blend_variants(w, R, 8, irf, torch)
    if not args.no_terrain:
        print("[bench] terrain (batched cascades) ...", file=sys.stderr, flush=True)
        line["batched"] = terrain_batched(irf, torch)
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
