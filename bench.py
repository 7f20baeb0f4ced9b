"""Benchmark of the Darknet-style CNN forward on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-secondary]

Headline workload: the 9-layer plain CNN (widths 16..512 with 2x2 pools, two
conv3x3 to 1024, linear 1x1 to 125) at batch 64 on 3x416x416 seeded
synthetic images, BF16 activations and weights on MFMA with FP32
accumulation, batch norm folded in FP64 at load, one hipGraph-captured
forward per step (ingest -> 9 convs with fused bias/BN/leaky/pool epilogues
-> egress), tile shapes chosen by the library's autotuner.  Inputs are
resident in HBM before the timed region starts.

One JSON line is printed with images/s, the roofline of the dominant kernel
(the conv3x3 1024->1024 at 13x13, K = 9216), p50/p99 step latency, the FP64
oracle timed on the host cores, and secondary figures (FP8, FP32 batch 64,
FP32 batch 1 resident vs per-layer-transfer).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "images/s per GPU (FP32 vs BF16/FP8), % MFMA peak, p50/p99 latency"
PEAK = {"bf16": 2.5e15, "fp8": 5.0e15, "f32": 157.3e12}
HBM_PEAK = 8.0e12
CSRC = os.path.join(ROOT, "paper_1811_03882_amd", "csrc")


def _tile_desc(dn, t: int) -> str:
    try:
        return "%dx%d tile, %dx%d waves, BF16 MFMA %d" % dn.tile_info(t)
    except Exception:
        return "direct kernel"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("conv.hip", "dn_kernels.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def conv_flops(net, batch, h, w):
    """2*M*N*K per conv layer (padded taps counted), logical channels."""
    import synth
    out, c, hh, ww = {}, net.in_c, h, w
    for i, L in enumerate(net.layers):
        if L.kind == synth.CONV:
            ho = (hh + 2 * L.pad - L.ksize) // L.stride + 1
            wo = (ww + 2 * L.pad - L.ksize) // L.stride + 1
            out[i] = (2.0 * batch * ho * wo * L.cout * c * L.ksize * L.ksize, batch * ho * wo, L.cout, c * L.ksize * L.ksize)
            c, hh, ww = L.cout, ho, wo
        elif L.kind == synth.MAXPOOL:
            hh, ww = (hh - 1) // L.stride + 1, (ww - 1) // L.stride + 1
    return out


def build_net(dn, torch, net, dtype, batch, h, w, params, use_graph=True, tune=True, mode=0, calib=None,
              input_u8=False):
    n = dn.Net(net.layers, net.in_c, h, w, batch, dtype=dtype, mode=mode, leaky_slope=net.leaky_slope,
               bn_eps=net.bn_eps, use_graph=use_graph, input_u8=input_u8)
    n.load_params(params)
    if dtype == dn.FP8:
        n.calibrate(calib, calib.shape[0], h, w)
    nbytes = n.arena_bytes(batch, h, w)
    arena = torch.empty(nbytes * (2 if tune else 1) + 256, dtype=torch.uint8, device="cuda")
    n.bind_arena(arena)
    if tune:
        n.autotune(batch, h, w)
    torch.cuda.synchronize()
    return n, arena


def time_steps(torch, fn, steps, warmup, stream):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) for a, b in evs])
    return wall, per


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s: float = 12.0):
    """The FP64 oracle, as it stands, on whole 416x416 images of the 9-layer
    net: all OpenMP threads for about budget_s, then one image on one thread."""
    import oracle
    import synth
    from oracle import net as onet
    net = synth.plain9()
    params = synth.make_params(net, synth.SEED_PLAIN)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.set_threads(threads)
    n, t0 = 0, time.perf_counter()
    while True:
        x = synth.make_input(net, 1, synth.SEED_PLAIN, tag=100 + n)
        onet.forward(net, params, x)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    t1 = time.perf_counter()
    onet.forward(net, params, synth.make_input(net, 1, synth.SEED_PLAIN, tag=99))
    single = time.perf_counter() - t1
    oracle.set_threads(threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": n / dt, "unit": "images/s", "cores": threads, "kind": "oracle",
            "sample": "%d whole 3x416x416 images of the 9-layer net, FP64 direct convolution, "
                      "OpenMP over (image, channel), %.1f s" % (n, dt),
            "single_thread_images_per_s": 1.0 / single, "cpu_model": _cpu_model(),
            "host_cpus": os.cpu_count(), "cpus_available": affinity}


def serving(torch, dn, n_requests: int = 10000, rate: float = 2000.0, log=print,
            sweep=(("bf16_continuous_batching", (4000.0, 8000.0, 16000.0, 32000.0, 48000.0)),
                   ("bf16_continuous_batching_u8frames", (8000.0, 16000.0, 32000.0, 48000.0, 64000.0, 96000.0)),
                   ("f32_plain_batch1", (1000.0, 2000.0, 4000.0, 8000.0)))):
    """Open-loop serving of the mixed-resolution trace: BF16 continuous batching
    (8 slots, batches padded to powers of two up to 64) vs the FP32 plain path
    (batch 1, one stream, arrival order) on the same GPU.  Both replay captured
    graphs on fixed per-slot regions, with tiles tuned for every (batch, size)
    they form.  Each path reports the device overlap of its batches (event
    timestamps) and a capacity sweep: offered rate against served rate and
    p99 latency, and the first rate at which p99 passes 50 ms."""
    import synth
    from paper_1811_03882_amd import serve
    net = synth.plain9()
    params = synth.make_params(net, synth.SEED_PLAIN)
    sizes = synth.serving_trace(1, rate, synth.SEED_SERVING).sizes
    # camera frames arrive in pinned host buffers (8 distinct frames per size),
    # as FP32 or as the 8-bit pixels they are quantised from
    frames = {s: [synth.serving_image(1000000 + 8 * j + k, s).astype(np.float32)[0] for k in range(8)]
              for j, s in enumerate(sizes)}
    pool = {s: [torch.from_numpy(f).pin_memory() for f in fs] for s, fs in frames.items()}
    pool8 = {s: [torch.from_numpy(np.round(f * 255.0).astype(np.uint8)).pin_memory() for f in fs]
             for s, fs in frames.items()}
    rates = dict(sweep)
    out = {}
    for name, dtype, slots, max_batch, bucketed, u8 in (("bf16_continuous_batching", dn.BF16, 8, 64, True, False),
                                                        ("bf16_continuous_batching_u8frames", dn.BF16, 8, 64, True, True),
                                                        ("f32_plain_batch1", dn.F32, 1, 1, False, False)):
        log("[bench] serving %s" % name)
        t_setup = time.perf_counter()
        src = pool8 if u8 else pool
        image_of = lambda r, src=src: src[r.size][r.rid % 8]
        n = dn.Net(net.layers, net.in_c, max(sizes), max(sizes), max_batch, dtype=dtype, use_graph=True,
                   input_u8=u8)
        n.load_params(params)
        batches = [1 << k for k in range(max_batch.bit_length()) if (1 << k) <= max_batch]
        # tune first (in a scratch arena with room for split-K candidates): the
        # executor sizes its slot regions from the tuned plans
        scratch = torch.empty(2 * max(n.arena_bytes(max_batch, S, S) for S in sizes) + (512 << 20),
                              dtype=torch.uint8, device="cuda")
        n.bind_arena(scratch)
        for S in sizes:
            for b in batches:
                n.autotune(b, S, S)
        torch.cuda.synchronize()
        ex = serve.DnExecutor(n, torch, budget_bytes=0, n_slots=slots, image_of=image_of, max_batch=max_batch,
                              max_size=max(sizes), keep_outputs=False, fixed_slots=True, sizes=sizes)
        n.bind_arena(ex.pool, ex.region)
        del scratch
        # warm-up: capture each slot's graph of every (batch, size), not counted
        for slot in range(slots):
            for S in sizes:
                for b in batches:
                    h = ex.launch(slot, [serve.Request(-1, S, 0.0)], b, S, 0)
                    h[0].synchronize()
        t_setup = time.perf_counter() - t_setup

        def run(rate_, count):
            trace = synth.serving_trace(count, rate_, synth.SEED_SERVING)
            sch = serve.Scheduler(ex, ex.pool.numel(), sizes, max_batch=max_batch, bucketed=bucketed,
                                  pad_pow2=bucketed)
            ex.intervals.clear()
            ref = torch.cuda.Event(enable_timing=True)
            ref.record()
            st = sch.run(serve.make_requests(trace))
            torch.cuda.synchronize()
            d = st.as_dict()
            d.update({"offered_per_s": rate_, "device": serve.device_overlap(ex.intervals, ref)})
            return d
        d = run(rate, n_requests)
        d.update({"dtype": {0: "f32", 1: "bf16"}[dtype], "slots": slots, "graph": True, "tuned": True,
                  "frames": "uint8" if u8 else "fp32", "budget_gb": ex.pool.numel() / 2 ** 30, "setup_s": t_setup})
        log("[bench]   %s" % d)
        points = []
        for r in rates.get(name, ()):
            pt = run(r, int(min(20000, r * 1.5)))
            points.append({k: pt[k] for k in ("offered_per_s", "images_per_s", "p50_ms", "p99_ms", "mean_batch",
                                              "max_inflight")} | {"overlap_frac": pt["device"]["overlap_frac"]})
            log("[bench]   capacity %s" % points[-1])
            if pt["p99_ms"] > 500.0:
                break
        cross = next((p["offered_per_s"] for p in [d] + points if p["p99_ms"] > 50.0), None)
        d["capacity"] = {"points": points, "first_rate_p99_over_50ms": cross}
        out[name] = d
        del ex
        n.close()
    return {"workload": "%d Poisson requests at %.0f req/s, S uniform over %s, 9-layer CNN; capacity sweep with "
                        "min(20000, 1.5 s) of requests per rate" % (n_requests, rate, sizes),
            **out}


def placement_search(dn, net, params, xh, log=print, population=30, generations=20, reps=3):
    """The paper's GA offload search (Sec. 3.3, 4; M, T, Pc, Pm, fitness and
    the timeout penalty of Sec. 5.1.2) over the per-layer CPU/GPU placement of
    the 9-layer net, FP32, batch 1, 416x416: best gene against all-GPU and
    all-CPU placements, with the crossings each implies."""
    H, W = xh.shape[2], xh.shape[3]
    n = dn.Net(net.layers, net.in_c, H, W, 1, dtype=dn.F32, leaky_slope=net.leaky_slope, bn_eps=net.bn_eps)
    n.load_params(params)
    import torch
    arena = torch.empty(max(n.placed_arena_bytes(1, H, W), n.arena_bytes(1, H, W)), dtype=torch.uint8, device="cuda")
    n.bind_arena(arena)
    y = np.empty((1,) + n.output_shape(H, W), np.float32)
    L = len(net.layers)

    def timed(gene, k=5):
        n.forward_placed(gene, xh, 1, H, W, y)
        t = []
        for _ in range(k):
            t0 = time.perf_counter()
            n.forward_placed(gene, xh, 1, H, W, y)
            t.append(time.perf_counter() - t0)
        return float(np.median(t))
    all_gpu, all_cpu = np.ones(L, np.uint8), np.zeros(L, np.uint8)
    t_gpu, t_cpu = timed(all_gpu), timed(all_cpu)
    log("[bench] placement: all-GPU %.3f ms, all-CPU %.3f ms" % (t_gpu * 1e3, t_cpu * 1e3))
    p = dn.ga_params(population=population, generations=generations, crossover=0.9, mutation=0.05,
                     timeout_s=180.0, penalty_s=1000.0, seed=1)
    t0 = time.perf_counter()
    best, gen, res = n.ga_place(p, xh, 1, H, W, y, reps=reps)
    wall = time.perf_counter() - t0
    t_best = timed(best)
    xfer = n.placed_transfers(best, 1, H, W)
    log("[bench] placement GA: best %s %.3f ms after %d evaluations (%.1f s)" %
        ("".join(map(str, best)), t_best * 1e3, res.evaluations, wall))
    out = {"workload": "placement search (GA of Sec. 3.3/4/5.1.2) over the 15 layers of the 9-layer net, f32 b1 "
                       "416x416: each gene's layers on the GPU (1) or the host CPU (0), copies by the Sec. 3.2 rule",
           "gene_length": L, "population": population, "generations": generations, "crossover": 0.9,
           "mutation": 0.05, "fitness": "time^-0.5", "reps_per_gene": reps,
           "host_threads": int(os.environ.get("DN_CPU_THREADS", os.environ.get("OMP_NUM_THREADS", "0")) or 0) or None,
           "best_gene": "".join(map(str, best)), "best_ms": t_best * 1e3, "best_ms_in_search": res.best_seconds * 1e3,
           "generation_best_ms": [g * 1e3 for g in gen], "evaluations": res.evaluations, "memo_hits": res.memo_hits,
           "search_wall_s": wall, "all_gpu_ms": t_gpu * 1e3, "all_cpu_ms": t_cpu * 1e3,
           "speedup_best_over_all_cpu": t_cpu / t_best,
           "best_gene_copies": {"h2d": xfer[0], "d2h": xfer[1], "h2d_bytes": xfer[2], "d2h_bytes": xfer[3]}}
    n.close()
    return out


def traffic_from_profiles(layer_key: str, tile: int):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    PMC summary, only if it was taken on the current kernel source and with
    the tile configuration this run chose (the autotuner may pick either of
    two near-equal tiles from run to run; the summary holds one entry each)."""
    path = os.path.join(ROOT, "profiles", "conv_dominant_b64_bf16_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        if d.get("kernel_source_hash") != kernel_source_hash():
            return None
        return d.get(layer_key, {}).get("tile%d" % tile, {}).get("hbm_bytes_per_launch")
    except (OSError, ValueError):
        return None


def _csv_rows(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def summarize_trace(trace_csv: str, min_run: int = 20) -> str:
    """Markdown summary of a rocprofv3 --kernel-trace CSV: per-kernel dispatch
    statistics, and every run of >= min_run consecutive dispatches of one
    kernel (the per-layer timing loops of this script; the first such run is
    the dominant conv, timed right after the graph-replay steps)."""
    rows = sorted(_csv_rows(trace_csv), key=lambda r: int(r["Start_Timestamp"]))
    per = {}
    for r in rows:
        per.setdefault(r["Kernel_Name"], []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = ["| kernel | dispatches | avg us | min us | max us | total ms |", "|---|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        out.append("| `%s` | %d | %.2f | %.2f | %.2f | %.3f |" % (k[:110], len(v), np.mean(v), min(v), max(v), sum(v) / 1e3))
    runs, i = [], 0
    while i < len(rows):
        j = i
        while j < len(rows) and rows[j]["Kernel_Name"] == rows[i]["Kernel_Name"]:
            j += 1
        if j - i >= min_run:
            d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows[i:j]]
            runs.append((rows[i]["Kernel_Name"], j - i, float(np.mean(d)), float(np.median(d))))
        i = j
    out += ["", "Runs of >= %d consecutive dispatches of one kernel (per-layer timing loops, in order):" % min_run, "",
            "| # | kernel | dispatches | avg us | median us |", "|---|---|---|---|---|"]
    for n, (k, c, a, m) in enumerate(runs):
        out.append("| %d | `%s` | %d | %.2f | %.2f |" % (n, k[:110], c, a, m))
    return "\n".join(out)


API_REPS = 20


def api_driver(torch, dn, net, params, x, stream, log=print):
    """Steady-state host API use per forward, for a rocprofv3 --hip-trace
    --marker-trace --kernel-trace run: each case runs API_REPS forwards inside
    one roctx range (warm-up, tuning and graph capture happen before it)."""
    import ctypes
    roctx = ctypes.CDLL("librocprofiler-sdk-roctx.so")
    roctx.roctxRangePushA.argtypes = [ctypes.c_char_p]
    roctx.roctxMarkA.argtypes = [ctypes.c_char_p]
    B, H, W = x.shape[0], x.shape[2], x.shape[3]

    def ranged(name, fn):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        roctx.roctxRangePushA(("%s x%d" % (name, API_REPS)).encode())
        for _ in range(API_REPS):
            fn()
        roctx.roctxRangePop()
        torch.cuda.synchronize()
        roctx.roctxMarkA(("%s x%d end" % (name, API_REPS)).encode())
        log("[api] %s done" % name)

    out_shape = None
    nb, ab = build_net(dn, torch, net, dn.BF16, B, H, W, params)
    out_shape = nb.output_shape(H, W)
    y = torch.empty((B,) + out_shape, dtype=torch.float32, device="cuda")
    ranged("bf16_b%d_graph_device_io" % B, lambda: nb.forward(x, B, H, W, y, stream))
    xh = torch.empty(x.shape, dtype=torch.float32, pin_memory=True)
    xh.copy_(x.cpu())
    yh = torch.empty(y.shape, dtype=torch.float32, pin_memory=True)
    xd = torch.empty_like(x)

    def with_pcie():
        with torch.cuda.stream(stream):
            xd.copy_(xh, non_blocking=True)
            nb.forward(xd, B, H, W, y, stream)
            yh.copy_(y, non_blocking=True)
    ranged("bf16_b%d_graph_pinned_host_io" % B, with_pcie)
    nb.close()
    x1 = x[:1].contiguous()
    y1 = torch.empty((1,) + out_shape, dtype=torch.float32, device="cuda")
    n3, a3 = build_net(dn, torch, net, dn.F32, 1, H, W, params)
    ranged("f32_b1_graph_device_io", lambda: n3.forward(x1, 1, H, W, y1, stream))
    n3.close()
    n4, a4 = build_net(dn, torch, net, dn.F32, 1, H, W, params, use_graph=False, tune=False)
    ranged("f32_b1_eager_device_io", lambda: n4.forward(x1, 1, H, W, y1, stream))
    n4.close()
    n5, a5 = build_net(dn, torch, net, dn.F32, 1, H, W, params, use_graph=False, tune=False, mode=dn.PER_LAYER)
    x1h = np.ascontiguousarray(x1.cpu().numpy())
    y1h = np.empty((1,) + out_shape, np.float32)
    ranged("f32_b1_per_layer_transfer", lambda: n5.forward(x1h, 1, H, W, y1h))
    n5.close()


def summarize_api(trace_dir: str) -> str:
    """Markdown summary of an api_driver run: per roctx range, HIP API calls
    per forward (copies, synchronisations, allocations, launches), and the
    GPU timeline of the range's kernels (busy time per forward and the idle
    gaps between kernels)."""
    import glob
    def one(pattern):
        f = sorted(glob.glob(os.path.join(trace_dir, "**", pattern), recursive=True))
        if not f:
            raise SystemExit("no %s under %s" % (pattern, trace_dir))
        return _csv_rows(f[0])
    api, marks, kern = one("*hip_api_trace.csv"), one("*marker_api_trace.csv"), one("*kernel_trace.csv")
    groups = [("graph launch", lambda f: f.startswith("hipGraphLaunch")),
              ("kernel launch", lambda f: f in ("hipLaunchKernel", "hipExtLaunchKernel", "hipModuleLaunchKernel")
               or f.startswith("__hipPushCallConfiguration")),
              ("copy host->device", None), ("copy device->host", None),
              ("copy (all hipMemcpy*)", lambda f: f.startswith("hipMemcpy")),
              ("synchronize", lambda f: "Synchronize" in f or f.startswith("hipEventSynchronize")),
              ("allocate / free", lambda f: f.startswith(("hipMalloc", "hipFree", "hipHostMalloc", "hipHostFree",
                                                          "hipExtMalloc"))),
              ("graph capture / instantiate", lambda f: "Capture" in f or "Instantiate" in f)]
    out = ["| range (%d forwards) | %s | all HIP calls | GPU busy us / fwd | kernels / fwd | idle us / fwd |"
           % (API_REPS, " | ".join(g[0] for g in groups if g[1] is not None)),
           "|---|" + "---|" * (sum(1 for g in groups if g[1] is not None) + 4)]
    ends = {m.get("Function", ""): int(m["Start_Timestamp"]) for m in marks}
    for m in marks:
        name = m.get("Function", "")
        if not name.endswith(" x%d" % API_REPS):
            continue
        t0, t1 = int(m["Start_Timestamp"]), int(m["End_Timestamp"])
        t_end = ends.get(name + " end", t1)  # after the caller's synchronisation: every kernel of the range ran
        calls = [a["Function"] for a in api if t0 <= int(a["Start_Timestamp"]) <= t1]
        cells = []
        for label, pred in groups:
            if pred is None:
                continue
            cells.append("%.2f" % (sum(1 for c in calls if pred(c)) / API_REPS))
        ks = sorted((int(k["Start_Timestamp"]), int(k["End_Timestamp"])) for k in kern
                    if t0 <= int(k["Start_Timestamp"]) <= t_end)
        busy = sum(e - b for b, e in ks)
        span = (ks[-1][1] - ks[0][0]) if ks else 0
        out.append("| %s | %s | %.1f | %.1f | %.1f | %.1f |" % (
            name, " | ".join(cells), len(calls) / API_REPS, busy / 1e3 / API_REPS, len(ks) / API_REPS,
            (span - busy) / 1e3 / API_REPS))
    return "\n".join(out)


def layer_alg_bytes(net, batch, h, w, esize, in_esize=None):
    """Algorithmic HBM bytes per conv launch (fused pool included): the input
    read once, the packed weights once and the (pooled) output written once, in
    the storage type with 16-byte channel padding; the first conv reads the
    FP32 NCHW image.  Keyed by the conv's layer index."""
    import synth
    seg = 16 // esize
    pad = lambda c: (c + seg - 1) // seg * seg
    out, c, hh, ww = {}, net.in_c, h, w
    L = net.layers
    for i, l in enumerate(L):
        if l.kind == synth.CONV:
            ho = (hh + 2 * l.pad - l.ksize) // l.stride + 1
            wo = (ww + 2 * l.pad - l.ksize) // l.stride + 1
            pooled = i + 1 < len(L) and L[i + 1].kind == synth.MAXPOOL and L[i + 1].stride == 2 and L[i + 1].ksize == 2
            oh, ow = (ho // 2, wo // 2) if pooled else (ho, wo)
            xin = batch * c * hh * ww * 4 if i == 0 else batch * hh * ww * pad(c) * esize
            wts = pad(l.cout) * l.ksize * l.ksize * pad(c) * esize
            out[i] = xin + wts + batch * oh * ow * pad(l.cout) * esize
            c, hh, ww = l.cout, ho, wo
        elif l.kind == synth.MAXPOOL:
            hh, ww = (hh - 1) // l.stride + 1, (ww - 1) // l.stride + 1
    return out


def summarize_pmc_layers(fetch_csv: str, write_csv: str, driver_json: str, launches: int = 5):
    """HBM bytes per launch of several convs from two rocprofv3 --pmc runs of
    `bench.py --pmc-driver --pmc-layers ...` (FETCH_SIZE, then WRITE_SIZE, KiB
    per dispatch), each scaled by what the counter reads for the driver's
    256 MiB device copy; the last dispatches are the layers' timed launches in
    the driver's order (fill kernels skipped)."""
    import synth
    drv = None
    for line in open(driver_json):
        line = line.strip()
        if line.startswith("{") and "pmc_driver" in line:
            drv = json.loads(line)
    layers, kpl = drv["layers"], drv["kernels_per_launch"]
    net = synth.plain9()
    alg = layer_alg_bytes(net, 64, 416, 416, 2)

    def load(path, counter):
        disp = {}
        for r in _csv_rows(path):
            if r["Counter_Name"] == counter:
                d = disp.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], 0.0])
                d[1] += float(r["Counter_Value"])
        return [disp[k] for k in sorted(disp)]

    res = {"kernel_source_hash": kernel_source_hash(), "batch": 64, "image": [3, 416, 416], "dtype": "bf16"}
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        d = load(path, counter)
        copy = next(v for k, v in d if "copyBuffer" in k)
        factor = copy * 1024.0 / (256 << 20)
        convs = [(k, v) for k, v in d if "fillBuffer" not in k]
        need = sum(launches * n for n in kpl)
        tail = convs[-need:]
        pos = 0
        for layer, n in zip(layers, kpl):
            chunk = tail[pos:pos + launches * n]
            pos += launches * n
            e = per.setdefault(str(layer), {"kernels": sorted({k[:100] for k, _ in chunk}), "factor": {}})
            e["factor"][counter] = factor
            e[counter.lower() + "_bytes_per_launch"] = sum(v for _, v in chunk) / launches * 1024.0 / factor
    for layer, e in per.items():
        e["hbm_bytes_per_launch"] = e["fetch_size_bytes_per_launch"] + e["write_size_bytes_per_launch"]
        e["algorithmic_bytes_per_launch"] = alg[int(layer)]
        e["traffic_over_algorithmic"] = e["hbm_bytes_per_launch"] / alg[int(layer)]
    res["layers"] = per
    return res


def summarize_counters(paths, launches: int = 5):
    """Mean per dispatch of every counter over the last `launches` dispatches
    (the dominant conv's timed launches of `bench.py --pmc-driver`) of one or
    more rocprofv3 --pmc CSVs, with the kernel name and grid."""
    out = {}
    for path in paths:
        disp = {}
        for r in _csv_rows(path):
            d = disp.setdefault(int(r["Dispatch_Id"]), {"kernel": r["Kernel_Name"], "grid": int(r["Grid_Size"]),
                                                       "vgpr": int(r["VGPR_Count"]), "agpr": int(r["Accum_VGPR_Count"]),
                                                       "lds": int(r["LDS_Block_Size"]), "counters": {}})
            d["counters"][r["Counter_Name"]] = d["counters"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        last = [disp[k] for k in sorted(disp)][-launches:]
        assert len({d["kernel"] for d in last}) == 1, "last dispatches are not one kernel"
        out.setdefault("kernel", last[0]["kernel"])
        for key in ("grid", "vgpr", "agpr", "lds"):
            out.setdefault(key, last[0][key])
        for name in last[0]["counters"]:
            out.setdefault("counters", {})[name] = float(np.mean([d["counters"][name] for d in last]))
    return out


def summarize_pmc(fetch_csv: str, write_csv: str, layer: int, tile: int, launches: int = 5):
    """HBM bytes per launch of the dominant conv from two rocprofv3 --pmc runs
    of `bench.py --pmc-driver` (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).
    Each counter is scaled by what it reads for the driver's 256 MiB device
    copy (the first copyBuffer dispatch), and the last `launches` dispatches
    are the dominant conv."""
    def load(path, counter):
        disp = {}
        for r in _csv_rows(path):
            if r["Counter_Name"] == counter:
                d = disp.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], 0.0])
                d[1] += float(r["Counter_Value"])
        return [disp[k] for k in sorted(disp)]

    res = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        d = load(path, counter)
        copy = next(v for k, v in d if "copyBuffer" in k)
        kern = d[-launches:]
        assert len({k for k, _ in kern}) == 1, "last dispatches are not one kernel"
        factor = copy * 1024.0 / (256 << 20)
        res[counter] = {"copy_kib": copy, "factor": factor, "kernel": kern[0][0],
                        "kib_per_launch": float(np.mean([v for _, v in kern])),
                        "bytes_per_launch": float(np.mean([v for _, v in kern])) * 1024.0 / factor}
    total = res["FETCH_SIZE"]["bytes_per_launch"] + res["WRITE_SIZE"]["bytes_per_launch"]
    return {"kernel_source_hash": kernel_source_hash(),
            "layer%d" % layer: {"tile%d" % tile: {"kernel": res["FETCH_SIZE"]["kernel"], "hbm_bytes_per_launch": total,
                                                  "fetch": res["FETCH_SIZE"], "write": res["WRITE_SIZE"]}}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--kernel-iters", type=int, default=50)
    ap.add_argument("--no-ga", action="store_true", help="skip the GA placement search line")
    ap.add_argument("--api-driver", action="store_true",
                    help="run only the steady-state forwards of api_driver (for rocprofv3 --hip-trace "
                         "--marker-trace --kernel-trace)")
    ap.add_argument("--pmc-layers", default="",
                    help="with --pmc-driver: comma-separated conv layers to launch 5 times each (default: the "
                         "dominant conv)")
    ap.add_argument("--summarize-pmc-layers", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "DRIVER_OUTPUT"),
                    help="print the per-layer HBM-traffic JSON of two --pmc-driver --pmc-layers runs and exit")
    ap.add_argument("--summarize-api", metavar="ROCPROF_DIR",
                    help="print the markdown summary of an --api-driver trace directory and exit (no GPU)")
    ap.add_argument("--placement-driver", action="store_true",
                    help="run only the GA placement search (9-layer f32 b1 416x416) and print its JSON")
    ap.add_argument("--pmc-driver", action="store_true",
                    help="run only the dominant conv kernel (5 launches) and a 256 MiB device copy, "
                         "for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs")
    ap.add_argument("--nightmare-driver", action="store_true",
                    help="run only 5 image-modification steps (BF16, batch 64, 416x416), for a kernel trace")
    ap.add_argument("--residual-driver", action="store_true",
                    help="run only 20 graph forwards of the 52-layer residual net (BF16, batch 16, 256x256), "
                         "for a kernel trace")
    ap.add_argument("--summarize-trace", metavar="KERNEL_TRACE_CSV",
                    help="print a markdown summary of a rocprofv3 --kernel-trace CSV and exit (no GPU)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "LAYER", "TILE"),
                    help="print the HBM-traffic JSON of two --pmc-driver counter runs (the dominant conv on "
                         "tile config TILE, as the driver printed it) and exit (no GPU)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="COUNTER_CSV",
                    help="print, per counter, the mean per dispatch over the last 5 dispatches (the dominant "
                         "conv's launches in --pmc-driver runs) of rocprofv3 --pmc CSVs, and exit (no GPU)")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return
    if args.summarize_pmc_layers:
        print(json.dumps(summarize_pmc_layers(*args.summarize_pmc_layers), indent=1))
        return
    if args.summarize_api:
        print(summarize_api(args.summarize_api))
        return
    if args.summarize_counters:
        print(json.dumps(summarize_counters(args.summarize_counters), indent=1))
        return
    if args.summarize_pmc:
        f, w, layer, tile = args.summarize_pmc
        print(json.dumps(summarize_pmc(f, w, int(layer), int(tile)), indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: inference is data-parallel with no per-forward exchange, "
              "so N GPUs would each run this plan on their own share of the images.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1811_03882_amd import dn

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.pmc_driver:
        # reference copy of known size first (its counters calibrate the HBM byte counts)
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    net = synth.plain9()
    params = synth.make_params(net, synth.SEED_PLAIN)
    B, H, W = 64, 416, 416
    x = torch.from_numpy(synth.make_input(net, B, synth.SEED_PLAIN).astype(np.float32)).cuda()
    stream = torch.cuda.Stream()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)

    if args.api_driver:
        api_driver(torch, dn, net, params, x, stream, log=log)
        return

    if args.placement_driver:
        print(json.dumps(placement_search(dn, net, params, np.ascontiguousarray(x[:1].cpu().numpy()), log=log)))
        return

    if args.residual_driver:
        rnet = synth.residual52()
        rparams = synth.make_params(rnet, synth.SEED_RESIDUAL)
        xr = torch.from_numpy(synth.make_input(rnet, 16, synth.SEED_RESIDUAL).astype(np.float32)).cuda()
        n6, a6 = build_net(dn, torch, rnet, dn.BF16, 16, 256, 256, params=rparams)
        yr = torch.empty((16,) + n6.output_shape(256, 256), device="cuda")
        for _ in range(20):
            n6.forward(xr, 16, 256, 256, yr, stream)
        torch.cuda.synchronize()
        print(json.dumps({"residual_driver": True, "forwards": 20, "batch": 16}))
        return
    if args.nightmare_driver:
        n5, a5 = build_net(dn, torch, net, dn.BF16, B, H, W, params, use_graph=False, tune=False)
        n5.autotune_backward(len(net.layers) - 1, B, H, W, stream)
        ga = torch.empty(n5.input_gradient_arena_bytes(len(net.layers) - 1, B, H, W), dtype=torch.uint8, device="cuda")
        n5.bind_arena(ga)
        torch.cuda.synchronize()
        for _ in range(6):
            n5.nightmare(len(net.layers) - 1, x, B, H, W, 0.01, 1, stream)
        torch.cuda.synchronize()
        print(json.dumps({"nightmare_driver": True, "steps": 6, "batch": B}))
        return

    # ---------------- headline: BF16 batch 64, graph-captured forward
    log("[bench] building BF16 b64 net + autotune")
    nb, arena_b = build_net(dn, torch, net, dn.BF16, B, H, W, params)
    if args.pmc_driver:
        flops = conv_flops(net, B, H, W)
        dom = max(flops, key=lambda k: flops[k][0])
        layers = [int(v) for v in args.pmc_layers.split(",") if v.strip()] or [dom]
        nb.forward(x, B, H, W, torch.empty((B,) + nb.output_shape(H, W), device="cuda"), stream)
        torch.cuda.synchronize()
        plans = {}
        for layer in layers:
            nb.time_layer(layer, B, H, W, 5, stream)
            torch.cuda.synchronize()
            plans[layer] = nb.layer_plan(layer, B, H, W)
        print(json.dumps({"pmc_driver": True, "copy_bytes": 256 << 20, "layer": dom, "layers": layers,
                          "kernels_per_launch": [2 if plans[l]["splits"] > 1 else 1 for l in layers],
                          "plan": plans[dom] if dom in plans else None, "plans": plans}))
        return
    out_shape = nb.output_shape(H, W)
    y = torch.empty((B,) + out_shape, dtype=torch.float32, device="cuda")
    fwd = lambda: nb.forward(x, B, H, W, y, stream)
    log("[bench] timing %d steps" % args.steps)
    wall, per = time_steps(torch, fwd, args.steps, args.warmup, stream)
    ms_step = wall * 1e3 / args.steps
    value = B * args.steps / wall
    log("[bench] bf16 b64: %.3f ms/step, %.0f images/s" % (ms_step, value))
    # step latency over 1000 graph replays (events around each replay)
    _, lat_b64 = time_steps(torch, fwd, 1000, 0, stream)
    log("[bench] bf16 b64 latency over 1000 replays: p50 %.3f ms, p99 %.3f ms"
        % (np.percentile(lat_b64, 50), np.percentile(lat_b64, 99)))

    # per-conv kernel times (HIP events on the launch stream), % MFMA; the
    # dominant conv first, so that its launches form one run in a kernel trace
    flops = conv_flops(net, B, H, W)
    dom = max(flops, key=lambda k: flops[k][0])  # the K = 9216 conv
    dom_ms = nb.time_layer(dom, B, H, W, args.kernel_iters, stream)
    per_layer = {}
    for li, (fl, M, N, K) in flops.items():
        ms = dom_ms if li == dom else nb.time_layer(li, B, H, W, args.kernel_iters, stream)
        plan = nb.layer_plan(li, B, H, W)
        per_layer[li] = {"ms": ms, "tflops": fl / (ms * 1e-3) / 1e12, "mfma_pct": 100.0 * fl / (ms * 1e-3) / PEAK["bf16"],
                         "M": M, "N": N, "K": K, "tile": plan["tile"], "splits": plan["splits"]}
        log("[bench]   conv layer %2d M=%6d N=%4d K=%5d tile=%d split=%d  %.4f ms  %.1f TFLOP/s  %.1f%% of BF16 peak"
            % (li, M, N, K, plan["tile"], plan["splits"], ms, per_layer[li]["tflops"], per_layer[li]["mfma_pct"]))
    achieved = flops[dom][0] / (dom_ms * 1e-3)
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["bf16"] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK["bf16"], "traffic": traffic_from_profiles("layer%d" % dom, per_layer[dom]["tile"]),
                "kernel": "conv layer %d bf16, tile config %d (%s): conv3x3 1024->1024 on 13x13, M=%d N=%d K=%d"
                          % (dom, per_layer[dom]["tile"], _tile_desc(dn, per_layer[dom]["tile"]), *flops[dom][1:]),
                "avg_launch_ms": dom_ms}

    # the matrix-core rate the chip sustains at its running clock (MFMA-only kernel)
    measured_peak = {name: dn.mfma_peak(dt) for name, dt in (("bf16", dn.BF16), ("fp8", dn.FP8), ("f32", dn.F32))}
    roofline["measured_mfma_peak"] = measured_peak["bf16"]
    roofline["frac_of_measured_peak"] = roofline["achieved"] / measured_peak["bf16"]
    log("[bench] measured MFMA peak: %s TFLOP/s" % {k: round(v, 1) for k, v in measured_peak.items()})

    cross = None
    if not args.no_secondary:
        # reference points from the vendor libraries (never in the product path):
        # hipBLASLt on the same GEMM shape without the im2col gather, MIOpen's conv
        M, N, K = flops[dom][1:]
        a_m = torch.randn(M, K, device="cuda", dtype=torch.bfloat16)
        b_m = torch.randn(K, N, device="cuda", dtype=torch.bfloat16)
        xc = torch.randn(B, K // 9, 13, 13, device="cuda", dtype=torch.bfloat16).to(memory_format=torch.channels_last)
        wc = torch.randn(N, K // 9, 3, 3, device="cuda", dtype=torch.bfloat16).to(memory_format=torch.channels_last)

        def t_ms(fn, it=30):
            for _ in range(5):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(it):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / it

        mm = t_ms(lambda: torch.matmul(a_m, b_m))
        cv = t_ms(lambda: torch.nn.functional.conv2d(xc, wc, padding=1))
        cross = {"hipblaslt_gemm_same_shape_ms": mm, "hipblaslt_tflops": flops[dom][0] / (mm * 1e-3) / 1e12,
                 "miopen_conv_nhwc_ms": cv, "miopen_tflops": flops[dom][0] / (cv * 1e-3) / 1e12,
                 "this_kernel_ms": dom_ms}
        log("[bench] cross-check: hipBLASLt %.4f ms, MIOpen %.4f ms, this kernel %.4f ms" % (mm, cv, dom_ms))
        del a_m, b_m, xc, wc

    secondary = []
    if not args.no_secondary:
        # PCIe-inclusive rate: pinned host input -> H2D -> forward -> D2H, serialised on one stream
        xh = x.cpu().pin_memory()
        yh = torch.empty(y.shape, dtype=torch.float32).pin_memory()

        def fwd_pcie():
            x.copy_(xh, non_blocking=True)
            nb.forward(x, B, H, W, y, stream)
            yh.copy_(y, non_blocking=True)

        with torch.cuda.stream(stream):
            wp, pp = time_steps(torch, fwd_pcie, 10, 2, stream)
        secondary.append({"workload": "9-layer b64 bf16 graph incl. PCIe (pinned H2D of the FP32 batch + D2H of the output)",
                          "images_per_s": B * 10 / wp, "ms_per_step": wp * 1e3 / 10})
        log("[bench] bf16 b64 incl. PCIe: %.3f ms/step" % (wp * 1e3 / 10))
        # the same with 8-bit frames (a camera's pixels, q / 255 on the device): a quarter of the H2D bytes
        n8, a8 = build_net(dn, torch, net, dn.BF16, B, H, W, params, input_u8=True)
        q = np.random.default_rng([synth.SEED_PLAIN, 9]).integers(0, 256, size=(B, net.in_c, H, W), dtype=np.uint8)
        xh8 = torch.from_numpy(q).pin_memory()
        x8 = torch.empty(xh8.shape, dtype=torch.uint8, device="cuda")

        def fwd_pcie8():
            x8.copy_(xh8, non_blocking=True)
            n8.forward(x8, B, H, W, y, stream)
            yh.copy_(y, non_blocking=True)

        with torch.cuda.stream(stream):
            wp8, _ = time_steps(torch, fwd_pcie8, 10, 2, stream)
            w8, _ = time_steps(torch, lambda: n8.forward(x8, B, H, W, y, stream), 10, 2, stream)
        secondary.append({"workload": "9-layer b64 bf16 graph incl. PCIe, 8-bit frames (pinned H2D of the uint8 batch, "
                                      "converted on the device, + D2H of the output)",
                          "images_per_s": B * 10 / wp8, "ms_per_step": wp8 * 1e3 / 10,
                          "device_resident_images_per_s": B * 10 / w8})
        log("[bench] bf16 b64 incl. PCIe, 8-bit frames: %.3f ms/step (resident %.3f ms)" % (wp8 * 1e3 / 10, w8 * 1e3 / 10))
        n8.close()
        del a8, x8, xh8
        calib = torch.from_numpy(synth.make_input(net, 4, synth.SEED_CALIB).astype(np.float32)).cuda()
        for name, dt in (("fp8", dn.FP8), ("f32", dn.F32)):
            log("[bench] %s b64" % name)
            n2, a2 = build_net(dn, torch, net, dt, B, H, W, params, calib=calib)
            w2, p2 = time_steps(torch, lambda: n2.forward(x, B, H, W, y, stream), max(5, args.steps // 3), 2, stream)
            l13 = n2.time_layer(dom, B, H, W, 20, stream)
            secondary.append({"workload": "9-layer b64 %s graph" % name, "images_per_s": B * len(p2) / w2,
                              "ms_per_step": w2 * 1e3 / len(p2), "p50_ms": float(np.percentile(p2, 50)),
                              "p99_ms": float(np.percentile(p2, 99)), "dominant_conv_ms": l13,
                              "dominant_conv_pct_peak": 100.0 * flops[dom][0] / (l13 * 1e-3) / PEAK[name]})
            n2.close()
            del a2
        # detection post-processing on the device (decode + per-class NMS) for
        # one batch of region outputs of the 9-layer head (64 x 125 x 13 x 13)
        log("[bench] detection post-processing b64")
        A_, C_, md = 5, 20, 50
        yr = torch.from_numpy(synth.region_output(B, A_, C_, 13, 13, tag=64, clusters=3)).cuda()
        wsb = dn.detect_workspace(B, A_, C_, 13, 13)
        wsd = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        dets = torch.empty((B, C_, md, 5), device="cuda")
        didx = torch.empty((B, C_, md), dtype=torch.int32, device="cuda")
        dcnt = torch.empty((B, C_), dtype=torch.int32, device="cuda")
        anc = synth.region_anchors(A_)
        run = lambda: dn.detect(yr, B, A_, C_, 13, 13, anc, 0.2, 0.45, md, wsd, wsb, dets, didx, dcnt, stream)
        with torch.cuda.stream(stream):
            wd, pd = time_steps(torch, run, 50, 5, stream)
        secondary.append({"workload": "detection post-processing, 64 images x 13x13x5 boxes x 20 classes "
                                      "(region decode + per-class greedy NMS, thresh 0.2, IoU 0.45)",
                          "ms_per_batch": float(np.percentile(pd, 50)), "kept_boxes": int(dcnt.sum().item()),
                          "region_tensor_bytes": int(yr.numel() * 4),
                          "kept_box_bytes": int(dcnt.sum().item()) * 24})
        log("[bench] detection: %.4f ms per batch, %d boxes kept" % (np.percentile(pd, 50), int(dcnt.sum().item())))
        del yr, wsd, dets, didx, dcnt

        # Jacobi/Laplace (the paper's second example of the transfer rule):
        # 4096 x 4096 FP64 grid, device-resident vs copied across PCIe every iteration
        log("[bench] jacobi 4096x4096")
        nj = 4096
        uj = torch.zeros((nj, nj), dtype=torch.float64, device="cuda")
        uj[0, :] = 1.0
        wj = torch.empty_like(uj)
        it_res = 200
        with torch.cuda.stream(stream):
            dn.jacobi(uj, wj, nj, nj, 10, None, stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dn.jacobi(uj, wj, nj, nj, it_res, None, stream)
            e1.record(stream)
            torch.cuda.synchronize()
        ms_res = e0.elapsed_time(e1) / it_res
        uh = np.zeros((nj, nj), np.float64)
        uh[0, :] = 1.0
        t0 = time.perf_counter()
        it_pl = 5
        dn.jacobi_per_iteration(uh, uj, wj, it_pl, stream)
        ms_pl = (time.perf_counter() - t0) * 1e3 / it_pl
        jbytes = 2 * 8 * nj * nj
        secondary.append({"workload": "Jacobi/Laplace 4096x4096 FP64: device-resident vs per-iteration transfer",
                          "resident_ms_per_iteration": ms_res, "per_iteration_transfer_ms_per_iteration": ms_pl,
                          "speedup_resident": ms_pl / ms_res,
                          "roofline": {"bound": "hbm", "achieved": jbytes / (ms_res * 1e-3) / 1e9, "peak": 8000.0,
                                       "unit": "GB/s", "frac": jbytes / (ms_res * 1e-3) / 8e12,
                                       "algorithmic_bytes_per_iteration": jbytes}})
        log("[bench] jacobi: resident %.4f ms/iter, per-iteration transfer %.3f ms/iter" % (ms_res, ms_pl))
        del uj, wj, uh

        # Deep residual CNN (52 convs, 23 shortcuts), BF16, batch 16, 3x256x256
        log("[bench] residual52 bf16 b16")
        rnet = synth.residual52()
        rparams = synth.make_params(rnet, synth.SEED_RESIDUAL)
        RB, RH = 16, 256
        xr = torch.from_numpy(synth.make_input(rnet, RB, synth.SEED_RESIDUAL).astype(np.float32)).cuda()
        n6, a6 = build_net(dn, torch, rnet, dn.BF16, RB, RH, RH, params=rparams)
        yr6 = torch.empty((RB,) + n6.output_shape(RH, RH), device="cuda")
        w6, p6 = time_steps(torch, lambda: n6.forward(xr, RB, RH, RH, yr6, stream), 200, 10, stream)
        rfl = sum(v[0] for v in conv_flops(rnet, RB, RH, RH).values())
        ms6 = float(np.mean(p6))
        secondary.append({"workload": "52-layer residual CNN bf16 b16 3x256x256 graph (stem, 5 stride-2 stages, 23 units)",
                          "images_per_s": RB * len(p6) / w6, "ms_per_step": w6 * 1e3 / len(p6),
                          "p50_ms": float(np.percentile(p6, 50)), "p99_ms": float(np.percentile(p6, 99)),
                          "gflop_per_batch": rfl / 1e9, "conv_tflops": rfl / (ms6 * 1e-3) / 1e12,
                          "conv_pct_peak": 100.0 * rfl / (ms6 * 1e-3) / PEAK["bf16"]})
        log("[bench] residual52: %.3f ms per batch of 16" % ms6)
        n6.close()
        del a6, xr, yr6

        # Single conv block, FP32, 1x3x32x32 (launch-bound: latency only)
        snet = synth.single_block()
        sparams = synth.make_params(snet, synth.SEED_SINGLE)
        xs = torch.from_numpy(synth.make_input(snet, 1, synth.SEED_SINGLE).astype(np.float32)).cuda()
        n7, a7 = build_net(dn, torch, snet, dn.F32, 1, 32, 32, params=sparams)
        ys = torch.empty((1,) + n7.output_shape(32, 32), device="cuda")
        _, p7 = time_steps(torch, lambda: n7.forward(xs, 1, 32, 32, ys, stream), 1000, 20, stream)
        secondary.append({"workload": "single conv block f32 1x3x32x32 graph (conv3x3 16 + BN + leaky + pool)",
                          "p50_ms": float(np.percentile(p7, 50)), "p99_ms": float(np.percentile(p7, 99)),
                          "replays": len(p7)})
        n7.close()
        del a7, xs, ys

        # Image modification (the workload's second program): one gradient-ascent
        # step on the energy of the last layer = unfused forward keeping every
        # layer output + backward to the image + update, batch 64 at 416x416
        fl_all = sum(v[0] for v in flops.values())
        for name, dt in (("bf16", dn.BF16), ("f32", dn.F32)):
            log("[bench] nightmare %s b64" % name)
            n5, a5 = build_net(dn, torch, net, dt, B, H, W, params, use_graph=False, tune=False)
            xn = x.clone()
            last = len(net.layers) - 1
            n5.autotune_backward(last, B, H, W, stream)
            ga = torch.empty(n5.input_gradient_arena_bytes(last, B, H, W), dtype=torch.uint8, device="cuda")
            n5.bind_arena(ga)
            run = lambda: n5.nightmare(last, xn, B, H, W, 0.01, 1, stream)
            with torch.cuda.stream(stream):
                wn, pn = time_steps(torch, run, 5, 1, stream)
            ms = wn * 1e3 / len(pn)
            secondary.append({"workload": "image modification, 9-layer %s b64 416x416: gradient ascent on the last "
                                          "layer's energy (forward keeping every output + backward to the image + update)" % name,
                              "images_per_s": B * len(pn) / wn, "ms_per_step": ms,
                              "conv_tflops": 2 * fl_all / (ms * 1e-3) / 1e12,
                              "conv_pct_peak": 100.0 * 2 * fl_all / (ms * 1e-3) / PEAK[name]})
            log("[bench] nightmare %s: %.3f ms per step" % (name, ms))
            n5.close()
            del a5, xn, ga

        # FP32 plain path, batch 1: resident (graph) vs per-layer transfers
        x1 = x[:1].contiguous()
        y1 = torch.empty((1,) + out_shape, dtype=torch.float32, device="cuda")
        log("[bench] f32 b1 resident")
        n3, a3 = build_net(dn, torch, net, dn.F32, 1, H, W, params)
        w3, p3 = time_steps(torch, lambda: n3.forward(x1, 1, H, W, y1, stream), 1000, 10, stream)
        secondary.append({"workload": "9-layer b1 f32 resident graph", "images_per_s": len(p3) / w3,
                          "p50_ms": float(np.percentile(p3, 50)), "p99_ms": float(np.percentile(p3, 99)),
                          "replays": len(p3)})
        n3.close()
        log("[bench] f32 b1 per-layer transfer")
        n4, a4 = build_net(dn, torch, net, dn.F32, 1, H, W, params, use_graph=False, tune=False, mode=dn.PER_LAYER)
        xh = np.ascontiguousarray(x1.cpu().numpy())
        yh = np.empty((1,) + out_shape, np.float32)
        n4.forward(xh, 1, H, W, yh)
        lat = []
        for _ in range(20):
            t0 = time.perf_counter()
            n4.forward(xh, 1, H, W, yh)
            lat.append((time.perf_counter() - t0) * 1e3)
        secondary.append({"workload": "9-layer b1 f32 per-layer-transfer (host in/out, 15 layers x H2D+D2H+sync)",
                          "images_per_s": 1e3 / float(np.mean(lat)), "p50_ms": float(np.percentile(lat, 50)),
                          "p99_ms": float(np.percentile(lat, 99))})
        n4.close()
        if not args.no_ga:
            secondary.append(placement_search(dn, net, params, xh, log=log))

    serving_res = None
    if not args.no_serving and not args.no_secondary:
        serving_res = serving(torch, dn, log=log)

    cpu = None
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline()

    rec = {
        "metric": METRIC, "value": value, "unit": "images/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic (seeded inputs, random-init weights)",
        "config": {"workload": "9-layer plain CNN (Darknet-style), batch 64, 3x416x416, BF16 MFMA / FP32 accumulate, "
                               "BN folded in FP64, hipGraph forward, autotuned tiles",
                   "global_batch": B, "image": [3, H, W], "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(lat_b64, 50)), "p99": float(np.percentile(lat_b64, 99)),
                       "replays": len(lat_b64)},
        "roofline": roofline,
        "mfma_measured_peak_tflops": measured_peak,
        "dominant_conv_cross_check": cross,
        "cpu_baseline": cpu,
        "per_conv": {str(k): v for k, v in per_layer.items()},
        "secondary": secondary,
        "serving": serving_res,
        "kernel_source_hash": kernel_source_hash(),
        "paper_context": "3x over CPU-only for the whole Darknet application (108.28 s -> 36.28 s) on an NVIDIA "
                         "Quadro K5200 with PGI 17.10 OpenACC; context only",
    }
    print(json.dumps(rec), flush=True)
    nb.close()


if __name__ == "__main__":
    main()
