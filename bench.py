"""Lloyd iterations per second on one MI355X.

Workload (default): n = 4,000,000 points in d = 512 from a 1,000-component
Gaussian mixture (means N(0, 4I), sigma_c uniform in [0.5, 1.5], row i in
component i mod 1000), k = 1000, k-means++ seeding (seed 0), W = 5 plain FP32
Lloyd iterations whose labels train the candidate router (1 epoch over the
5 n pairs, batch 8192, Adam lr 1e-3), then K = 15 timed Lloyd iterations
(iterations 6..20) from the same centers on every exact path: router
proposals + certificate (BF16 or FP8 GEMM for the other rows), the same with
bounds carried across iterations, the non-learned forms (bounds + previous
label, previous label alone), the full BF16 / FP8 / FP32 GEMM paths, eager and
replayed as a graph.  Each path is timed --repeats times (median reported);
each timed call includes the router's forward pass (one per call) and the
final assignment.  `value` is the fastest path that uses the router (the
method's router + mixed-precision form), reported only when every path
returned identical labels and centers and its final cost equals the FP32
path's within 1e-6 relative; the fastest path overall is reported beside it.

Prints ONE JSON line.  Data is synthetic and generated on the device before
the timed region; seeding, the plain iterations, training and the oracle
(FP64 CPU timing and the FP64 errors of the reported results) are outside it.
--workload rotated|streamed|batched|piecy|small prints the other workloads'
lines;
--only assign and --traffic are the counter-collection modes.
"""
from __future__ import annotations

import argparse
import re
import hashlib
import glob
import csv
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Lloyd iter/s (n=4M,d=512,k=1000) vs plain FP32 GPU, equal cost ±1e-6 rel"
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 MFMA
FP8_PEAK_TFLOPS = 5000.0     # MI355X dense FP8 MFMA
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 matrix
HBM_PEAK_GBS = 8000.0

STREAMED = dict(n=10_000_000, d_in=4096, r=64, k=100, chunk=65536, sample=100_000,
                name="rank-64 signal in d=4096 + N(0,0.05^2) noise, n=1e7 in chunks of 65536, "
                     "projected to 64 dims, k=100")

PIECY = dict(ell=50, y=4000, d=1000, x=50, k=50, svd=64, piece=20000, np_=4,
             name="StructuredWithNoise l=50 y=4000 (n=2e5) d=1000 x=50 (Delta=10, delta=0.5), "
                  "k=50, projected to 64 dims")

WORKLOADS = {
    "router": dict(n=4_000_000, d=512, k=1000, name="gaussian mixture n=4e6 d=512 k=1000 "
                   "(means N(0,4I), sigma U[0.5,1.5])"),
    "small": dict(n=10_000, d=64, k=10, name="isotropic mixture n=1e4 d=64 k=10 "
                  "(means U[-10,10]^64, sigma 1)"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(key):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes, scaled by the copy-kernel calibration; None once the kernel source
    no longer matches the hash recorded with the counters."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "assign_traffic_n4m_d512_k1000.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, rec["kernel_source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != rec["kernel_source_sha256"]:
            return None
        return rec[key]["hbm_bytes"]
    except (OSError, KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# HBM traffic of the assignment GEMMs from two rocprofv3 counter passes over
# `bench.py --only assign` (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch):
#   python bench.py --traffic <fetch_dir> <write_dir> <out.json>
# The three plain 1 GiB device copies at the end of that mode calibrate both
# counters (bytes moved / counter value); for each precision the full-size
# GEMM dispatches (largest grid of that kernel) are averaged.  The record
# carries the sha256 of the kernel source, so the headline stops reporting the
# traffic once the kernel changes.
# ---------------------------------------------------------------------------
TRAFFIC_SOURCE = "paper_1502_04265_amd/csrc/k_assign.hip"
TRAFFIC_MODES = {0: "assign_fp32", 1: "assign_bf16", 2: "assign_fp8"}


def _traffic_rows(d):
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        out.extend(csv.DictReader(open(f)))
    return out


def _traffic_by_kernel(rows):
    gemm, copies = {}, []
    for r in rows:
        name, val, grid = r["Kernel_Name"], float(r["Counter_Value"]), int(r["Grid_Size"])
        m = re.search(r"assign_kernel<(\d+),", name)
        if m:
            gemm.setdefault(int(m.group(1)), []).append((grid, val))
        elif "copyBuffer" in name or "copy" in name.lower():
            copies.append((int(r["Dispatch_Id"]), grid, val))
    return gemm, copies


def traffic_convert(fetch_dir, write_dir):
    fg, fc = _traffic_by_kernel(_traffic_rows(fetch_dir))
    wg, wc = _traffic_by_kernel(_traffic_rows(write_dir))
    gib_kib = 1 << 20

    def calib(copies, full):
        # the three 1 GiB copies are the last copies of the largest grid
        big = max(g for _, g, _ in copies)
        vals = [v for _, g, v in sorted(copies) if g == big][-3:]
        return full / (sum(vals) / len(vals)), sum(vals) / len(vals)

    ff, fcopy = calib(fc, gib_kib)
    wf, wcopy = calib(wc, gib_kib)
    rec = {"kernel_source": TRAFFIC_SOURCE,
           "kernel_source_sha256": hashlib.sha256(open(os.path.join(ROOT, TRAFFIC_SOURCE), "rb").read()).hexdigest(),
           "fetch_factor": ff, "write_factor": wf,
           "copy_1GiB": {"fetch_kib": fcopy, "write_kib": wcopy}}
    for mode, key in TRAFFIC_MODES.items():
        if mode not in fg or mode not in wg:
            continue
        def full_mean(v):
            g = max(x for x, _ in v)
            sel = [y for x, y in v if x == g]
            return sum(sel) / len(sel)
        fk, wk = full_mean(fg[mode]), full_mean(wg[mode])
        rec[key] = {"fetch_kib": fk, "write_kib": wk, "hbm_bytes": (fk * ff + wk * wf) * 1024.0}
    return rec


# ---------------------------------------------------------------------------
# HBM traffic of the exact re-check on the headline path, from two counter
# passes (FETCH_SIZE, then WRITE_SIZE) over
#   bench.py --paths bounded_routed_fp8 --repeats 1 ...
# with the kernel filter "reset_small_kernel|bounds_test_kernel|recheck_|
# assign_kernel<2": every assignment begins with reset_small_kernel, so the
# dispatches split into assignments; the bounded call is its first assignment
# (the full-grid FP8 pass) followed by the run of assignments that hold a
# bound test.  The counters are scaled by the copy calibration of the
# assignment traffic record taken in the same session, and divided by the
# entries the run's JSON line reports for that path:
#   python bench.py --traffic-recheck <fetch_dir> <write_dir> <fetch_run_stdout> <out.json>
# ---------------------------------------------------------------------------
RECHECK_SOURCE = "paper_1502_04265_amd/csrc/k_recheck.hip"


def _recheck_bytes(d):
    rows = _traffic_rows(d)
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    segs, cur = [], None
    for r in rows:
        name = r["Kernel_Name"]
        if "reset_small_kernel" in name:
            cur = {"bounds": False, "kib": 0.0, "launches": 0}
            segs.append(cur)
        elif cur is not None:
            if "bounds_test_kernel" in name:
                cur["bounds"] = True
            elif "recheck_" in name:
                cur["kib"] += float(r["Counter_Value"])
                cur["launches"] += 1
    first = next(i for i, s in enumerate(segs) if s["bounds"])
    last = first
    while last + 1 < len(segs) and segs[last + 1]["bounds"]:
        last += 1
    call = segs[max(first - 1, 0):last + 1]
    return sum(s["kib"] for s in call), len(call), sum(s["launches"] for s in call)


def traffic_recheck_convert(fetch_dir, write_dir, run_stdout):
    cal = json.load(open(os.path.join(ROOT, "profiles", "assign_traffic_n4m_d512_k1000.json")))
    line = [l for l in open(run_stdout) if l.startswith("{")][-1]
    rec = json.loads(line)
    entries = rec["paths"]["bounded_routed_fp8"]["short_recheck_entries"]
    d = rec["config"]["d"]
    fk, nseg, nl = _recheck_bytes(fetch_dir)
    wk, _, _ = _recheck_bytes(write_dir)
    hbm = (fk * cal["fetch_factor"] + wk * cal["write_factor"]) * 1024.0
    return {"kernel_source": RECHECK_SOURCE,
            "kernel_source_sha256": hashlib.sha256(
                open(os.path.join(ROOT, RECHECK_SOURCE), "rb").read()).hexdigest(),
            "calibration": "fetch_factor / write_factor of assign_traffic_n4m_d512_k1000.json",
            "fetch_kib": fk, "write_kib": wk, "assignments": nseg, "launches": nl,
            "entries": entries, "hbm_bytes": hbm,
            "hbm_bytes_per_entry": hbm / max(entries, 1),
            "algorithmic_bytes_per_entry": 4.0 * d + 24}


def measured_recheck_traffic(entries, steps):
    """HBM bytes per step of the exact re-check from the committed counter
    record (bytes per listed entry x entries per step); None once the kernel
    source no longer matches the hash recorded with the counters."""
    path = os.path.join(ROOT, "profiles", "recheck_traffic_n4m_d512_k1000.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, rec["kernel_source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != rec["kernel_source_sha256"]:
            return None
        return rec["hbm_bytes_per_entry"] * entries / steps
    except (OSError, KeyError, ValueError):
        return None


def host_cpu():
    """Host CPU model and the threads the process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": model, "nproc": usable}


def library_reference():
    """What plain library work reaches on this part, timed once: a streaming
    read (torch sum) and a copy of 4 GiB, and square 8192 GEMMs in BF16 and
    FP8 E4M3 through torch (hipBLASLt).  Context beside the datasheet peaks
    the rooflines use, not a ceiling: the reduction here reads faster than
    torch's sum."""
    import torch
    dev = "cuda:0"
    out = {}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    x = torch.ones(1 << 30, dtype=torch.float32, device=dev)      # 4 GiB
    y = torch.empty_like(x)
    nb = x.numel() * 4
    out["hbm_read_gbs"] = nb / timed(lambda: x.sum(), 5) / 1e9
    out["hbm_copy_gbs"] = 2 * nb / timed(lambda: y.copy_(x), 5) / 1e9
    del x, y
    m = 8192
    g = torch.Generator(device=dev).manual_seed(0)
    a = torch.randn(m, m, device=dev, generator=g).to(torch.bfloat16)
    b = torch.randn(m, m, device=dev, generator=g).to(torch.bfloat16)
    out["bf16_gemm_tflops"] = 2 * m ** 3 / timed(lambda: torch.mm(a, b), 10) / 1e12
    try:
        f8 = torch.float8_e4m3fn
        a8 = a.to(f8)
        b8 = b.to(f8)                   # rows of b8 are the columns of the product
        one = torch.ones((), device=dev)
        out["fp8_gemm_tflops"] = 2 * m ** 3 / timed(
            lambda: torch._scaled_mm(a8, b8.t(), scale_a=one, scale_b=one,
                                     out_dtype=torch.bfloat16), 10) / 1e12
    except (RuntimeError, AttributeError, TypeError) as e:
        out["fp8_gemm_tflops"] = None
        out["fp8_note"] = str(e)[:120]
    del a, b
    torch.cuda.empty_cache()
    out["what"] = ("torch sum / copy of 4 GiB FP32; 8192^3 torch.mm (BF16) and _scaled_mm "
                   "(FP8 E4M3) through hipBLASLt")
    return out


def _oracle_chunk(args):
    """One worker of the all-core oracle timing: assignment + clustering
    features of a block of rows (plain oracle calls)."""
    rows, C = args
    from oracle import kmeans as ok
    lab, _, _ = ok.assign(rows, C)
    ok.clustering_features(rows, None, lab, C.shape[0])
    return len(rows)


def cpu_baseline(X_host_rows, C_host, n_full, seconds_target=10.0, gpu_labels=None):
    """Times the FP64 oracle (assignment + update of one Lloyd iteration) on a
    bounded row sample, on one core and on every usable core (a process per
    core, each running the oracle on its share of the rows), and scales to the
    full n.  With gpu_labels (the path's labels of the same rows against the
    same centers), also counts the rows whose label differs from the oracle's
    outside its 1e-6 relative top-2 margin."""
    import multiprocessing as mp
    import numpy as np
    from oracle import kmeans as ok

    rows = X_host_rows
    t0 = time.perf_counter()
    probe = rows[:100]
    lab, _, _ = ok.assign(probe, C_host)
    ok.update(probe, None, lab, C_host)
    t_probe = time.perf_counter() - t0
    m = int(min(len(rows), max(100, 100 * seconds_target / max(t_probe, 1e-6))))
    sample = rows[:m]
    t0 = time.perf_counter()
    lab, d1, d2 = ok.assign(sample, C_host)
    ok.update(sample, None, lab, C_host)
    t = time.perf_counter() - t0
    sec_per_iter = t * n_full / m
    host = host_cpu()
    res = {"value": 1.0 / sec_per_iter, "unit": "iter/s", "cores": 1, "kind": "oracle",
           "sample": f"one Lloyd iteration (FP64 assign + update) on {m} of {n_full} rows, "
                     f"all {C_host.shape[0]} centers; {t:.1f} s measured on one core, scaled by n",
           "sec_per_iter": sec_per_iter, "host": host}
    # every usable core: one process per core on equal shares of a larger sample
    # (at most 16: the CPU share of one GPU on the boxes this runs on)
    cores = max(1, min(16, int(host["nproc"] or 1)))
    if cores > 1:
        m_all = int(min(len(rows), m * cores))
        step = (m_all + cores - 1) // cores
        shares = [(rows[a:min(a + step, m_all)], C_host) for a in range(0, m_all, step)]
        # fresh interpreters: the workers import only NumPy and the oracle
        ctx = mp.get_context("spawn")
        with ctx.Pool(processes=cores) as pool:
            pool.map(_oracle_chunk, [(r[:50], c) for r, c in shares])   # warm the workers
            t0 = time.perf_counter()
            done = sum(pool.map(_oracle_chunk, shares))
            t_all = time.perf_counter() - t0
        res["all_cores"] = {"value": done / (t_all * n_full), "unit": "iter/s", "cores": cores,
                            "sample": f"{done} rows in {cores} processes, {t_all:.1f} s wall, "
                                      f"scaled by n"}
    if gpu_labels is not None:
        g = np.asarray(gpu_labels[:m])
        bad = (g != lab) & ~((d2 - d1) < 1e-6 * d2)
        res["label_check"] = {"rows": m, "differ_outside_margin": int(bad.sum()),
                              "inside_margin": int(((d2 - d1) < 1e-6 * d2).sum())}
    return res


def fp64_errors(X_host, labels, C_T, cost_T, C_next, k):
    """Errors of a path's results against the FP64 oracle on the same
    partition: cost(C_T) from the clustering features of the final labels
    (Sec. 2.1), and the centroids of that partition (the next update)."""
    import numpy as np
    from oracle import kmeans as ok

    Cn, W, S, Q = ok.update(X_host, None, labels, C_T)
    cost_o = ok.cost_from_features(W, S, Q, C_T)
    G = np.asarray(C_next, dtype=np.float64)
    rel = [float(np.linalg.norm(G[j] - Cn[j]) / max(np.linalg.norm(Cn[j]), 1e-3))
           for j in range(k)]
    return {"cost_rel_err": abs(cost_T - cost_o) / cost_o, "cost_oracle": cost_o,
            "centroid_rel_err_max": max(rel), "centroid_rel_err_mean": float(np.mean(rel)),
            "what": "final cost and the centroids of the final labels against the FP64 oracle "
                    "(clustering features of the same partition, all rows)"}


def batched_main(args):
    """Many uneven weighted instances: n ~ U[1e3, 2e5], d in {16..512}, k ~ U[5, 200],
    log-normal(0,1) weights, Gaussian-mixture points; weighted k-means++ per
    instance, tile shapes from the autotuner, then the batched Lloyd loop (one
    assignment launch per width group, iteration replayed as a graph) against
    the same iterations run instance by instance."""
    import numpy as np
    import torch

    import synth
    from paper_1502_04265_amd import kmx

    dev = "cuda:0"
    torch.cuda.set_device(0)
    ctx = kmx.Context(0)
    descs = synth.uneven_instances(args.instances, seed=0)
    log(f"[bench] generating {len(descs)} instances, sum n = {sum(d['n'] for d in descs)}")
    data = []
    for i, desc in enumerate(descs):
        X, w = synth.instance_device(desc, device=dev)
        data.append({"X": X, "k": desc["k"], "w": w})
    torch.cuda.synchronize()
    # k-means++ of every instance: one batched call (round r of all instances
    # with k > r in one launch), and instance by instance for comparison
    ctx.seed_batched(data[:2], [0, 1])                            # buffers
    t0 = time.perf_counter()
    seeded = ctx.seed_batched(data, list(range(len(data))))
    torch.cuda.synchronize()
    seed_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    single = [ctx.seed(p["X"], p["k"], w=p["w"], rng_seed=i) for i, p in enumerate(data)]
    torch.cuda.synchronize()
    seed_single_s = time.perf_counter() - t0
    seed_same = all(torch.equal(a[1], b[1]) for a, b in zip(seeded, single))
    log(f"[bench] seeding: batched {seed_s:.3f} s, one by one {seed_single_s:.3f} s, "
        f"identical {seed_same}")
    probs = [{"X": p["X"], "C": c[0], "w": p["w"]} for p, c in zip(data, seeded)]
    # autotuner cache (JSON lines keyed by device); KMX_TILE_CACHE overrides
    cache = os.environ.get("KMX_TILE_CACHE",
                           os.path.join(tempfile.gettempdir(), "kmx_batched_tiles.jsonl"))
    os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
    t0 = time.perf_counter()
    loaded = ctx.batched_autotune(probs, cache)
    tune_s = time.perf_counter() - t0
    log(f"[bench] seeding {seed_s:.2f} s, autotune {tune_s:.2f} s (cache {'hit' if loaded else 'written'})")
    ctx.lloyd_batched(probs, 1, labels=False)                   # warmup (graph, buffers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.lloyd_batched(probs, args.steps, labels=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] batched: {wall * 1e3 / args.steps:.3f} ms per iteration of all instances")
    t0 = time.perf_counter()
    seq = []
    for p in probs:
        seq.append(ctx.lloyd(p["X"], p["C"], args.steps, w=p["w"], prec="bf16", labels=True))
    torch.cuda.synchronize()
    wseq = time.perf_counter() - t0
    log(f"[bench] one by one: {wseq * 1e3 / args.steps:.3f} ms per iteration of all instances")
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) for a, b in zip(res, seq))
    rel = max(abs(a[2][-1] - b[2][-1]) / max(b[2][-1], 1e-300) for a, b in zip(res, seq))
    flops = sum(2.0 * d["n"] * d["k"] * d["d"] for d in descs)
    # bytes one iteration moves at least: the BF16 copy of every row and its
    # label (the assignment), plus the first update's full pass over the FP32
    # rows spread over the timed iterations (later updates read only the rows
    # whose label changed, not counted)
    it_bytes = sum(d["n"] * (2.0 * d["d"] + 8.0) + d["n"] * (4.0 * d["d"] + 4.0) / args.steps
                   for d in descs)
    it_gbs = it_bytes / (wall / args.steps) / 1e9
    tiles = {}
    for d in descs:
        t, ppb = ctx.batched_tiles(d["d"], d["k"])
        tiles[f"d={d['d']},k<={24 if d['k'] <= 24 else (96 if d['k'] <= 96 else 200)}"] = [t, ppb]
    out = {
        "metric": "batched Lloyd: iterations/s of all instances together",
        "value": args.steps / wall, "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"{len(descs)} weighted instances, n U[1e3,2e5], d in "
                               f"{{16..512}}, k U[5,200], log-normal weights",
                   "sum_n": sum(d["n"] for d in descs), "sum_k": sum(d["k"] for d in descs)},
        "one_by_one": {"iter_per_s": args.steps / wseq, "ms_per_step": wseq * 1e3 / args.steps},
        "speedup_vs_one_by_one": wseq / wall,
        "identical_to_one_by_one": bool(same), "max_final_cost_rel_diff": rel,
        "roofline": {"bound": "hbm", "achieved": it_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": it_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole batched iteration (one captured graph; delta update after the first)",
                     "algorithmic_bytes": it_bytes},
        "assign_flops_per_iteration": flops,
        "whole_iteration_tflops": flops / (wall / args.steps) / 1e12,
        "prepared_inputs": "the timed call reuses the grouped rows, weights and row statistics "
                           "the warm-up call made for the same problems (one by one, each call "
                           "prepares its own copy: the context keeps one X)",
        "tiles": tiles, "seed_s": seed_s, "seed_one_by_one_s": seed_single_s,
        "seed_identical_to_one_by_one": seed_same, "autotune_s": tune_s,
    }
    print(json.dumps(out), flush=True)


def rotated_main(args):
    """Plain vs mixed precision on the largest SWN / Random shape of the
    paper's experiments (n = 1,000,000 points in d = 1000, k = 50): a
    50-component mixture with a random rotation and log-uniform eigenvalues per
    component, k-means++ (seed 0), then --steps Lloyd iterations (default 50)
    from the same centers on the plain FP32 path and on the BF16 / FP8 paths
    with the exact re-check (and with carried bounds).  `value` is the BF16
    path, valid only when every path returns the same labels, centers and
    cost."""
    import torch

    import synth
    from paper_1502_04265_amd import kmx

    n, d, k = 1_000_000, 1000, 50
    steps = args.steps if args.steps_given else 50
    dev = "cuda:0"
    torch.cuda.set_device(0)
    ctx = kmx.Context(0)
    log(f"[bench] generating rotated mixture {n}x{d}, {k} components")
    X, _ = synth.rotated_mixture_device(n, d, k, seed=0, device=dev)
    torch.cuda.synchronize()
    C0, _ = ctx.seed(X, k, rng_seed=0)
    for prec in ("bf16", "fp8", "fp32"):
        ctx.lloyd(X, C0, 1, prec=prec, labels=False)           # quantized copies, buffers
    res, paths = {}, {}

    def run(name, fn, dtype):
        walls, kts, out = [], [], None
        for _ in range(args.repeats):
            ctx.timing(True, True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t)
            kts.append(ctx.timing_read())
            ctx.timing(False, True)
        order = sorted(range(len(walls)), key=lambda q: walls[q])
        med = order[len(order) // 2]
        res[name] = out
        kk = kts[med]
        paths[name] = {"iter_per_s": steps / walls[med], "ms_per_step": walls[med] * 1e3 / steps,
                       "ms_per_step_runs": [w * 1e3 / steps for w in walls],
                       "final_cost": out[2][-1], "dtype": dtype,
                       "kernel_ms_per_step": {c: v[0] / steps for c, v in kk.items() if v[1]},
                       "assign_avg_ms": kk["assign"][0] / max(kk["assign"][1], 1),
                       "reduce_avg_ms": kk["reduce"][0] / max(kk["reduce"][1], 1)}
        log(f"[bench] {name}: {walls[med] * 1e3 / steps:.3f} ms/iter, cost {out[2][-1]:.9e}")

    run("fp32", lambda: ctx.lloyd(X, C0, steps, prec="fp32"), "f32")
    run("bf16", lambda: ctx.lloyd(X, C0, steps, prec="bf16"), "bf16")
    run("fp8", lambda: ctx.lloyd(X, C0, steps, prec="fp8"), "fp8e4m3")
    run("bounded_bf16", lambda: ctx.lloyd_bounded(X, C0, steps, prec="bf16"), "bf16")
    ctx.lloyd(X, C0, 1, prec="bf16", labels=False, graph=True)
    run("bf16_graph", lambda: ctx.lloyd(X, C0, steps, prec="bf16", graph=True), "bf16")
    same = all(torch.equal(r[1], res["fp32"][1]) and torch.equal(r[0], res["fp32"][0])
               for r in res.values())
    base = paths["fp32"]["final_cost"]
    for p in paths.values():
        p["equal_cost_rel_diff"] = abs(p["final_cost"] - base) / base
    best = "bf16"
    valid = bool(same and paths[best]["equal_cost_rel_diff"] <= 1e-6)
    dp = (d + 31) // 32 * 32
    a_ms = paths["bf16"]["assign_avg_ms"]
    a_bytes = n * (2.0 * dp + 16 + 4)          # BF16 rows, row statistics, labels
    # the full reduction alone (kmx_update sums every row; inside Lloyd the
    # later updates take the delta path)
    ctx.update(X, res["bf16"][1], res["bf16"][0])
    ctx.timing(True, True)
    for _ in range(3):
        ctx.update(X, res["bf16"][1], res["bf16"][0])
    kr = ctx.timing_read()
    ctx.timing(False, True)
    r_ms = kr["reduce"][0] / max(kr["reduce"][1], 1)
    r_bytes = n * (4.0 * d + 4)
    out = {
        "metric": "Lloyd iter/s (n=1e6,d=1000,k=50), BF16 MFMA + exact re-check vs plain FP32, "
                  "equal cost",
        "value": paths[best]["iter_per_s"] if valid else 0.0, "unit": "iter/s", "n_gpus": 1,
        "steps": steps, "warmup": 1, "ms_per_step": paths[best]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "rotated gaussian mixture n=1e6 d=1000 k=50 (means U[-5,5]^d, "
                               "Haar rotation, eigenvalues 10^U[-2,0])", "n": n, "d": d, "k": k,
                   "path": best, "timed": f"{steps} Lloyd iterations from the k-means++ centers, "
                                          f"median of {args.repeats} runs"},
        "valid": valid, "identical_paths": bool(same),
        "roofline": {"bound": "hbm", "achieved": a_bytes / (a_ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": a_bytes / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "assign_kernel<bf16> (2 k flop per BF16 row byte: HBM-bound)",
                     "avg_ms": a_ms, "algorithmic_bytes": a_bytes},
        "update_roofline": {"bound": "hbm", "achieved": r_bytes / (r_ms * 1e-3) / 1e9,
                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": r_bytes / (r_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                            "kernel": "cf_reduce_kernel, full update", "avg_ms": r_ms},
        "paths": paths,
        "speedup_vs_fp32": paths[best]["iter_per_s"] / paths["fp32"]["iter_per_s"],
        "fastest_path": max(paths, key=lambda q: paths[q]["iter_per_s"]),
    }
    if not args.no_cpu_baseline:
        lab_b, Cb_ = res[best][1], res[best][0]
        rows = X[:200000].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(rows, Cb_.cpu().numpy(), n,
                                           gpu_labels=lab_b[:200000].cpu().numpy())
        del rows
        C_next, _, _ = ctx.update(X, lab_b, Cb_)
        out["fp64_error"] = fp64_errors(X.cpu().numpy(), lab_b.cpu().numpy(),
                                        Cb_.cpu().numpy().astype("float64"),
                                        paths[best]["final_cost"], C_next.cpu().numpy(), k)
    print(json.dumps(out), flush=True)


def streamed_main(args):
    """Streamed high-dimensional workload: chunks generated on the device,
    projected onto a basis from a randomized SVD of a sample (host), then
    k-means++ and Lloyd on the projected rows with the FP8 distance GEMM; the
    BF16 and FP32 GEMMs run the same iterations from the same centers."""
    import numpy as np
    import torch

    import synth
    from paper_1502_04265_amd import kmx

    W = STREAMED
    d_in, r, k, rows = W["d_in"], W["r"], W["k"], W["chunk"]
    nchunks = args.chunks or (W["n"] + rows - 1) // rows
    n = nchunks * rows
    dev = "cuda:0"
    torch.cuda.set_device(0)
    ctx = kmx.Context(0)
    F = torch.from_numpy(synth.lowrank_factors(d_in, r, seed=0)).to(dev)
    log(f"[bench] basis from a {W['sample']}-row sample (randomized range finder on the GPU)")
    sample = torch.cat([synth.lowrank_chunk_device(rows, F, seed=0, chunk=1_000_000 + c,
                                                   device=dev)
                        for c in range((W["sample"] + rows - 1) // rows)])[:W["sample"]]
    sample = sample.contiguous()
    ctx.range_basis(sample, r, oversample=16, power_iters=1, seed=0)      # buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Vd, _ = ctx.range_basis(sample, r, oversample=16, power_iters=1, seed=0)
    torch.cuda.synchronize()
    svd_s = time.perf_counter() - t0
    del sample
    Y = torch.empty((n, r), dtype=torch.float32, device=dev)
    ctx.timing(True, True)
    gen_ms = 0.0
    for c in range(nchunks):
        t1 = time.perf_counter()
        Xc = synth.lowrank_chunk_device(rows, F, seed=0, chunk=c, device=dev)
        torch.cuda.synchronize()
        gen_ms += (time.perf_counter() - t1) * 1e3
        ctx.project(Xc, Vd, out=Y[c * rows:(c + 1) * rows])
        if c % 32 == 0:
            log(f"[bench] chunk {c}/{nchunks}")
    torch.cuda.synchronize()
    kt = ctx.timing_read()
    ctx.timing(False, True)
    del Xc
    p_ms, p_cnt = kt["project"]
    p_avg = p_ms / max(p_cnt, 1)
    p_bytes = rows * d_in * 4 + rows * r * 4 + d_in * r * 4
    log(f"[bench] projection: {p_avg:.3f} ms per chunk, {p_bytes / (p_avg * 1e-3) / 1e9:.0f} GB/s")

    C0, _ = ctx.seed(Y, k, rng_seed=0)
    res = {}
    for prec in ("fp8", "bf16", "fp32"):
        ctx.lloyd(Y, C0, 1, prec=prec, labels=False)            # per-precision copy of Y
        ctx.timing(True, True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Cp, _, hist, it = ctx.lloyd(Y, C0, args.steps, prec=prec, labels=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        kk = ctx.timing_read()
        ctx.timing(False, True)
        listed, via_fp32, full = ctx.assign_stats()
        a_ms, a_cnt = kk["assign"]
        res[prec] = {"iter_per_s": args.steps / wall, "ms_per_step": wall * 1e3 / args.steps,
                     "final_cost": hist[-1], "assign_ms": a_ms / max(a_cnt, 1),
                     "recheck_ms_per_step": (kk["recheck"][0] + kk["short_recheck"][0])
                                            / args.steps,
                     "final_listed": listed, "final_via_fp32_gemm": via_fp32,
                     "final_all_centers": full,
                     "kernel_ms_per_step": {c: v[0] / args.steps for c, v in kk.items() if v[1]}}
        log(f"[bench] {prec}: {wall * 1e3 / args.steps:.3f} ms/iter, cost {hist[-1]:.9e}, "
            f"listed {listed}, via FP32 {via_fp32}")
    base = res["fp32"]["final_cost"]
    flops = 2.0 * n * k * r
    # bytes one full assignment must read: the GEMM operand rows (+ FP8 scales)
    opbytes = {"fp8": n * (r + 1), "bf16": n * 2 * ((r + 31) // 32 * 32), "fp32": n * 4 * r}
    peaks = {"fp8": FP8_PEAK_TFLOPS, "bf16": BF16_PEAK_TFLOPS, "fp32": FP32_PEAK_TFLOPS}
    roofs = {}
    for prec, rr in res.items():
        a_ms = rr["assign_ms"]
        if flops / opbytes[prec] >= peaks[prec] * 1e12 / (HBM_PEAK_GBS * 1e9):
            ach = flops / (a_ms * 1e-3) / 1e12
            roofs[prec] = {"bound": "mfma", "achieved": ach, "peak": peaks[prec],
                           "unit": "TFLOP/s", "frac": ach / peaks[prec], "traffic": None,
                           "kernel": f"assign_kernel<{prec}>", "avg_ms": a_ms}
        else:
            ach = opbytes[prec] / (a_ms * 1e-3) / 1e9
            roofs[prec] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                           "kernel": f"assign_kernel<{prec}>", "avg_ms": a_ms,
                           "algorithmic_bytes": opbytes[prec]}
    best = max(res, key=lambda q: res[q]["iter_per_s"])
    dtypes = {"fp8": "fp8e4m3", "bf16": "bf16", "fp32": "f32"}
    out = {
        "metric": "streamed pipeline: projected rows/s and Lloyd iter/s on the projected rows",
        "value": res[best]["iter_per_s"], "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": res[best]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtypes[best], "data": "synthetic",
        "config": {"workload": W["name"], "n": n, "d_in": d_in, "d": r, "k": k,
                   "chunks": nchunks, "path": best,
                   "value_is": "the fastest of the exact GEMM precisions (identical results)"},
        "projection": {"ms_per_chunk": p_avg, "rows_per_s": rows / (p_avg * 1e-3),
                       "roofline": {"bound": "hbm", "achieved": p_bytes / (p_avg * 1e-3) / 1e9,
                                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": p_bytes / (p_avg * 1e-3) / 1e9 / HBM_PEAK_GBS},
                       "tflops": 2.0 * rows * d_in * r / (p_avg * 1e-3) / 1e12,
                       "fp32_mfma_frac": 2.0 * rows * d_in * r / (p_avg * 1e-3) / 1e12
                                         / FP32_PEAK_TFLOPS,
                       "generation_ms_per_chunk": gen_ms / nchunks, "svd_s": svd_s},
        "roofline": roofs[best],
        "gemm_rooflines": roofs,
        "paths": res,
        "equal_cost_rel_diff": {p: abs(res[p]["final_cost"] - base) / base for p in res},
    }
    print(json.dumps(out), flush=True)


def piecy_main(args):
    """piecy and piecy-mr (Sec. 2.2, 2.3) end to end on a StructuredWithNoise
    instance (Sec. 3), rows in a random order, resident on the device: per
    piece the range finder, the projection and the lift on the device, BICO
    insertion on the host with its first-level search on the device, then
    k-means++ and 20 Lloyd iterations on the summary.  value = input points per
    second of the whole pipeline (piecy); the summary's centers are scored on
    the full data against k-means++ + 20 Lloyd iterations run on the full data.
    cpu_baseline: the same pipeline in the FP64 oracle (exact SVD, oracle/bico,
    oracle k-means) on a bounded sample of the rows."""
    import numpy as np
    import torch

    import synth
    from oracle import bico as ob
    from oracle import kmeans as ok
    from oracle import project as op
    from paper_1502_04265_amd import kmx, piecy

    W = PIECY
    k, svd = W["k"], W["svd"]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    log("[bench] generating StructuredWithNoise")
    X = synth.structured_with_noise(W["ell"], W["y"], W["d"], W["x"], seed=0)
    X = X[np.random.default_rng(0).permutation(X.shape[0])]
    n = X.shape[0]
    Xd = torch.from_numpy(X).to(dev)
    ctx = kmx.Context(0)
    log("[bench] warm-up: piecy on 4000 rows")
    piecy.piecy(ctx, [Xd[:4000]], k, svd, lloyd_iters=2)        # buffers
    torch.cuda.synchronize()

    def progress(q, rows, st):
        log(f"[bench]   piece {q}: {st['count']} features, T {st['T']:.4g}, "
            f"{st['rebuilds']} rebuilds, {st['gpu_rows']} rows searched on the device, "
            f"{st['host_scans']} host scans")
    res = {}
    for name in ("piecy", "piecy_mr"):
        ps = W["piece"] if name == "piecy" else 200 * k
        pieces = [Xd[a:a + ps] for a in range(0, n, ps)]
        ctx.timing(True, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        log(f"[bench] {name}: {len(pieces)} pieces of {ps} rows")
        if name == "piecy":
            r = piecy.piecy(ctx, iter(pieces), k, svd, lloyd_iters=20, seed=1, progress=progress)
        else:
            r = piecy.piecy_mr(ctx, iter(pieces), k, svd, np_=W["np_"], lloyd_iters=20, seed=1,
                               progress=progress)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = ctx.timing_read()
        ctx.timing(False, True)
        cost = ctx.cost(Xd, r["C"])
        dev_query_ms = (kt["assign"][0] + kt["recheck"][0] + kt["short_recheck"][0]
                        + kt["prep"][0])
        pairs = sum(b["pairs"] for b in r["bico"] + r.get("handed_on", []))
        search_tf = 2.0 * pairs * W["d"] / (dev_query_ms * 1e-3) / 1e12 if dev_query_ms else 0.0
        res[name] = {"points_per_s": n / wall, "wall_s": wall, "piece_rows": ps,
                     "device_search": {"pairs": pairs, "ms": dev_query_ms,
                                       "tflops": search_tf,
                                       "roofline": {"bound": "mfma", "achieved": search_tf,
                                                    "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                                    "frac": search_tf / FP32_PEAK_TFLOPS,
                                                    "kernel": "assign_kernel<fp32> + re-check + "
                                                              "row / center preparation"}},
                     "reduce_s": r["reduce_s"], "bico_s": r["bico_s"], "kmeans_s": r["kmeans_s"],
                     "bico_device_search_ms": dev_query_ms,
                     "project_lift_range_ms": kt["project"][0],
                     "summary_points": int(r["P"].shape[0]), "cost": cost, "bico": r["bico"]}
        log(f"[bench] {name}: {n / wall:.0f} points/s ({wall:.2f} s: reduce {r['reduce_s']:.2f}, "
            f"bico {r['bico_s']:.2f}, k-means {r['kmeans_s']:.2f}), summary {r['P'].shape[0]}, "
            f"cost {cost:.6e}")
    C0, _ = ctx.seed(Xd, k, rng_seed=1)
    Cf, _, _, _ = ctx.lloyd(Xd, C0, 20, prec="fp32")
    full_cost = ctx.cost(Xd, Cf)
    for r in res.values():
        r["cost_vs_full_data_lloyd"] = r["cost"] / full_cost
    cpu = None
    if not args.no_cpu_baseline:
        m_s = 2000
        log(f"[bench] oracle pipeline on {m_s} rows")
        t0 = time.perf_counter()
        A = X[:m_s].astype(np.float64)
        Y = op.rank_m_rows(A, svd)
        b = ob.summarize(Y.astype(np.float32), 200 * k, piecy.initial_threshold(
            ctx, torch.from_numpy(Y.astype(np.float32)).to(dev), 200 * k))
        P, wP = b.coreset()
        C0o, _, _ = ok.seed(P, wP, k, 1)
        ok.lloyd(P, wP, C0o, 20)
        t = time.perf_counter() - t0
        cpu = {"value": m_s / t, "unit": "points/s", "cores": 1, "kind": "oracle",
               "sample": f"piecy on the first {m_s} of {n} rows as one piece (exact SVD, "
                         f"oracle BICO, oracle k-means++ + 20 Lloyd), {t:.1f} s on one core",
               "host": host_cpu()}
    best = res["piecy"]
    out = {
        "metric": "piecy points/s (StructuredWithNoise n=2e5 d=1000 k=50), summary cost vs "
                  "full-data Lloyd",
        "value": best["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": best["wall_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": W["name"], "n": n, "d": W["d"], "k": k, "svd": svd,
                   "piece_rows": W["piece"], "summary_size": 200 * k, "np": W["np_"]},
        "roofline": best["device_search"]["roofline"],
        "roofline_note": "the pipeline is bound by BICO's sequential host work (bico_s); the "
                         "dominant device work is BICO's closest-reference searches",
        "paths": res, "full_data_lloyd_cost": full_cost,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=15,
                    help="timed Lloyd iterations (after the warmup iterations)")
    ap.add_argument("--warmup", type=int, default=5,
                    help="plain FP32 iterations whose labels train the router")
    ap.add_argument("--batch", type=int, default=8192, help="router training batch")
    ap.add_argument("--lr", type=float, default=1e-3, help="router learning rate (Adam)")
    ap.add_argument("--workload", default="router",
                    choices=sorted(WORKLOADS) + ["streamed", "batched", "rotated", "piecy"])
    ap.add_argument("--instances", type=int, default=256,
                    help="batched workload: number of instances")
    ap.add_argument("--chunks", type=int, default=None,
                    help="streamed workload: number of chunks (default: all of n)")
    ap.add_argument("--traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT_JSON"),
                    help="convert two rocprofv3 counter passes of --only assign into the traffic "
                         "record (no GPU)")
    ap.add_argument("--traffic-recheck", nargs=4,
                    metavar=("FETCH_DIR", "WRITE_DIR", "FETCH_RUN_STDOUT", "OUT_JSON"),
                    help="convert two rocprofv3 counter passes of the headline path into the "
                         "re-check traffic record (no GPU)")
    ap.add_argument("--paths", default=None,
                    help="profiling: comma-separated subset of the headline paths to run (the "
                         "full BF16 path always runs: the others are checked against it)")
    ap.add_argument("--repeats", type=int, default=3,
                    help="timed runs per path (the median is reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-library-reference", action="store_true",
                    help="skip timing torch's read / copy / GEMMs for context")
    ap.add_argument("--only", choices=["assign"], default=None,
                    help="profiling mode: only the assignment on the workload's data (centers = "
                         "first k rows + noise), plus a plain 1 GiB device copy whose counters "
                         "calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    args.steps_given = any(a == "--steps" or a.startswith("--steps=") for a in sys.argv[1:])

    if args.traffic:
        rec = traffic_convert(args.traffic[0], args.traffic[1])
        json.dump(rec, open(args.traffic[2], "w"), indent=1)
        print(json.dumps(rec, indent=1))
        return
    if args.traffic_recheck:
        a = args.traffic_recheck
        rec = traffic_recheck_convert(a[0], a[1], a[2])
        json.dump(rec, open(a[3], "w"), indent=1)
        print(json.dumps(rec, indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(run it with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1502_04265_amd import kmx

    if args.workload == "streamed":
        return streamed_main(args)
    if args.workload == "batched":
        return batched_main(args)
    if args.workload == "rotated":
        return rotated_main(args)
    if args.workload == "piecy":
        return piecy_main(args)
    wl = WORKLOADS[args.workload]
    n, d, k = wl["n"], wl["d"], wl["k"]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    log(f"[bench] generating {n}x{d} on device")
    if args.workload == "router":
        X, means, sig = synth.router_mixture_device(n, d, k, seed=0, device=dev)
    else:
        Xh, _ = synth.isotropic_mixture(n, d, k, seed=0)
        X = torch.from_numpy(Xh).to(dev)
    torch.cuda.synchronize()
    ctx = kmx.Context(0)

    if args.only == "assign":
        g = torch.Generator(device=dev)
        g.manual_seed(1)
        C = X[:k].contiguous() + 0.05 * torch.randn(k, d, device=dev, generator=g)
        cal = torch.empty(1 << 28, dtype=torch.float32, device=dev)      # 1 GiB
        dst = torch.empty_like(cal)
        for prec in ("bf16", "fp8", "fp32"):
            ctx.assign(X, C, prec=prec, want_d=False)
            for _ in range(args.steps):
                ctx.assign(X, C, prec=prec, want_d=False)
            log(f"[bench] assign {prec} x{args.steps}")
        for _ in range(3):
            dst.copy_(cal)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "assign-only", "n": n, "d": d, "k": k, "steps": args.steps,
                          "copy_bytes_each_way": cal.numel() * 4}), flush=True)
        return

    # ---- seeding (not part of the per-iteration metric) ----
    log("[bench] k-means++ seeding")
    ctx.timing(True, True)
    t0 = time.perf_counter()
    C0, idx = ctx.seed(X, k, rng_seed=0)
    torch.cuda.synchronize()
    seed_ms = (time.perf_counter() - t0) * 1e3
    seed_ev_ms = ctx.timing_read()["seed"][0]      # HIP events around the k rounds
    ctx.timing(False, True)
    seed_rows = ctx.seed_stats()                    # rows whose distance a round computed
    # rounds 1 .. k-1: every row's D2 and closest-center index (12 bytes), and
    # for the rows read the row itself plus the D2 / index writes (4d + 12 bytes)
    seed_bytes = 12.0 * n * (k - 1) + float(seed_rows) * (4 * d + 12)
    seed_gbs = seed_bytes / (seed_ev_ms * 1e-3) / 1e9
    seed_frac_read = seed_rows / float(n * max(k - 1, 1))
    log(f"[bench] seeding {seed_ms:.1f} ms ({seed_ev_ms / k:.3f} ms per round, {seed_gbs:.0f} GB/s, "
        f"{100 * seed_frac_read:.1f}% of the rows read per round)")

    # ---- warmup = plain FP32 iterations 1..W, labels recorded for training ----
    t0 = time.perf_counter()
    sets = []
    C = C0
    for _ in range(args.warmup):
        C, lab, _, _ = ctx.lloyd(X, C, 1, prec="fp32", labels=True)
        sets.append(lab)
    torch.cuda.synchronize()
    Cw = C
    warm_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] plain FP32 iterations 1..{args.warmup}: {warm_ms:.1f} ms")

    # ---- router training on the recorded (x, label) pairs ----
    router = ctx.router(d, k, init_seed=0)
    train = {}
    if sets:
        labels = torch.stack(sets).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = router.train(X, labels, epochs=1, batch=args.batch, lr=args.lr, shuffle_seed=1)
        torch.cuda.synchronize()
        train_ms = (time.perf_counter() - t0) * 1e3
        del labels
        pairs = len(sets) * n
        flops_step = 6.0 * (d * 256 + 256 * k)          # forward + two backward products
        train = {"ms": train_ms, "steps": len(losses), "batch": args.batch, "lr": args.lr,
                 "pairs": pairs, "loss_first": losses[0], "loss_last": losses[-1],
                 "tflops": flops_step * pairs / (train_ms * 1e-3) / 1e12}
        log(f"[bench] router training: {len(losses)} steps, {train_ms:.1f} ms, loss "
            f"{losses[0]:.3f} -> {losses[-1]:.4f}")
    del sets

    # ---- one-off per dataset: the BF16 and FP8 copies of X and their row
    # statistics (cached by the context; every timed path below reuses them) ----
    prep_once = {}
    for prec in ("bf16", "fp8"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.assign(X, Cw, prec=prec, want_d=False)
        torch.cuda.synchronize()
        prep_once[prec] = (time.perf_counter() - t0) * 1e3
    log(f"[bench] quantized copies of X (one-off, with one assignment each): {prep_once}")

    # ---- timed region: K Lloyd iterations from the same centers on every
    # exact path, each timed REPEATS times (the median is reported) ----
    def run_timed(label, fn):
        walls, kts, res = [], [], None
        for _ in range(args.repeats):
            ctx.timing(True, True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t)
            kts.append(ctx.timing_read())
            ctx.timing(False, True)
        order = sorted(range(len(walls)), key=lambda q: walls[q])
        med = order[len(order) // 2]
        w = walls[med]
        log(f"[bench] {label}: {w * 1e3 / args.steps:.3f} ms/iter (median of {len(walls)}: "
            f"{', '.join(f'{x * 1e3 / args.steps:.3f}' for x in walls)}), cost {res[2][-1]:.9e}")
        return res, w, kts[med], walls

    def per_step(kk):
        return {c: (v[0] / args.steps) for c, v in kk.items() if v[1]}

    paths, results = {}, {}

    only = set(args.paths.split(",")) if args.paths else None

    def add(name, fn, assign, uses_router, dtype):
        if only is not None and name not in only and name != "full_bf16":
            return {}
        res, w, kk, walls = run_timed(name, fn)
        results[name] = res
        paths[name] = {"iter_per_s": args.steps / w, "ms_per_step": w * 1e3 / args.steps,
                       "ms_per_step_runs": [x * 1e3 / args.steps for x in walls],
                       "final_cost": res[2][-1], "kernel_ms_per_step": per_step(kk),
                       "assign": assign, "router": uses_router, "dtype": dtype}
        if len(res) > 4:
            paths[name]["gemm_rows_per_assignment"] = res[4]
        if len(res) > 5:
            paths[name]["bound_kept_rows_per_assignment"] = res[5]
        listed, full = ctx.run_stats()          # the last timed run (all runs are identical)
        paths[name]["short_recheck_entries"] = listed + full
        return kk

    S = args.steps
    kt = add("routed_bf16", lambda: ctx.lloyd_routed(X, Cw, S, router=router, prec="bf16"),
             "router proposals + Elkan certificate, BF16 MFMA GEMM + exact re-check for the "
             "other rows", True, "bf16")
    add("routed_fp8", lambda: ctx.lloyd_routed(X, Cw, S, router=router, prec="fp8"),
        "router proposals + certificate, FP8 E4M3 GEMM cascade for the other rows", True,
        "fp8e4m3")
    kb8r = add("bounded_routed_fp8",
               lambda: ctx.lloyd_bounded(X, Cw, S, router=router, prec="fp8"),
               "bounds carried across iterations; rows they cannot keep: router proposals + "
               "certificate, then the FP8 E4M3 GEMM cascade", True, "fp8e4m3")
    kb8 = add("bounded_fp8", lambda: ctx.lloyd_bounded(X, Cw, S, router=None, prec="fp8"),
              "bounds carried across iterations; rows they cannot keep: previous-label "
              "certificate, then the FP8 E4M3 GEMM cascade", False, "fp8e4m3")
    add("previous_labels", lambda: ctx.lloyd_routed(X, Cw, S, router=None, prec="bf16"),
        "previous label + certificate, BF16 GEMM for the other rows", False, "bf16")
    ktb = add("full_bf16", lambda: ctx.lloyd(X, Cw, S, prec="bf16"),
              "BF16 MFMA GEMM with fused top-4, split-BF16 GEMM pass and exact re-check of "
              "undecided rows", False, "bf16")
    kt8 = add("full_fp8", lambda: ctx.lloyd(X, Cw, S, prec="fp8"),
              "FP8 E4M3 MFMA GEMM (per-row scales) with fused top-3, BF16 then split-BF16 GEMM "
              "passes and exact re-check of undecided rows", False, "fp8e4m3")
    if "full_fp8" in paths:
        paths["full_fp8"]["final_listed_via_fp32_all"] = list(ctx.assign_stats())
    for prec in ("bf16", "fp8"):     # the first capture on a context pays one-off costs
        if only is None or f"full_{prec}_graph" in only:
            ctx.lloyd(X, Cw, 1, prec=prec, labels=False, graph=True)
    add("full_bf16_graph", lambda: ctx.lloyd(X, Cw, S, prec="bf16", graph=True),
        "as full_bf16, the iteration replayed as a HIP graph", False, "bf16")
    add("full_fp8_graph", lambda: ctx.lloyd(X, Cw, S, prec="fp8", graph=True),
        "as full_fp8, the iteration replayed as a HIP graph", False, "fp8e4m3")
    ktf = None
    if not args.no_fp32:
        ktf = add("fp32", lambda: ctx.lloyd(X, Cw, S, prec="fp32"),
                  "plain FP32 MFMA GEMM with fused top-3 and exact re-check (the reference path "
                  "of the metric)", False, "f32")

    if only is not None:      # profiling subset: the timings only
        same = all(torch.equal(r[1], results["full_bf16"][1]) for r in results.values())
        print(json.dumps({"mode": "paths", "identical_labels": bool(same), "paths": paths}),
              flush=True)
        return
    base_lab, base_C = results["full_bf16"][1], results["full_bf16"][0]
    same = all(torch.equal(r[1], base_lab) and torch.equal(r[0], base_C) for r in results.values())
    cost_ref = paths["fp32"]["final_cost"] if "fp32" in paths else paths["full_bf16"]["final_cost"]
    for p in paths.values():
        p["equal_cost_rel_diff"] = abs(p["final_cost"] - cost_ref) / cost_ref

    # ---- rooflines ----
    def avg(kk, cls):
        ms, cnt = kk.get(cls, (0.0, 0))
        return ms / max(cnt, 1), cnt

    flops = 2.0 * n * k * d
    a_ms, _ = avg(ktb, "assign")
    achieved = flops / (a_ms * 1e-3) / 1e12
    a8_ms, _ = avg(kt8, "assign")           # the FP8 pass (its BF16 cascade is timed as re-check)
    achieved8 = flops / (a8_ms * 1e-3) / 1e12
    # the full reduction alone: kmx_update sums every row (one launch each)
    lab_f, C_f = results["full_bf16"][1], results["full_bf16"][0]
    ctx.update(X, lab_f, C_f)
    ctx.timing(True, True)
    for _ in range(3):
        ctx.update(X, lab_f, C_f)
    kr = ctx.timing_read()
    ctx.timing(False, True)
    r_ms, _ = avg(kr, "reduce")
    reduce_bytes = n * d * 4 + n * 4          # rows of X (FP32) + the permutation
    reduce_gbs = reduce_bytes / (r_ms * 1e-3) / 1e9
    f_ms, f_cnt = avg(kt, "router")
    router_flops = 2.0 * n * (d * 256 + 256 * k)
    c_ms, c_cnt = avg(kt, "certificate")
    cert_bytes = n * (2 * d + 64 + 4 + 16)     # BF16 row, 16 proposals, label, row statistics
    bd_ms, bd_cnt = avg(kb8, "bounds")

    # `value`: the router form of the method (router proposals + mixed precision,
    # with or without carried bounds), valid only when every path returned the
    # same labels and centers and the same final cost as the FP32 path
    routed = [p for p in paths if paths[p]["router"]]
    best = max(routed, key=lambda q: paths[q]["iter_per_s"])
    fastest = max(paths, key=lambda q: paths[q]["iter_per_s"])
    equal_cost = paths[best]["equal_cost_rel_diff"] <= 1e-6
    valid = bool(same and equal_cost)
    value = paths[best]["iter_per_s"] if valid else 0.0
    ms_per_step = paths[best]["ms_per_step"]
    bf16_roof = {"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS,
                 "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS,
                 "traffic": measured_traffic("assign_bf16") if args.workload == "router" else None,
                 "kernel": "assign_kernel<bf16> (full assignment)", "avg_ms": a_ms,
                 "algorithmic_flops": flops}
    fp8_roof = {"bound": "mfma", "achieved": achieved8, "peak": FP8_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved8 / FP8_PEAK_TFLOPS,
                "traffic": measured_traffic("assign_fp8") if args.workload == "router" else None,
                "kernel": "assign_kernel<fp8> (full assignment)", "avg_ms": a8_ms,
                "algorithmic_flops": flops}
    update_roof = {"bound": "hbm", "achieved": reduce_gbs, "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "frac": reduce_gbs / HBM_PEAK_GBS,
                   "traffic": None,
                   "kernel": "cf_reduce_kernel, full update (every row; exact fixed-point "
                             "clustering features)", "avg_ms": r_ms,
                   "algorithmic_bytes": reduce_bytes}
    # the exact short / every-center re-check of the reported path: each entry
    # reads its FP32 row once (the candidate centers stay in L2)
    sr_ms_total = paths[best]["kernel_ms_per_step"].get("short_recheck", 0.0) * args.steps
    sr_entries = paths[best].get("short_recheck_entries", 0)
    sr_bytes = sr_entries * (4.0 * d + 24)
    sr_gbs = sr_bytes / (sr_ms_total * 1e-3) / 1e9 if sr_ms_total > 0 else 0.0
    short_roof = {"bound": "hbm", "achieved": sr_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": sr_gbs / HBM_PEAK_GBS,
                  "traffic": (measured_recheck_traffic(sr_entries, args.steps)
                              if args.workload == "router" else None),
                  "kernel": "recheck_pair_kernel + recheck_full_kernel (exact re-check of the "
                            "listed rows)",
                  "ms_per_step": sr_ms_total / args.steps, "entries": sr_entries,
                  "algorithmic_bytes": sr_bytes}
    # the dominant kernel of the reported path among those whose work is known
    # per launch: the exact re-check, the full-grid FP8 GEMM (once per call),
    # the full reduction (once per call)
    kms = paths[best]["kernel_ms_per_step"]
    cand = {"short_recheck": sr_ms_total / args.steps,
            "fp8_gemm": a8_ms / args.steps, "reduce": r_ms / args.steps}
    dom = max(cand, key=lambda c: cand[c])
    roofline = {"short_recheck": short_roof, "fp8_gemm": fp8_roof, "reduce": update_roof}[dom]

    out = {
        "metric": METRIC, "value": value, "unit": "iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": paths[best]["dtype"], "data": "synthetic",
        "config": {"workload": wl["name"], "n": n, "d": d, "k": k, "path": best,
                   "assign": paths[best]["assign"],
                   "reduce": "exact fixed-point clustering features, delta update after the "
                             "first",
                   "timed": f"Lloyd iterations {args.warmup + 1}..{args.warmup + args.steps} "
                            f"from the centers after {args.warmup} plain FP32 iterations, "
                            f"median of {args.repeats} runs",
                   "value_is": "the fastest path that uses the router (router proposals + "
                               "mixed precision); reported only when every path returned "
                               "identical labels and centers and its final cost equals the "
                               "FP32 path's within 1e-6 relative"},
        "valid": valid,
        "roofline": roofline,
        "roofline_dominant_kernel_class": dom,
        "bf16_gemm_roofline": bf16_roof,
        "fp8_gemm_roofline": fp8_roof,
        "update_roofline": update_roof,
        "short_recheck_roofline": short_roof,
        "seed_roofline": {"bound": "hbm", "achieved": seed_gbs, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": seed_gbs / HBM_PEAK_GBS,
                          "kernel": "seed_round_kernel", "avg_ms": seed_ev_ms / k, "rounds": k,
                          "rows_read_fraction": seed_frac_read},
        "router_roofline": {"bound": "mfma", "achieved": router_flops / (f_ms * 1e-3) / 1e12,
                            "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": router_flops / (f_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                            "kernel": "router_fwd_kernel", "avg_ms": f_ms, "launches": f_cnt},
        "certificate_roofline": {"bound": "hbm", "achieved": cert_bytes / (c_ms * 1e-3) / 1e9,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": cert_bytes / (c_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "kernel": "center table + router_cert_kernel", "avg_ms": c_ms},
        "bound_test_ms": bd_ms,
        "paths": paths,
        "fastest_path": {"path": fastest, "iter_per_s": paths[fastest]["iter_per_s"]},
        "router_gain": {
            "routed_fp8_vs_full_fp8": paths["routed_fp8"]["iter_per_s"]
            / paths["full_fp8"]["iter_per_s"],
            "bounded_routed_fp8_vs_bounded_fp8": paths["bounded_routed_fp8"]["iter_per_s"]
            / paths["bounded_fp8"]["iter_per_s"]},
        "identical_paths": bool(same),
        "equal_cost": bool(equal_cost),
        "router_training": train,
        "seed_ms": seed_ms, "warmup_ms": warm_ms,
        "quantized_copies_once_ms": prep_once,
        "final_cost": paths[best]["final_cost"],
    }
    if "fp32" in paths:
        out["fp32_path"] = {"iter_per_s": paths["fp32"]["iter_per_s"],
                            "ms_per_step": paths["fp32"]["ms_per_step"],
                            "final_cost": paths["fp32"]["final_cost"]}
        out["speedup_vs_fp32"] = paths[best]["iter_per_s"] / paths["fp32"]["iter_per_s"]
        out["equal_cost_rel_diff"] = paths[best]["equal_cost_rel_diff"]
        if n <= 1_000_000:
            # small problems are launch-bound: the same iterations replayed as a graph
            ctx.lloyd(X, Cw, 1, prec="fp32", labels=False, graph=True)
            res, wfg, _, _ = run_timed("fp32 graph",
                                       lambda: ctx.lloyd(X, Cw, S, prec="fp32", graph=True))
            out["fp32_path"]["graph_ms_per_step"] = wfg * 1e3 / S
            out["fp32_path"]["graph_identical"] = bool(torch.equal(res[0], results["fp32"][0])
                                                       and res[2] == results["fp32"][2])
    if not valid:
        out["invalid_reason"] = ("paths differ" if not same else "final cost differs from the "
                                 "FP32 path by more than 1e-6 relative")

    # ---- plain library work on the same part, for context ----
    if not args.no_library_reference:
        out["library_reference"] = library_reference()
        log(f"[bench] library reference {out['library_reference']}")

    # ---- the FP64 oracle: timed on the host's cores, and the error of the
    # reported path's results against it ----
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        Cb_, lab_b = results[best][0], results[best][1]
        rows = X[:min(n, 320000)].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(rows, Cb_.cpu().numpy(), n,
                                           gpu_labels=lab_b[:min(n, 320000)].cpu().numpy())
        del rows
        log("[bench] FP64 errors of the results")
        C_next, _, _ = ctx.update(X, lab_b, Cb_)
        out["fp64_error"] = fp64_errors(X.cpu().numpy(), lab_b.cpu().numpy(),
                                        Cb_.cpu().numpy().astype("float64"),
                                        paths[best]["final_cost"], C_next.cpu().numpy(), k)
        log(f"[bench] fp64 errors {out['fp64_error']}")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
