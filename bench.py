"""Lloyd iterations per second on one MI355X.

Workload (default): n = 4,000,000 points in d = 512 from a 1,000-component
Gaussian mixture (means N(0, 4I), sigma_c uniform in [0.5, 1.5], row i in
component i mod 1000), k = 1000, k-means++ seeding (seed 0), W = 5 plain FP32
Lloyd iterations whose labels train the candidate router (1 epoch over the
5 n pairs, batch 8192, Adam lr 1e-3), then K = 15 timed Lloyd iterations
(iterations 6..20).  One step = one Lloyd iteration: certified router
proposals, BF16 MFMA distance GEMM + exact re-check for the other rows,
FP64 segmented reduction, new centroids, FP64 cost; the timed call includes
the router's forward pass (one per call) and the final assignment.  The
same iterations run from the same centers on the plain FP32 path, the full
BF16 path and with previous labels as the only candidates; the results must
agree (identical labels and centers; FP32 cost within 1e-6 relative).

Prints ONE JSON line.  Data is synthetic and generated on the device before
the timed region; seeding, the plain iterations, training and the
comparison runs are timed separately and reported as extra fields.
"""
from __future__ import annotations

import argparse
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


def cpu_baseline(X_host_rows, C_host, n_full, seconds_target=10.0, gpu_labels=None):
    """Times the FP64 oracle (assignment + update of one Lloyd iteration) on a
    bounded row sample and scales to the full n.  With gpu_labels (the path's
    labels of the same rows against the same centers), also counts the rows
    whose label differs from the oracle's outside its 1e-6 relative top-2
    margin."""
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
    res = {"value": 1.0 / sec_per_iter, "unit": "iter/s", "cores": 1, "kind": "oracle",
           "sample": f"one Lloyd iteration (FP64 assign + update) on {m} of {n_full} rows, "
                     f"all {C_host.shape[0]} centers; {t:.1f} s measured, scaled by n",
           "sec_per_iter": sec_per_iter, "host": host_cpu()}
    if gpu_labels is not None:
        g = np.asarray(gpu_labels[:m])
        bad = (g != lab) & ~((d2 - d1) < 1e-6 * d2)
        res["label_check"] = {"rows": m, "differ_outside_margin": int(bad.sum()),
                              "inside_margin": int(((d2 - d1) < 1e-6 * d2).sum())}
    return res


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
    probs = []
    t0 = time.perf_counter()
    for i, desc in enumerate(descs):
        X, w = synth.instance_device(desc, device=dev)
        C0, _ = ctx.seed(X, desc["k"], w=w, rng_seed=i)
        probs.append({"X": X, "C": C0, "w": w})
    torch.cuda.synchronize()
    seed_s = time.perf_counter() - t0
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
    # bytes one iteration must move at least: the BF16 copy of every row (the
    # assignment) and the FP32 row plus its permutation entry (the reduction)
    it_bytes = sum(d["n"] * (2.0 * d["d"] + 4.0 * d["d"] + 4.0) for d in descs)
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
                     "kernel": "whole batched iteration (one captured graph)",
                     "algorithmic_bytes": it_bytes},
        "assign_flops_per_iteration": flops,
        "whole_iteration_tflops": flops / (wall / args.steps) / 1e12,
        "tiles": tiles, "seed_s": seed_s, "autotune_s": tune_s,
    }
    print(json.dumps(out), flush=True)


def streamed_main(args):
    """Streamed high-dimensional workload: chunks generated on the device,
    projected onto a basis from a randomized SVD of a sample (host), then
    k-means++ and Lloyd on the projected rows with the FP8 distance GEMM; the
    BF16 and FP32 GEMMs run the same iterations from the same centers."""
    import numpy as np
    import torch

    import synth
    from paper_1502_04265_amd import kmx, subspace

    W = STREAMED
    d_in, r, k, rows = W["d_in"], W["r"], W["k"], W["chunk"]
    nchunks = args.chunks or (W["n"] + rows - 1) // rows
    n = nchunks * rows
    dev = "cuda:0"
    torch.cuda.set_device(0)
    ctx = kmx.Context(0)
    F = torch.from_numpy(synth.lowrank_factors(d_in, r, seed=0)).to(dev)
    log(f"[bench] basis from a {W['sample']}-row sample (randomized SVD on the host)")
    t0 = time.perf_counter()
    parts = []
    for c in range((W["sample"] + rows - 1) // rows):
        parts.append(synth.lowrank_chunk_device(rows, F, seed=0, chunk=1_000_000 + c,
                                                device=dev).cpu().numpy())
    sample = np.concatenate(parts)[:W["sample"]]
    V = subspace.top_right_singular_vectors(sample, r, power_iters=1, seed=0)
    del parts, sample
    svd_s = time.perf_counter() - t0
    Vd = torch.from_numpy(V).to(dev)
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
                     "recheck_ms_per_step": kk["recheck"][0] / args.steps,
                     "final_listed": listed, "final_via_fp32_gemm": via_fp32,
                     "final_all_centers": full}
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
                    choices=sorted(WORKLOADS) + ["streamed", "batched"])
    ap.add_argument("--instances", type=int, default=256,
                    help="batched workload: number of instances")
    ap.add_argument("--chunks", type=int, default=None,
                    help="streamed workload: number of chunks (default: all of n)")
    ap.add_argument("--fp32-steps", type=int, default=None,
                    help="iterations of the plain FP32 comparison (default: --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-library-reference", action="store_true",
                    help="skip timing torch's read / copy / GEMMs for context")
    ap.add_argument("--only", choices=["assign"], default=None,
                    help="profiling mode: only the assignment on the workload's data (centers = "
                         "first k rows + noise), plus a plain 1 GiB device copy whose counters "
                         "calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()

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

    # ---- timed region: K routed Lloyd iterations (BF16 GEMM for the rest) ----
    ctx.timing(True, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Cr, lab_r, hist_r, it_r, rows_r = ctx.lloyd_routed(X, Cw, args.steps, router=router,
                                                       prec="bf16", labels=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = ctx.timing_read()
    ctx.timing(False, True)
    ms_per_step = wall * 1e3 / args.steps
    value = args.steps / wall
    log(f"[bench] routed: {ms_per_step:.3f} ms/iter, {value:.2f} iter/s, cost {hist_r[-1]:.9e}, "
        f"GEMM rows {rows_r}")

    def run_timed(label, fn):
        ctx.timing(True, True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        w = time.perf_counter() - t
        kk = ctx.timing_read()
        ctx.timing(False, True)
        log(f"[bench] {label}: {w * 1e3 / args.steps:.3f} ms/iter, cost {res[2][-1]:.9e}")
        return res, w, kk

    # ---- the same iterations without the router: full BF16 GEMM, previous labels ----
    (Cb, lab_b, hist_b, _), wb, ktb = run_timed(
        "full bf16", lambda: ctx.lloyd(X, Cw, args.steps, prec="bf16", labels=True))
    (Cp, lab_p, hist_p, _, rows_p), wp, _ = run_timed(
        "previous labels", lambda: ctx.lloyd_routed(X, Cw, args.steps, router=None, prec="bf16",
                                                    labels=True))
    (C8, lab_8, hist_8, _), w8, kt8 = run_timed(
        "full fp8", lambda: ctx.lloyd(X, Cw, args.steps, prec="fp8", labels=True))
    fp8_stats = ctx.assign_stats()
    (Cr8, lab_r8, hist_r8, _, rows_r8), wr8, ktr8 = run_timed(
        "routed fp8", lambda: ctx.lloyd_routed(X, Cw, args.steps, router=router, prec="fp8",
                                               labels=True))
    # the same full paths with the iteration replayed as a graph (kmx_lloyd_graph);
    # one untimed call each first (the first capture on a context pays one-off costs)
    for prec in ("bf16", "fp8"):
        ctx.lloyd(X, Cw, 1, prec=prec, labels=False, graph=True)
    (Cgb, lab_gb, hist_gb, _), wgb, _ = run_timed(
        "full bf16 graph", lambda: ctx.lloyd(X, Cw, args.steps, prec="bf16", labels=True,
                                             graph=True))
    (Cg8, lab_g8, hist_g8, _), wg8, _ = run_timed(
        "full fp8 graph", lambda: ctx.lloyd(X, Cw, args.steps, prec="fp8", labels=True,
                                            graph=True))
    same = bool(torch.equal(lab_r, lab_b) and torch.equal(Cr, Cb) and torch.equal(lab_p, lab_b)
                and torch.equal(lab_8, lab_b) and torch.equal(C8, Cb)
                and torch.equal(lab_r8, lab_b) and torch.equal(Cr8, Cb)
                and torch.equal(lab_gb, lab_b) and torch.equal(Cgb, Cb)
                and torch.equal(lab_g8, lab_b) and torch.equal(Cg8, Cb))

    # ---- rooflines ----
    def avg(kk, cls):
        ms, cnt = kk.get(cls, (0.0, 0))
        return ms / max(cnt, 1), cnt

    flops = 2.0 * n * k * d
    a_ms, _ = avg(ktb, "assign")
    achieved = flops / (a_ms * 1e-3) / 1e12
    a8_ms, _ = avg(kt8, "assign")           # the FP8 pass (its BF16 cascade is timed as re-check)
    achieved8 = flops / (a8_ms * 1e-3) / 1e12
    r_ms, _ = avg(kt, "reduce")
    reduce_bytes = n * d * 4 + n * 4          # rows of X (FP32) + the permutation
    reduce_gbs = reduce_bytes / (r_ms * 1e-3) / 1e9
    f_ms, f_cnt = avg(kt, "router")
    router_flops = 2.0 * n * (d * 256 + 256 * k)
    c_ms, c_cnt = avg(kt, "certificate")
    cert_bytes = n * (2 * d + 64 + 4 + 16)     # BF16 row, 16 proposals, label, row statistics
    gemm_rows_mean = sum(rows_r) / len(rows_r)

    def per_step(kk):
        return {c: (v[0] / args.steps) for c, v in kk.items() if v[1]}

    # every path returns the same labels and centers; `value` is the fastest
    paths = {
        "routed": {"iter_per_s": value, "ms_per_step": ms_per_step, "final_cost": hist_r[-1],
                   "kernel_ms_per_step": per_step(kt), "gemm_rows_per_assignment": rows_r,
                   "gemm_row_fraction": gemm_rows_mean / n,
                   "assign": "router proposals + certificate, bf16 MFMA GEMM + FP32 re-check "
                             "for the other rows"},
        "previous_labels": {"iter_per_s": args.steps / wp, "ms_per_step": wp * 1e3 / args.steps,
                            "final_cost": hist_p[-1], "gemm_rows_per_assignment": rows_p,
                            "assign": "previous label + certificate, bf16 MFMA GEMM for the "
                                      "other rows"},
        "full_bf16": {"iter_per_s": args.steps / wb, "ms_per_step": wb * 1e3 / args.steps,
                      "final_cost": hist_b[-1], "kernel_ms_per_step": per_step(ktb),
                      "assign": "bf16 MFMA GEMM with fused top-4, FP32 GEMM pass and exact "
                                "re-check of undecided rows"},
        "routed_fp8": {"iter_per_s": args.steps / wr8, "ms_per_step": wr8 * 1e3 / args.steps,
                       "final_cost": hist_r8[-1], "kernel_ms_per_step": per_step(ktr8),
                       "gemm_rows_per_assignment": rows_r8,
                       "assign": "router proposals + certificate, fp8 e4m3 MFMA GEMM cascade "
                                 "for the other rows"},
        "full_bf16_graph": {"iter_per_s": args.steps / wgb, "ms_per_step": wgb * 1e3 / args.steps,
                            "final_cost": hist_gb[-1],
                            "assign": "as full_bf16, the iteration replayed as a HIP graph"},
        "full_fp8_graph": {"iter_per_s": args.steps / wg8, "ms_per_step": wg8 * 1e3 / args.steps,
                           "final_cost": hist_g8[-1],
                           "assign": "as full_fp8, the iteration replayed as a HIP graph"},
        "full_fp8": {"iter_per_s": args.steps / w8, "ms_per_step": w8 * 1e3 / args.steps,
                     "final_cost": hist_8[-1], "kernel_ms_per_step": per_step(kt8),
                     "final_listed_via_fp32_all": list(fp8_stats),
                     "assign": "fp8 e4m3 MFMA GEMM (per-row scales) with fused top-4, bf16 "
                               "then FP32 GEMM passes and exact re-check of undecided rows"},
    }
    best = max(paths, key=lambda q: paths[q]["iter_per_s"])
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
    value = paths[best]["iter_per_s"]
    ms_per_step = paths[best]["ms_per_step"]

    out = {
        "metric": METRIC, "value": value, "unit": "iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp8e4m3" if best in ("full_fp8", "routed_fp8", "full_fp8_graph") else "bf16", "data": "synthetic",
        "config": {"workload": wl["name"], "n": n, "d": d, "k": k, "path": best,
                   "assign": paths[best]["assign"], "reduce": "fp64",
                   "timed": f"Lloyd iterations {args.warmup + 1}..{args.warmup + args.steps} "
                            f"from the centers after {args.warmup} plain FP32 iterations",
                   "value_is": "the fastest of the exact paths below (identical labels and "
                               "centers)"},
        "roofline": fp8_roof if best in ("full_fp8", "routed_fp8", "full_fp8_graph") else bf16_roof,
        "bf16_gemm_roofline": bf16_roof,
        "fp8_gemm_roofline": fp8_roof,
        "seed_roofline": {"bound": "hbm", "achieved": seed_gbs, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": seed_gbs / HBM_PEAK_GBS,
                          "kernel": "seed_round_kernel", "avg_ms": seed_ev_ms / k, "rounds": k,
                          "rows_read_fraction": seed_frac_read},
        "update_roofline": {"bound": "hbm", "achieved": reduce_gbs, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": reduce_gbs / HBM_PEAK_GBS,
                            "kernel": "reduce_kernel", "avg_ms": r_ms},
        "router_roofline": {"bound": "mfma", "achieved": router_flops / (f_ms * 1e-3) / 1e12,
                            "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": router_flops / (f_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                            "kernel": "router_fwd_kernel", "avg_ms": f_ms, "launches": f_cnt},
        "certificate_roofline": {"bound": "hbm", "achieved": cert_bytes / (c_ms * 1e-3) / 1e9,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": cert_bytes / (c_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "kernel": "center table + router_cert_kernel", "avg_ms": c_ms},
        "paths": paths,
        "router_vs_full_bf16": paths["routed"]["iter_per_s"] / paths["full_bf16"]["iter_per_s"],
        "identical_paths": same,
        "router_training": train,
        "seed_ms": seed_ms, "warmup_ms": warm_ms,
        "quantized_copies_once_ms": prep_once,
        "final_cost": paths[best]["final_cost"],
    }

    # ---- plain FP32 path from the same start ----
    if not args.no_fp32:
        ks = args.fp32_steps or args.steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Cf, lab_f, hist_f, it_f = ctx.lloyd(X, Cw, ks, prec="fp32", labels=False)
        torch.cuda.synchronize()
        wf = time.perf_counter() - t0
        log(f"[bench] fp32: {wf * 1e3 / ks:.3f} ms/iter, cost {hist_f[-1]:.9e}")
        out["fp32_path"] = {"iter_per_s": ks / wf, "ms_per_step": wf * 1e3 / ks, "steps": ks,
                            "final_cost": hist_f[-1]}
        if n <= 1_000_000:
            # small problems are launch-bound: the same iterations replayed as a graph
            ctx.lloyd(X, Cw, 1, prec="fp32", labels=False, graph=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Cfg, _, hist_fg, _ = ctx.lloyd(X, Cw, ks, prec="fp32", labels=False, graph=True)
            torch.cuda.synchronize()
            wfg = time.perf_counter() - t0
            log(f"[bench] fp32 graph: {wfg * 1e3 / ks:.3f} ms/iter, cost {hist_fg[-1]:.9e}")
            out["fp32_path"]["graph_ms_per_step"] = wfg * 1e3 / ks
            out["fp32_path"]["graph_identical"] = bool(torch.equal(Cfg, Cf) and hist_fg == hist_f)
        out["speedup_vs_fp32"] = value / (ks / wf)
        if ks == args.steps:
            rel = abs(hist_f[-1] - paths[best]["final_cost"]) / hist_f[-1]
            out["equal_cost_rel_diff"] = rel
            out["equal_cost"] = bool(rel <= 1e-6)

    # ---- plain library work on the same part, for context ----
    if not args.no_library_reference:
        out["library_reference"] = library_reference()
        log(f"[bench] library reference {out['library_reference']}")

    # ---- CPU oracle baseline on a bounded sample ----
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        rows = X[:20000].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(rows, Cr.cpu().numpy(), n,
                                           gpu_labels=lab_r[:20000].cpu().numpy())

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
