"""Throughput benchmark of the batched p-FHT-FSCL-L-M decoder on one MI355X.

Headline workload: RM(2,9) (N = 512, K = 46), P = 20 permuted decoders of
list size L = 4 per frame, BPSK/AWGN frames at Eb/N0 = 2.0, 2.5, 3.0, 3.5,
4.0 dB, 262,144 frames per Eb/N0 point.  One step decodes one point's batch
(one kernel launch); steps cycle through the points.  All inputs are
generated (seeded, synthetic) and copied to HBM before the timed region.

The default run also measures, into extra keys of the same JSON line:
"configs" -- RM(2,7) with one plain FHT-FSC decoder (FER on 10,000 frames,
throughput on 2^21 frames against the HBM roofline), RM(2,9) with 512
permuted decoders of list size 1 and RM(3,8) with 8 permuted decoders of list
size 8 (131,072 frames per point, 2.0-4.5 dB, ALU rooflines); "mixed" -- the
fused mixed-code launch (graph-replayed) over RM(2,7) P=8, RM(2,8) P=16,
RM(2,9) P=20 and RM(2,10) P=32 at L = 4, with the launch choices of the
library's autotuner; "serving" -- the request server at 0.5, 1, 2, 5, 10 and
20 M requests/s.

``--workload mixed|serve|biglist|configs`` prints only that part (one JSON
line per configuration for ``configs``).  Diagnostics go to stderr.
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

METRIC = "frames/s & info Gbit/s, RM(9,2) 20×L4 FHT-FSCL; serving p50/p99 latency"
M, R, P, L = 9, 2, 20, 4
FRAMES = 262144
EBN0 = [2.0, 2.5, 3.0, 3.5, 4.0]
SEED = 0
# Algorithmic work per frame: the paper's normalised complexity of
# p-FHT-FSCL-4-20 on RM(2,9), floating-point additions and comparisons
# (Table 5).  Per-op peak: MI355X's FP32 vector rate, 157.3 TFLOP/s with an
# FMA counted as two, is 256 CUs x 64 lanes x 2 instructions per lane per
# clock x 2.4 GHz; one addition or comparison takes one such slot.  (Plain
# FP32 adds issue at that rate on gfx950; min/max, med3, 64-bit compares and
# instructions with a DPP operand at half of it.)
OPS_PER_FRAME = 4.2e5
ALU_PEAK_TOPS = 256 * 64 * 2 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
KERNEL_NAME = "rm_decode_kernel<9, 2, 4, 2, 4>"  # (m, r, L, decoders per wave, waves per SIMD)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rm_decode_rm29_p20_l4_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2108_12550_amd", "csrc", f)
                  for f in ("rmdec_device.hpp", "rmdec_kernels.hpp", "rmdec_inst_a.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(sources=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in sources:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_FILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    if they were taken on a different version of the kernel source."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash(sources):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(dev, stream):
    """A plain 1 GiB device copy, for scaling the HBM counters of a profiled
    run (what FETCH_SIZE and WRITE_SIZE read for known bytes)."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        dst.copy_(src)
    stream.synchronize()
    del src, dst
    log("copy calibration: 1 GiB read + 1 GiB written")


def fer_ci(errors: int, n: int, z: float = 1.96):
    """Frame error rate with its Wilson score interval (95% for z = 1.96)."""
    p = errors / n
    den = 1 + z * z / n
    mid = (p + z * z / (2 * n)) / den
    half = z * np.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return {"fer": float(p), "errors": int(errors), "frames": int(n),
            "ci95": [float(max(0.0, mid - half)), float(min(1.0, mid + half))]}


def host_cpu():
    """Threads the oracle may use (the CPU share of this process, at most 16
    per GPU) and what the host reports about its processor."""
    nproc = os.cpu_count() or 1
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = nproc
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"threads": max(1, min(16, share)), "nproc": nproc, "affinity": share, "cpu_model": model}


def cpu_baseline(llr_host: np.ndarray, gpu_bits: np.ndarray, budget_s: float, threads: int, perm_mode: int = 1):
    """The CPU oracle on a bounded sample of the same frames."""
    import oracle
    od = oracle.OracleDecoder(M, R, P, L, seed=SEED, perm_mode=perm_mode)
    chunk = 64 * threads
    done = 0
    t0 = time.perf_counter()
    same = True
    while done < llr_host.shape[0] and time.perf_counter() - t0 < budget_s:
        sl = slice(done, min(done + chunk, llr_host.shape[0]))
        bits, _ = od.decode_batch(llr_host[sl], n_threads=threads, frame0=sl.start)
        same &= bool(np.array_equal(bits, gpu_bits[sl]))
        done = sl.stop
    dt = time.perf_counter() - t0
    h = host_cpu()
    return {"value": done / dt, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "per_core": done / dt / threads, "nproc": h["nproc"], "cpu_model": h["cpu_model"],
            "sample": f"first {done} frames of the 3.0 dB batch ({dt:.1f} s): one single-threaded oracle decoder "
                      f"per thread on {threads} threads (this process's CPU share: {h['affinity']} of "
                      f"{h['nproc']} logical CPUs, at most 16 per GPU), bit-exact vs GPU: {same}"}, same


def hip_ms(stream, fn, steps):
    """Average milliseconds of fn() over `steps` calls, by HIP events recorded
    on the stream the kernels run on."""
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / max(1, steps)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=FRAMES)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter scaling)")
    ap.add_argument("--workload", choices=("rm29", "mixed", "serve", "biglist", "configs"), default="rm29")
    ap.add_argument("--serve-ms", type=float, default=50.0, help="arrival window per rate of the serving trace")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving part of the default run")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the RM(2,9) P=20 L=4 measurement (no configs, mixed or serving parts)")
    ap.add_argument("--fresh", action="store_true",
                    help="rm29 workload with maps drawn afresh for every frame (the draw is timed with the decode)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); frames are independent, "
              "so N GPUs would each run this same launch on their share of the frames.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "mixed":
        print(json.dumps(bench_mixed(args, with_cpu=not args.no_cpu_baseline)), flush=True)
        return
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "biglist":
        return run_biglist(args)
    if args.workload == "configs":
        for rec in bench_configs(args):
            print(json.dumps(rec), flush=True)
        return

    out = bench_headline(args)
    if not args.headline_only:
        import torch
        torch.cuda.empty_cache()
        out["configs"] = bench_configs(args)
        torch.cuda.empty_cache()
        out["mixed"] = bench_mixed(args, with_cpu=False)
        torch.cuda.empty_cache()
        if not args.no_serve:
            out["serving"] = serve_sweep(SERVE_RATES, args.serve_ms)
    print(json.dumps(out), flush=True)


def bench_headline(args):
    import torch
    import paper_2108_12550_amd as rmd
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    K = synth.code_dimension(M, R)
    n = args.frames
    log(f"generating {len(EBN0)} x {n} frames of RM({R},{M})")
    t0 = time.perf_counter()
    batches = []
    for k, e in enumerate(EBN0):
        x, llr = synth.frames(M, R, n, e, seed=1000 + k)
        batches.append((x, llr, torch.from_numpy(llr).to(dev)))
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s")

    mode = rmd.RM_PERM_FRESH if args.fresh else rmd.RM_PERM_PFHT
    dec = rmd.Decoder(M, R, P, L, seed=SEED, perm_mode=mode)
    stream = torch.cuda.Stream(device=dev)
    outs = [(torch.empty((n, 64), dtype=torch.uint8, device=dev), torch.empty((n,), dtype=torch.float32, device=dev))
            for _ in EBN0]

    if args.copy_calibration:
        copy_calibration(dev, stream)

    def step(i):
        b = i % len(EBN0)
        dec.decode(batches[b][2], out_bits=outs[b][0], out_metric=outs[b][1], stream=stream)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step(args.warmup + i)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / max(1, args.steps)
    fps = n / (ms_per_step / 1e3)

    # frame error rate per point (from the last decode of each point)
    fer = {}
    for k, e in enumerate(EBN0):
        xb = synth.unpack_bits(outs[k][0].cpu().numpy(), 1 << M)
        fer[str(e)] = fer_ci(int(np.any(xb != batches[k][0], axis=1).sum()), xb.shape[0])
    log(f"FER per Eb/N0: {fer}")
    dec_bits_30 = outs[EBN0.index(3.0)][0].cpu().numpy()
    llr_30 = batches[EBN0.index(3.0)][1]
    dec.close()
    del batches, outs

    ops_per_launch = OPS_PER_FRAME * n
    achieved = ops_per_launch / (ms_per_step / 1e3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(ALU_PEAK_TOPS, 4), "unit": "TFLOP/s",
            "frac": round(achieved / ALU_PEAK_TOPS, 5), "traffic": None if args.fresh else measured_traffic(),
            "kernel": KERNEL_NAME + (" + rm_fresh_maps_kernel" if args.fresh else ""),
            "avg_launch_ms": round(ms_per_step, 4),
            "hbm_gbs_algorithmic": round((4 * 512 + 64 + 4) * fps / 1e9, 2)}

    cpu = None
    if not args.no_cpu_baseline:
        threads = host_cpu()["threads"]
        cpu, same = cpu_baseline(llr_30, dec_bits_30, args.cpu_budget, threads, perm_mode=mode)
        log(f"cpu_baseline: {cpu}")

    return {
        "metric": METRIC, "value": round(fps, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"RM(9,2) N=512 K=46 (paper's RM(2,9)), P=20 permuted decoders, L=4, "
                               f"p-FHT-FSCL{' with per-frame fresh maps' if args.fresh else ''}, "
                               f"BPSK/AWGN Eb/N0 2.0-4.0 dB step 0.5",
                   "frames_per_step": n, "ebn0_db": EBN0, "seed": SEED},
        "info_gbit_s": round(fps * K / 1e9, 4),
        "wall_s_timed": round(wall, 3),
        "fer": fer,
        "roofline": roof,
        "cpu_baseline": cpu,
    }


# --- fused mixed-code launch -------------------------------------------------
MIXED_CODES = [(7, 2, 8, 4), (8, 2, 16, 4), (9, 2, 20, 4), (10, 2, 32, 4)]  # (m, r, P, L)
# per-frame algorithmic ops of each code's decoder set (op model of the
# paper's complexity count: f/g, LM, FHT, selection, SPC, times P)
MIXED_OPS = {7: 3.58e4, 8: 1.56e5, 9: 4.27e5, 10: 1.49e6}
MIXED_KERNEL = "rm_mixed_kernel<4, Code<7,2,4,4>, Code<8,2,4,4>, Code<9,2,4,2>, Code<10,2,4,1>>"
MIXED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rm_mixed_c4_traffic.txt")
MIXED_SOURCES = [os.path.join(ROOT, "paper_2108_12550_amd", "csrc", f)
                 for f in ("rmdec_device.hpp", "rmdec_mixed.hip")]


def mixed_cpu_baseline(data, gpu_bits, budget_s, threads):
    """Oracle rate on the first frames of each code, budget split evenly; the
    mix rate is the harmonic combination (equal frame counts per code)."""
    import oracle
    per = {}
    same = True
    for (m, r, P, L), (x, llr) in zip(MIXED_CODES, data):
        od = oracle.OracleDecoder(m, r, P, L, seed=SEED)
        chunk = 16 * threads
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget_s / len(MIXED_CODES):
            sl = slice(done, done + chunk)
            bits, _ = od.decode_batch(llr[sl], n_threads=threads)
            same &= bool(np.array_equal(bits, gpu_bits[m][sl]))
            done += chunk
        per[m] = (done, time.perf_counter() - t0)
    t_frame = sum(dt / n for n, dt in per.values()) / len(per)
    sample = ", ".join(f"RM(2,{m}): {n} frames in {dt:.1f} s" for m, (n, dt) in per.items())
    return {"value": 1.0 / t_frame, "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"first frames of each code ({sample}); 1:1:1:1 mix rate = 1/mean(time per frame); "
                      f"{threads} threads; bit-exact vs GPU: {same}"}, same


def bench_mixed(args, with_cpu=True):
    import torch
    import paper_2108_12550_amd as rmd
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.frames
    log(f"generating 4 x {n} frames (Eb/N0 ~ U[2,4] per frame)")
    t0 = time.perf_counter()
    data, dbuf = [], []
    for m, r, P, L in MIXED_CODES:
        e = synth.uniform_ebn0(n, 2.0, 4.0, seed=2000 + m)
        x, llr = synth.frames(m, r, n, e, seed=3000 + m)
        data.append((x, llr))
        dbuf.append((torch.from_numpy(llr).to(dev), torch.empty((n, (1 << m) // 8), dtype=torch.uint8, device=dev),
                     torch.empty((n,), dtype=torch.float32, device=dev)))
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s")
    decs = [rmd.Decoder(m, r, P, L, seed=SEED) for m, r, P, L in MIXED_CODES]
    stream = torch.cuda.Stream(device=dev)
    if args.copy_calibration:
        copy_calibration(dev, stream)
    mx = rmd.MixedLauncher(max_tiles=4 * n + 16)

    def segs(tiles):
        return [(d, t, b, p, tf) for d, (t, b, p), tf in zip(decs, dbuf, tiles)]

    t0 = time.perf_counter()
    tune = mx.autotune(segs([0] * 4), stream=stream, reps=1)
    log(f"autotune ({time.perf_counter() - t0:.1f} s): {tune}")
    mx.capture(segs(tune["tile_frames"]), stream)

    # per-code separate launches on the same stream, for comparison and as
    # the equality check of the fused results
    sep = [(torch.empty_like(b), torch.empty_like(p)) for _, b, p in dbuf]

    def separate():
        for d, (t, _, _), (b, p) in zip(decs, dbuf, sep):
            d.decode(t, out_bits=b, out_metric=p, stream=stream)

    def timed(fn, steps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(steps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / max(1, steps)

    for _ in range(args.warmup):
        mx.replay()
    t_wall = time.perf_counter()
    ms_fused = timed(mx.replay, args.steps)
    wall = time.perf_counter() - t_wall
    separate()
    ms_sep = timed(separate, max(1, args.steps // 2))
    total = 4 * n
    fps = total / (ms_fused / 1e3)
    log(f"fused {ms_fused:.3f} ms/step ({fps / 1e6:.3f} M frames/s); separate launches {ms_sep:.3f} ms/step")

    gpu_bits, fer, same_sep = {}, {}, True
    for (m, r, P, L), (x, _), (_, b, p), (sb, sp) in zip(MIXED_CODES, data, dbuf, sep):
        bb = b.cpu().numpy()
        gpu_bits[m] = bb
        same_sep &= bool(np.array_equal(bb, sb.cpu().numpy()) and torch.equal(p, sp))
        fer[f"RM(2,{m})"] = fer_ci(int(np.any(synth.unpack_bits(bb, 1 << m) != x, axis=1).sum()), x.shape[0])
    log(f"FER per code: {fer}; fused == separate: {same_sep}")

    ops = sum(MIXED_OPS[m] for m, *_ in MIXED_CODES) * n
    achieved = ops / (ms_fused / 1e3) / 1e12
    byts = sum(4 * (1 << m) + (1 << m) // 8 + 4 for m, *_ in MIXED_CODES) * n
    roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(ALU_PEAK_TOPS, 4), "unit": "TFLOP/s",
            "frac": round(achieved / ALU_PEAK_TOPS, 5),
            "traffic": measured_traffic(MIXED_TRAFFIC_FILE, MIXED_SOURCES),
            "kernel": MIXED_KERNEL, "avg_launch_ms": round(ms_fused, 4),
            "hbm_gbs_algorithmic": round(byts / (ms_fused / 1e3) / 1e9, 2)}
    cpu = None
    if with_cpu:
        threads = host_cpu()["threads"]
        cpu, _ = mixed_cpu_baseline(data, gpu_bits, args.cpu_budget, threads)
        log(f"cpu_baseline: {cpu}")
    K = {m: synth.code_dimension(m, r) for m, r, *_ in MIXED_CODES}
    for d in decs:
        d.close()
    mx.close()
    out = {
        "metric": METRIC, "value": round(fps, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_fused, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "fused mixed-code launch: RM(7,2) P=8, RM(8,2) P=16, RM(9,2) P=20, RM(10,2) P=32, "
                               "all L=4, 1:1:1:1, Eb/N0 ~ U[2,4] dB per frame, hipGraph replay",
                   "frames_per_step": total, "seed": SEED, "tuning": tune},
        "info_gbit_s": round(sum(K.values()) * n / (ms_fused / 1e3) / 1e9, 4),
        "separate_launches_ms_per_step": round(ms_sep, 4),
        "fused_equals_separate": same_sep,
        "wall_s_timed": round(wall, 3),
        "fer": fer,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    return out


# --- request server -----------------------------------------------------------
SERVE_CODES = [(7, 2), (8, 2), (9, 2), (10, 2), (8, 3)]
SERVE_WEIGHTS = [0.3, 0.25, 0.2, 0.15, 0.1]
SERVE_P = [8, 20, 32]
SERVE_L = [1, 4, 8]
SERVE_RATES = [0.5, 1.0, 2.0, 5.0, 10.0, 20.0]  # M requests/s
SERVE_POOL = 32768  # frames per code held in HBM; requests draw rows from it


def serve_sweep(rates, window_ms, seed=5):
    """Poisson arrivals at each rate for window_ms, replayed open-loop by the
    library's trace driver; device-resident frames.  Per rate: offered and
    completed requests/s, p50/p99/max latency (arrival to completion seen
    by the host), batches launched."""
    import torch
    import paper_2108_12550_amd as rmd
    import synth

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    pools = []
    for k, (m, r) in enumerate(SERVE_CODES):
        e = synth.uniform_ebn0(SERVE_POOL, 2.0, 4.0, seed=4000 + k)
        _, llr = synth.frames(m, r, SERVE_POOL, e, seed=5000 + k)
        pools.append(torch.from_numpy(llr).to(dev))
    decs = {(k, P, L): rmd.Decoder(m, r, P, L, seed=SEED)
            for k, (m, r) in enumerate(SERVE_CODES) for P in SERVE_P for L in SERVE_L}
    srv = rmd.Server(batch_bytes=256 << 20, max_batch=65536, depth=2)
    for t in pools:
        srv.register_pool(t)

    def trace(lam, n):
        arrival = np.cumsum(rng.exponential(1.0 / lam, size=n))  # us
        code = rng.choice(len(SERVE_CODES), size=n, p=SERVE_WEIGHTS)
        Ps = rng.choice(SERVE_P, size=n)
        Ls = rng.choice(SERVE_L, size=n)
        rows = rng.integers(0, SERVE_POOL, size=n)
        base = np.array([t.data_ptr() for t in pools], dtype=np.uint64)
        fbytes = np.array([4 << m for m, _ in SERVE_CODES], dtype=np.uint64)
        table = {key: d._h for key, d in decs.items()}
        hkey = np.array([[[table[(k, P, L)] for L in SERVE_L] for P in SERVE_P] for k in range(len(SERVE_CODES))],
                        dtype=np.uint64)
        handles = hkey[code, np.searchsorted(SERVE_P, Ps), np.searchsorted(SERVE_L, Ls)]
        ptrs = base[code] + fbytes[code] * rows.astype(np.uint64)
        return srv.run_trace_arrays(handles, ptrs, np.ones(n, np.int32), arrival)

    trace(1.0, 20000)  # warm-up: first launches of every serving kernel
    results = []
    for lam in rates:
        n = int(lam * window_ms * 1e3)
        lat, st = trace(lam, n)
        el = st["elapsed_us"]
        res = {"offered_mreq_s": lam, "requests": n, "completed_mreq_s": round(n / el, 4),
               "p50_us": round(float(np.percentile(lat, 50)), 1), "p99_us": round(float(np.percentile(lat, 99)), 1),
               "max_us": round(float(lat.max()), 1), "batches": st["batches"], "largest_batch": st["largest_batch"]}
        log(f"serve {res}")
        results.append(res)
    srv.close()
    return {"workload": "Poisson single-frame requests; codes RM(7,2)/RM(8,2)/RM(9,2)/RM(10,2)/RM(8,3) "
                        "w 0.3/0.25/0.2/0.15/0.1; P in {8,20,32}, L in {1,4,8}; Eb/N0 ~ U[2,4] dB; "
                        f"frames resident in HBM; depth 2; each request's decoders split over 4 waves; "
                        f"{window_ms} ms of arrivals per rate after a warm-up trace",
            "rates": results}


def run_serve(args):
    import torch
    torch.cuda.set_device(0)
    sv = serve_sweep(SERVE_RATES, args.serve_ms)
    best = max(sv["rates"], key=lambda r: r["completed_mreq_s"])
    out = {"metric": METRIC, "value": round(best["completed_mreq_s"] * 1e6, 1), "unit": "frames/s", "n_gpus": 1,
           "steps": len(SERVE_RATES), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "serving loop: " + sv["workload"]}, "serving": sv,
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


# --- large lists: one workgroup per frame ------------------------------------
# RM(3,8) (N = 256, K = 93) with one p-FHT-FSCL-64 decoder, the p-FHT-FSCL-L
# column of Table 5, whose normalised complexity is 5.2e5 operations per frame.
BIG_CODE = (8, 3, 1, 64)  # (m, r, P, L)
BIG_OPS = 5.2e5
BIG_FRAMES = 32768
BIG_KERNEL = "big::rm_biglist_kernel<8, 3, 64>"


def run_biglist(args):
    import torch
    import oracle
    import paper_2108_12550_amd as rmd
    import synth
    m, r, P, L = BIG_CODE
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = BIG_FRAMES
    x, llr = synth.frames(m, r, n, 3.0, seed=31)
    t = torch.from_numpy(llr).to(dev)
    dec = rmd.Decoder(m, r, P, L, seed=SEED)
    stream = torch.cuda.Stream(device=dev)
    bits = torch.empty((n, (1 << m) // 8), dtype=torch.uint8, device=dev)
    pm = torch.empty((n,), dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        dec.decode(t, out_bits=bits, out_metric=pm, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        dec.decode(t, out_bits=bits, out_metric=pm, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / max(1, args.steps)
    fps = n / (ms / 1e3)
    xb = synth.unpack_bits(bits.cpu().numpy(), 1 << m)
    fer = fer_ci(int(np.any(xb != x, axis=1).sum()), n)
    achieved = BIG_OPS * fps / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(ALU_PEAK_TOPS, 4), "unit": "TFLOP/s",
            "frac": round(achieved / ALU_PEAK_TOPS, 5), "traffic": None, "kernel": BIG_KERNEL,
            "avg_launch_ms": round(ms, 4), "hbm_gbs_algorithmic": round((4 * 256 + 32 + 4) * fps / 1e9, 3)}
    cpu = None
    if not args.no_cpu_baseline:
        threads = host_cpu()["threads"]
        od = oracle.OracleDecoder(m, r, P, L, seed=SEED)
        done, same, t0 = 0, True, time.perf_counter()
        gb = bits.cpu().numpy()
        while done < n and time.perf_counter() - t0 < args.cpu_budget:
            sl = slice(done, min(done + 16 * threads, n))
            ob, _ = od.decode_batch(llr[sl], n_threads=threads, frame0=sl.start)
            same &= bool(np.array_equal(ob, gb[sl]))
            done = sl.stop
        dt = time.perf_counter() - t0
        cpu = {"value": done / dt, "unit": "frames/s", "cores": threads, "kind": "oracle",
               "sample": f"first {done} frames ({dt:.1f} s), {threads} threads, bit-exact vs GPU: {same}"}
    out = {"metric": METRIC, "value": round(fps, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "RM(8,3) N=256 K=93 (paper's RM(3,8)), one p-FHT-FSCL decoder with L=64 "
                                  "(Table 5, p-FHT-FSCL-L), BPSK/AWGN Eb/N0 3.0 dB", "frames_per_step": n},
           "fer": {"3.0": fer}, "roofline": roof, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


# Operations per frame: the paper's counts (Section III-B, Tables 1-2)
# summed over Alg. 2's node schedule -- exact at L = 1 (Fig. 6's L = 1
# points and Table 5's p-FHT-FSCL-1-M column are reproduced by this count);
# at L = 8 an approximate list-node model (within 6% of Fig. 6's list points).
C1_OPS = 880.0          # RM(2,7), one plain FHT-FSC decoder: f/g 2^s per node, s 2^s per transform, 2^s per SPC node
C1_BYTES = 4 * 128 + 128 // 8 + 4  # LLRs in, codeword and metric out
C3A_OPS = 2614783.0     # RM(2,9), 512 decoders of list size 1 (exact count; Table 5 prints 5.1e5 for 100)
C3B_OPS = 195015.0      # RM(3,8), 8 decoders of list size 8 (list-node model)
C1_KERNEL = "rm_decode_packed_kernel<7, 2, 1, 8, 3>"
C1_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rm_decode_rm27_p1_l1_traffic.txt")
C1_SOURCES = [os.path.join(ROOT, "paper_2108_12550_amd", "csrc", f)
              for f in ("rmdec_device.hpp", "rmdec_kernels.hpp", "rmdec_inst_b.hip")]
C1_FRAMES = 1 << 21

# (name, m, r, P, L, permutation mode, frames per point, Eb/N0 points,
#  operations per frame, where they come from, kernel)
CONFIGS = [
    ("RM(9,2) N=512 K=46 (paper's RM(2,9)), P=512 permuted decoders, L=1",
     9, 2, 512, 1, "pfht", 131072, [2.0, 2.5, 3.0, 3.5, 4.0, 4.5], C3A_OPS,
     "exact L = 1 count: 512 x 5107 + 511 (Table 5's p-FHT-FSCL-1-100, 5.1e5, is the same count for 100)",
     "rm_decode_kernel<9, 2, 1, 8, 3>"),
    ("RM(8,3) N=256 K=93 (paper's RM(3,8)), P=8 permuted decoders, L=8",
     8, 3, 8, 8, "pfht", 131072, [2.0, 2.5, 3.0, 3.5, 4.0, 4.5], C3B_OPS,
     "list-node model (parity unpinned; the paper prints no figure for p-FHT-FSCL-8-8)",
     "rm_decode_kernel<8, 3, 8, 1, 3>"),
]


def bench_c1(args, dev, stream):
    """RM(2,7) with one plain FHT-FSC decoder: FER on the configuration's
    10,000 frames (seed 0, 3.0 dB), throughput on 2^21 frames (1.07 GB of
    LLRs, beyond the 256 MB last-level cache) against the HBM roofline."""
    import torch
    import paper_2108_12550_amd as rmd
    import synth
    m, r = 7, 2
    N = 1 << m
    if args.copy_calibration:
        copy_calibration(dev, stream)
    dec = rmd.Decoder(m, r, 1, 1, seed=SEED, perm_mode=rmd.RM_PERM_NONE)
    x, llr = synth.frames(m, r, 10000, 3.0, seed=0)
    bits, _ = dec.decode(torch.from_numpy(llr).to(dev), stream=stream)
    torch.cuda.synchronize()
    fer = {"3.0": fer_ci(int(np.any(synth.unpack_bits(bits.cpu().numpy(), N) != x, axis=1).sum()), 10000)}
    n = C1_FRAMES
    _, big = synth.frames(m, r, n, 3.0, seed=1)
    t = torch.from_numpy(big).to(dev)
    del big
    ob = torch.empty((n, N // 8), dtype=torch.uint8, device=dev)
    op = torch.empty((n,), dtype=torch.float32, device=dev)

    def step():
        dec.decode(t, out_bits=ob, out_metric=op, stream=stream)

    # a launch takes about 0.3 ms: warm up for about 50 ms (the clocks ramp
    # after the host-side input generation) and time at least 100 launches
    for _ in range(max(args.warmup, 150)):
        step()
    reps = max(100, 2 * args.steps)
    ms = hip_ms(stream, step, reps)
    fps = n / (ms / 1e3)
    gbs = C1_BYTES * fps / 1e9
    log(f"RM(2,7) P=1 L=1: {fps / 1e9:.3f} G frames/s, {gbs:.0f} GB/s")
    roof = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": measured_traffic(C1_TRAFFIC_FILE, C1_SOURCES),
            "kernel": C1_KERNEL, "avg_launch_ms": round(ms, 4), "bytes_per_frame": C1_BYTES,
            "alu_frac": round(C1_OPS * fps / 1e12 / ALU_PEAK_TOPS, 5), "ops_per_frame": C1_OPS}
    dec.close()
    return {"metric": "frames/s", "value": round(fps, 1), "unit": "frames/s", "n_gpus": 1, "steps": reps,
            "warmup": max(args.warmup, 150), "ms_per_step": round(ms, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "RM(7,2) N=128 K=29 (paper's RM(2,7)), one plain FHT-FSC decoder (P=1, L=1, "
                                   "identity permutation), BPSK/AWGN 3.0 dB; FER on 10,000 frames from seed 0, "
                                   "throughput on 2^21 frames from seed 1", "frames_per_step": n},
            "info_gbit_s": round(fps * synth.code_dimension(m, r) / 1e9, 4), "fer": fer, "roofline": roof}


def bench_configs(args):
    import torch
    import paper_2108_12550_amd as rmd
    import synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    recs = [bench_c1(args, dev, stream)]
    torch.cuda.empty_cache()
    reps = max(1, min(args.steps, 3))
    for name, m, r, P, L, mode, n, points, ops, ops_src, kname in CONFIGS:
        perm = rmd.RM_PERM_NONE if mode == "none" else rmd.RM_PERM_PFHT
        dec = rmd.Decoder(m, r, P, L, seed=SEED, perm_mode=perm)
        N = 1 << m
        bits = torch.empty((n, N // 8), dtype=torch.uint8, device=dev)
        pm = torch.empty((n,), dtype=torch.float32, device=dev)
        total_ms, fers = 0.0, {}
        for k, e in enumerate(points):
            x, llr = synth.frames(m, r, n, e, seed=SEED + k)
            t = torch.from_numpy(llr).to(dev)

            def step():
                dec.decode(t, out_bits=bits, out_metric=pm, stream=stream)

            for _ in range(max(1, args.warmup)):
                step()
            total_ms += hip_ms(stream, step, reps)
            xb = synth.unpack_bits(bits.cpu().numpy(), N)
            fers[str(e)] = fer_ci(int(np.any(xb != x, axis=1).sum()), n)
        ms = total_ms / len(points)
        fps = n / (ms / 1e3)
        log(f"{name.split(',')[0]} P={P} L={L}: {fps / 1e6:.3f} M frames/s")
        achieved = ops * fps / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": round(ALU_PEAK_TOPS, 4), "unit": "TFLOP/s",
                "frac": round(achieved / ALU_PEAK_TOPS, 5), "traffic": None, "ops_per_frame": ops,
                "ops_source": ops_src, "kernel": kname, "avg_launch_ms": round(ms, 4)}
        recs.append({"metric": "frames/s", "value": round(fps, 1), "unit": "frames/s", "n_gpus": 1, "steps": reps,
                     "warmup": max(1, args.warmup), "ms_per_step": round(ms, 4), "higher_is_better": True,
                     "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                     "config": {"workload": name + ", BPSK/AWGN", "frames_per_point": n, "ebn0_db": points},
                     "info_gbit_s": round(fps * rmd.code_dimension(m, r) / 1e9, 4), "fer": fers, "roofline": roof})
        dec.close()
        torch.cuda.empty_cache()
    return recs


if __name__ == "__main__":
    main()
