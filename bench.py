#!/usr/bin/env python3
"""F-statistic grid throughput on one MI355X.

One step = one fstat_grid call over the whole all-sky grid of the 2-day
workload: N = 344656 samples at dt = 0.5 s, nfft = 2^20, 1024 sky positions
(uniform on the sphere) x 16 spindowns in [-1e-9, 0] Hz/s = 16384 nodes, FP64
phase with FP32 resampling/FFT/combination, two-step (Fourier x2 + linear)
resampling, the full F map on bins [0, nfft/2) written to HBM.  Inputs are
resident on the GPU before the timed region.

Prints one JSON line: nodes/s, the roofline of the dominant kernel (timed
with HIP events around each launch, on the launch stream), the plain FP64
one-node-per-launch path on a subset of the grid, the FP32-vs-FP64 difference
of F on sampled nodes, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
FP64_PEAK_GFLOPS = 78600.0   # MI355X vector FP64
PROFILES = os.path.join(ROOT, "profiles")
# sources that compile into the two FFT-pass kernels
KERNEL_SOURCES = ("grid.hip", "tiles.h", "moments.h", "fft_block.h", "cplx.h", "demod.h", "geometry.h", "internal.h")
# sources of the refinement kernels (F and its adjoint at continuous parameters)
GRAD_SOURCES = ("grad.hip", "candidate.h", "moments.h", "cplx.h", "demod.h", "geometry.h", "internal.h")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--max-batch", type=int, default=0, help="nodes per FFT batch (0 = library default)")
    ap.add_argument("--plain-nodes", type=int, default=256)
    ap.add_argument("--plain-repeats", type=int, default=5)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (uneven segments, 6-day grid, refinement)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--interbin", action="store_true",
                    help="the same grid with nfft = nextpow2(N) = 2^19 and interbinning (Eq. intbin): F at the "
                         "Fourier bins and the half bins, as many output frequencies as the padded 2^20 map")
    ap.add_argument("--lattice", choices=("deep_holes", "covering"), default=None,
                    help="the grid of Sec. IV instead of the uniform one: every node of the constrained A4* "
                         "lattice over the whole sky and the same spindown range, with its rule for nu; "
                         "the F map is written 16384 nodes at a time")
    ap.add_argument("--counters", action="store_true",
                    help="short run for hardware-counter collection: one grid call on two node batches "
                         "of the benchmark's (autotuned) schedule "
                         "and a 1 GiB device copy of known size (the calibration of the byte counters)")
    ap.add_argument("--log", default=None, metavar="FILE",
                    help="append to FILE one JSON line per node chunk of every timed step (the chunk's node "
                         "range, the place a resumed run restarts from, its HIP-event time and nodes/s), then "
                         "the result line")
    ap.add_argument("--leg", choices=("uneven_segments", "large6d", "refinement"), default=None,
                    help="run one of the other workloads alone and print its JSON object (for profiling)")
    ap.add_argument("--refine-counters", action="store_true",
                    help="short run for FP64 instruction counters: one F + gradient call (fstat_grad) on the "
                         "4096 refinement candidates")
    return ap.parse_args()


def counters_run(args):
    """One grid call on two node batches of the benchmark's schedule, then a
    plain copy of exactly 2^30 bytes: the copy's FETCH_SIZE / WRITE_SIZE
    readings give the scale from counter units to bytes moved."""
    import torch
    from paper_1003_0844_amd import fstat
    w, x, nodes = workload()
    ib = bool(args.interbin)
    nfft = (w.nfft // 2) if ib else w.nfft
    half = nfft // 2
    # the benchmark's schedule: autotuned (read back from FSTAT_TUNE_CACHE when
    # the benchmark run wrote it there) or the given batch
    plan = fstat.Plan([fstat.SegmentSpec(x=x, dt=w.dt, n_days=w.days, nfft=nfft)], fstat.default_detector(),
                      fstat.Ephemeris(), interp=fstat.LINEAR_UP2, prec=fstat.FP32, max_batch=args.max_batch,
                      autotune=True)
    sub = nodes[:2 * plan.schedule()["batch"]]
    F = torch.empty((len(sub), (2 if ib else 1) * half), dtype=torch.float32, device="cuda")
    plan.grid_map(sub, 0, half, F, interbin=ib)
    torch.cuda.synchronize()
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    dst.copy_(src)
    torch.cuda.synchronize()
    ev[0].record()
    dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    print(json.dumps({"counters_run": "done", "grid_nodes": len(sub), "nfft": nfft, "interbin": ib,
                      "schedule": plan.schedule(), "copy_bytes_each_way": 1 << 30,
                      "copy_ms": round(ms, 4), "copy_GBps_read_plus_write": round(2 * (1 << 30) / ms / 1e6, 1)}),
          flush=True)


def source_digest(names) -> str:
    """First 16 hex digits of the SHA-256 of the named kernel sources and of
    the library's device compile flags (include paths left out), so that a
    change of either retires the counter records taken before it."""
    import hashlib
    from paper_1003_0844_amd import _build
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1003_0844_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    h.update(" ".join(f for f in _build.common_flags() if not f.startswith("-I")).encode())
    return h.hexdigest()[:16]


def kernel_digest() -> str:
    """The digest of the pass-kernel sources (source_digest)."""
    return source_digest(KERNEL_SOURCES)


def traffic_record(kernel: str, sched: dict, nfft: int, interbin: bool):
    """HBM bytes per launch of a kernel from the committed counter summaries
    (profiles/*traffic*.md, lines 'record: key=value ...'), or None when no
    record matches the kernel, its FFT length, schedule and output kind, and
    the current kernel sources."""
    digest = kernel_digest()
    want = "C%d,batch%d" % (sched["C"], sched["batch"])
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if "traffic" not in name:
            continue
        with open(os.path.join(PROFILES, name)) as f:
            for line in f:
                line = line.strip().strip("`")
                if not line.startswith("record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line[len("record:"):].split() if "=" in t)
                if (kv.get("kernel") == kernel and kv.get("schedule") == want and kv.get("digest") == digest
                        and kv.get("nfft") == str(nfft) and kv.get("interbin") == str(int(interbin))):
                    return float(kv["bytes_per_launch"])
    return None


def flop_record(kernels: str, n: int):
    """FP64 floating-point operations per candidate of the refinement kernels
    from the committed counter summaries (profiles/*flops*.md, lines
    'record: kernels=... n=... digest=... flop_per_candidate=...'), or None
    when none matches the current sources of those kernels."""
    digest = source_digest(GRAD_SOURCES)
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if "flops" not in name:
            continue
        with open(os.path.join(PROFILES, name)) as f:
            for line in f:
                line = line.strip().strip("`")
                if not line.startswith("record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line[len("record:"):].split() if "=" in t)
                if kv.get("kernels") == kernels and kv.get("n") == str(n) and kv.get("digest") == digest:
                    return float(kv["flop_per_candidate"])
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload():
    import numpy as np
    from paper_1003_0844_amd import fstat, synth
    w = synth.GRID2D
    g, x, sigs = synth.segment_data(w)
    alpha, delta = synth.sky_uniform(g, w.n_sky)
    fd = synth.spindown_grid(w.n_fdot)
    nodes = fstat.nodes_array(np.repeat(alpha, w.n_fdot), np.repeat(delta, w.n_fdot), np.tile(fd, w.n_sky))
    return w, x, nodes


def copy_probe_gbps():
    """The best bandwidth (one read + one write per byte) of the library's
    streaming copy over a few grid sizes, on 2^30 bytes."""
    import torch
    from paper_1003_0844_amd import fstat
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    best, best_blocks = 0.0, 0
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for blocks in (256, 512, 1024, 2048, 4096, 8192):
        fstat.copy_probe(dst, src, blocks)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(5):
            fstat.copy_probe(dst, src, blocks)
        ev[1].record()
        torch.cuda.synchronize()
        gbps = 2 * 5 * (1 << 30) / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9
        if gbps > best:
            best, best_blocks = gbps, blocks
    del src, dst
    torch.cuda.empty_cache()
    return best, best_blocks


def spill_write_probe_gbps(nodes: int, R: int, C: int, b2: int) -> float:
    """The rate of the first FFT pass's spill stores alone (the library's
    probe of the same workgroups, thread-to-bin map and layout, without the
    transform): bytes over the median of 5 timed launches after one untimed."""
    import torch
    from paper_1003_0844_amd import fstat
    buf = torch.empty((nodes * R * C, 4), dtype=torch.float32, device="cuda")
    fstat.spill_write_probe(buf, nodes, R, C, b2)
    torch.cuda.synchronize()
    ts = []
    for _ in range(5):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        fstat.spill_write_probe(buf, nodes, R, C, b2)
        ev[1].record()
        torch.cuda.synchronize()
        ts.append(ev[0].elapsed_time(ev[1]))
    ts.sort()
    del buf
    torch.cuda.empty_cache()
    return nodes * R * C * 16 / (ts[2] * 1e-3) / 1e9


def lattice_workload(w, x, rule):
    """The full-sky lattice of the segment (Sec. IV, C0 = 3/4) over the uniform
    grid's spindown range, f_sky at the top of the band."""
    from paper_1003_0844_amd import fstat, synth
    spec = fstat.SegmentSpec(x=x, dt=w.dt, n_days=w.days, nfft=w.nfft)
    r = fstat.NU_COVERING if rule == "covering" else fstat.NU_DEEP_HOLES
    lat = fstat.Lattice.for_segment(spec, fstat.default_detector(), fstat.Ephemeris(), rule=r)
    fd = synth.spindown_grid(w.n_fdot)
    nodes = lat.nodes(synth.F_REF + 1 / (2 * w.dt), float(fd.min()), float(fd.max()), fstat.Ephemeris())
    return lat, nodes


def _oracle_worker(job):
    """One worker process of the CPU baseline: the oracle on its share of the
    nodes until the deadline.  Returns (nodes done, seconds)."""
    x, dt, days, nfft, ib, nodes, budget_s = job
    from oracle import method, model
    from paper_1003_0844_amd import synth
    det, eph = model.default_detector(), model.Ephemeris()
    seg = method.Segment(x=x, dt=dt, n_days=days, f_ref=synth.F_REF, sigma2=1.0, nfft=nfft)
    fn = method.fstat_bins_interbinned if ib else method.fstat_bins
    t0 = time.perf_counter()
    done = 0
    for nd in nodes:
        fn(seg, float(nd["fdot"]), float(nd["alpha"]), float(nd["delta"]), det, eph, method.LINEAR_UP2, dft="fft",
           bin_offset=float(nd["bin_offset"]))
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return done, time.perf_counter() - t0


def cpu_cores() -> int:
    """Host cores the baseline may use: those this process may run on, at
    most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, x, nodes, budget_s, nfft, ib):
    """The FP64 oracle (resampling method, FP64 numpy FFT for the DFT step) on
    nodes of the same grid, one single-threaded worker process per host core,
    each on its own nodes until the time budget is used; nodes/s = all nodes
    done over the wall time of the pool."""
    import multiprocessing as mp
    cores = cpu_cores()
    per = max(4, int(budget_s) + 4)    # more nodes than a worker finishes in the budget
    jobs = [(x, w.dt, w.days, nfft, ib, nodes[c * per:(c + 1) * per], budget_s) for c in range(cores)]
    env_threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_threads:
        os.environ[k] = "1"   # one thread per worker (inherited by the spawned processes)
    try:
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            res = pool.map(_oracle_worker, jobs, chunksize=1)
        wall = time.perf_counter() - t0
    finally:
        for k, v in env_threads.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    done = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return {"value": done / wall, "unit": "nodes/s", "cores": cores, "kind": "oracle",
            "sample": "%d nodes of the same grid (full band, %d %s each) in %d single-threaded worker processes "
                      "(one per host core), FP64 resampling method with numpy FP64 FFT; %.1f s wall incl. process "
                      "start and each worker's 2x upsampling of the segment (%.1f s in the slowest worker's loop)"
                      % (done, nfft // 2, "bins and half bins" if ib else "bins", cores, wall, busy)}


def _median_time(fn, reps):
    import torch
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    ts.sort()
    return ts[len(ts) // 2]


def _call_bytes(plan, fn):
    """Algorithmic HBM bytes of one eager grid call, from the library's
    per-launch accounting (sky records, spill, outputs)."""
    import torch
    from paper_1003_0844_amd import fstat
    plan.profile(True)
    fn()
    torch.cuda.synchronize()
    b = sum(plan.profile_read(k)["bytes"] for k in (fstat.K_SKY, fstat.K_PASS1, fstat.K_PASS2))
    plan.profile(False)
    return b


def uneven_leg():
    """256 segments of 1-6 sidereal days with 0-10 % gaps, 64 sky x 8 spindowns
    each (131072 nodes, nfft 2^19-2^21), per-node maxima over the bins common to
    all segments, the whole call replayed as one launch of its HIP graph."""
    import numpy as np
    import torch
    from paper_1003_0844_amd import fstat, synth
    u = synth.UNEVEN
    t0 = time.perf_counter()
    segs, grids = synth.uneven_segments(u)
    specs = [fstat.SegmentSpec(x=x, dt=u.dt, n_days=d, t0=t, mask=m) for d, t, x, m in segs]
    nodes = np.concatenate([fstat.nodes_array(a, dl, fd, i) for i, (a, dl, fd) in enumerate(grids)])
    k_hi = min(1 << int(math.ceil(math.log2(2 * len(x)))) for _, _, x, _ in segs) // 2
    plan = fstat.Plan(specs, fstat.default_detector(), fstat.Ephemeris(), interp=fstat.LINEAR_UP2, prec=fstat.FP32,
                      autotune=True)
    log("uneven: data and plan (autotuned) in %.1f s" % (time.perf_counter() - t0))
    nbytes = _call_bytes(plan, lambda: plan.grid_max(nodes, 0, k_hi))
    graph = plan.graph_max(nodes, 0, k_hi)
    graph.launch()
    s = _median_time(graph.launch, 3)
    ref = (graph.outputs["Fmax"].clone(), graph.outputs["kmax"].clone())
    graph.close()
    scheds = {}
    for i, (d, _, _, _) in enumerate(segs):
        scheds.setdefault(str(d), plan.schedule(i))
    del plan
    torch.cuda.empty_cache()
    gbs = nbytes / s / 1e9
    log("uneven: %.0f nodes/s (%.3f s per launch), %.1f GB/s algorithmic" % (len(nodes) / s, s, gbs))
    # the same call as one launch of the persistent kernel, recorded in a graph
    pp = fstat.Plan(specs, fstat.default_detector(), fstat.Ephemeris(), interp=fstat.LINEAR_UP2, prec=fstat.FP32,
                    launch=fstat.LAUNCH_PERSISTENT)
    gp = pp.graph_max(nodes, 0, k_hi)
    gp.launch()
    sp = _median_time(gp.launch, 2)
    same = bool(torch.equal(gp.outputs["Fmax"], ref[0]) and torch.equal(gp.outputs["kmax"], ref[1]))
    gp.close()
    pp.status()
    del pp
    torch.cuda.empty_cache()
    log("uneven, persistent launch: %.0f nodes/s (%.3f s per launch), outputs equal: %s" % (len(nodes) / sp, sp, same))
    return {"workload": u.name + ", per-node maximum on bins [0, %d), LINEAR_UP2, FP32 with FP64 phase" % k_hi,
            "launch": "one HIP-graph launch of the whole call as passes (median of 3)",
            "nodes": int(len(nodes)), "value": round(len(nodes) / s, 1), "unit": "nodes/s", "s_per_call": round(s, 4),
            "bytes_per_node": round(nbytes / len(nodes)), "path_GBps": round(gbs, 1),
            "path_frac": round(gbs / HBM_PEAK_GBS, 4), "schedule_by_days": scheds,
            "persistent": {"launch": "one HIP-graph launch of one persistent kernel over the whole call (median of 2)",
                           "value": round(len(nodes) / sp, 1), "unit": "nodes/s", "s_per_call": round(sp, 4),
                           "outputs_equal_to_passes": same}}


def large6d_leg():
    """6 sidereal days (N = 1033968, nfft = 2^21), 8192 sky x 32 spindowns,
    per-node maximum over the band: FP32 on the whole grid, FP64 (autotuned
    batches) on its first 8192 nodes, and their per-node maxima compared."""
    import numpy as np
    import torch
    from paper_1003_0844_amd import fstat, synth
    w = synth.LARGE6D
    g, x, _ = synth.segment_data(w)
    al, de = synth.sky_uniform(g, w.n_sky)
    fd = synth.spindown_grid(w.n_fdot)
    nodes = fstat.nodes_array(np.repeat(al, w.n_fdot), np.repeat(de, w.n_fdot), np.tile(fd, w.n_sky))
    half = w.nfft // 2
    spec = fstat.SegmentSpec(x=x, dt=w.dt, n_days=w.days, nfft=w.nfft)
    res = {"workload": w.name + ", per-node maximum on bins [0, nfft/2), LINEAR_UP2", "nodes": int(len(nodes))}
    p32 = fstat.Plan([spec], fstat.default_detector(), fstat.Ephemeris(), interp=fstat.LINEAR_UP2, prec=fstat.FP32,
                     autotune=True)
    sub = nodes[:8192]
    p32.grid_max(sub, 0, half)   # warm-up
    torch.cuda.synchronize()
    p32.profile(True)
    t = time.perf_counter()
    F32, k32 = p32.grid_max(nodes, 0, half)
    torch.cuda.synchronize()
    s32 = time.perf_counter() - t
    b32 = sum(p32.profile_read(k)["bytes"] for k in (fstat.K_SKY, fstat.K_PASS1, fstat.K_PASS2))
    p32.profile(False)
    gbs = b32 / s32 / 1e9
    res["fp32"] = {"value": round(len(nodes) / s32, 1), "unit": "nodes/s", "s": round(s32, 3),
                   "bytes_per_node": round(b32 / len(nodes)), "path_GBps": round(gbs, 1),
                   "path_frac": round(gbs / HBM_PEAK_GBS, 4), "schedule": p32.schedule()}
    F32s, k32s = F32[:len(sub)].double().cpu().numpy(), k32[:len(sub)].cpu().numpy()
    del p32, F32, k32
    torch.cuda.empty_cache()
    log("6-day FP32: %.0f nodes/s, %.1f GB/s algorithmic" % (len(nodes) / s32, gbs))
    p64 = fstat.Plan([spec], fstat.default_detector(), fstat.Ephemeris(), interp=fstat.LINEAR_UP2, prec=fstat.FP64,
                     autotune=True)
    p64.grid_max(sub[:256], 0, half)
    torch.cuda.synchronize()
    t = time.perf_counter()
    F64, k64 = p64.grid_max(sub, 0, half)
    torch.cuda.synchronize()
    s64 = time.perf_counter() - t
    F64, k64 = F64.cpu().numpy(), k64.cpu().numpy()
    res["fp64_batched"] = {"value": round(len(sub) / s64, 1), "unit": "nodes/s", "nodes": len(sub),
                           "s": round(s64, 3), "schedule": p64.schedule()}
    del p64
    torch.cuda.empty_cache()
    res["fp32_vs_fp64_max_rel_err"] = float(np.max(np.abs(F32s - F64) / np.maximum(np.abs(F64), 1.0)))
    res["argmax_agree"] = "%d/%d" % (int(np.sum(k32s == k64)), len(sub))
    log("6-day FP64 batched: %.0f nodes/s; FP32 vs FP64 %.2e" % (len(sub) / s64, res["fp32_vs_fp64_max_rel_err"]))
    return res


def refine_leg(reps=5):
    """4096 candidates half a cell (per parameter) from a point of the 1-day
    workload (N = 43082, dt = 2 s, LINEAR_UP2): F and dF/d(f, fdot, alpha,
    delta) in FP64 (fstat_grad: forward kernel, then the adjoint)."""
    import numpy as np
    import torch
    from paper_1003_0844_amd import fstat, synth
    w = synth.TINY
    g, x, sigs = synth.segment_data(w)
    sig = sigs[0]
    plan = fstat.Plan([fstat.SegmentSpec(x=x, dt=w.dt, n_days=w.days, nfft=w.nfft)], fstat.default_detector(),
                      fstat.Ephemeris(), interp=fstat.LINEAR_UP2, prec=fstat.FP64)
    df = 1.0 / (w.nfft * w.dt)
    v_c = fstat.AU * 2 * math.pi / fstat.YEAR / fstat.C_LIGHT
    cell = np.array([df, 1.0 / (w.n * w.dt) ** 2, df / (synth.F_REF * v_c), df / (synth.F_REF * v_c)])
    P = torch.tensor(np.array([sig["f"], sig["fdot"], sig["alpha"], sig["delta"]])
                     + 0.5 * cell * synth.candidate_offsets(1003, 4096), dtype=torch.float64, device="cuda")
    plan.grad(P)
    torch.cuda.synchronize()
    if reps <= 1:
        log("refinement counters run: one warm-up call and this one, 4096 candidates")
        return None
    s = _median_time(lambda: plan.grad(P), reps)
    res = {"workload": "4096 candidates at +-1/2 cell around a 1-day point (N=43082, dt=2 s), LINEAR_UP2, FP64",
           "value": round(4096 / s, 1), "unit": "candidates/s", "s_per_call": round(s, 5)}
    flops = flop_record("k_eval+k_adjoint", w.n)
    if flops is not None:
        gf = flops * 4096 / s / 1e9
        res["alu"] = {"bound": "alu", "achieved": round(gf, 1), "peak": FP64_PEAK_GFLOPS, "unit": "GFLOP/s",
                      "frac": round(gf / FP64_PEAK_GFLOPS, 4), "flop_per_candidate": flops}
    log("refinement: %.0f candidates/s" % (4096 / s))
    return res



def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the F-statistic grid shards over sky positions, "
              "and bench.py measures one GPU's share only: run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.counters:
        counters_run(args)
        return
    if args.refine_counters:
        refine_leg(reps=1)
        return
    if args.leg:
        leg = {"uneven_segments": uneven_leg, "large6d": large6d_leg, "refinement": refine_leg}[args.leg]
        print(json.dumps({args.leg: leg()}), flush=True)
        return
    import numpy as np
    import torch
    from paper_1003_0844_amd import fstat

    w, x, nodes = workload()
    lat = None
    if args.lattice:
        lat, nodes = lattice_workload(w, x, args.lattice)
        log("lattice (%s): theta %.4f, %d nodes" % (args.lattice, lat.theta, len(nodes)))
    nn = len(nodes)
    chunk = min(nn, 16384)
    ib = bool(args.interbin)
    nfft = (w.nfft // 2) if ib else w.nfft   # interbinning: nextpow2(N) instead of nextpow2(2N)
    half = nfft // 2
    width = 2 * half if ib else half
    log("workload: %s%s; building plan (autotuned)" % (w.name, ", interbinned at nfft %d" % nfft if ib else ""))
    t_plan = time.perf_counter()
    plan = fstat.Plan([fstat.SegmentSpec(x=x, dt=w.dt, n_days=w.days, nfft=nfft)], fstat.default_detector(),
                      fstat.Ephemeris(), interp=fstat.LINEAR_UP2, prec=fstat.FP32, max_batch=args.max_batch,
                      autotune=True)
    sched = plan.schedule()
    log("schedule: %s (plan built in %.2f s, tuning included unless read from FSTAT_TUNE_CACHE)"
        % (sched, time.perf_counter() - t_plan))
    F = torch.empty((chunk, width), dtype=torch.float32, device="cuda")

    def step(marks=None):
        for c0 in range(0, nn, chunk):
            part = nodes[c0:c0 + chunk]
            plan.grid_map(part, 0, half, F[:len(part)], interbin=ib)
            if marks is not None:   # --log: an event after each node chunk
                ev = torch.cuda.Event(enable_timing=True)
                ev.record()
                marks.append((c0, c0 + len(part), ev))

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup step %d done" % i)
    plan.profile(True)
    # with --log, an event after every node chunk of every step (no
    # synchronisation inside the timed region)
    marks = [] if args.log else None
    start = torch.cuda.Event(enable_timing=True) if args.log else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if start is not None:
        start.record()
    for i in range(args.steps):
        step(marks)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    chunk_log = []
    if marks is not None:
        prev = start
        for j, (c0, c1, ev) in enumerate(marks):
            chunk_log.append({"step": j // -(-nn // chunk), "nodes": [c0, c1], "ms": round(prev.elapsed_time(ev), 3)})
            prev = ev
    if nn > chunk:   # leave the first chunk's map in F for the FP64 comparison
        plan.grid_map(nodes[:chunk], 0, half, F, interbin=ib)
        torch.cuda.synchronize()
    log("timed %d steps: %.3f s" % (args.steps, el))
    prof = {k: plan.profile_read(k) for k in (fstat.K_SKY, fstat.K_PASS1, fstat.K_PASS2, fstat.K_OTHER)}
    plan.profile(False)
    names = {fstat.K_SKY: "k_sky_prep", fstat.K_PASS1: "k_pass1", fstat.K_PASS2: "k_pass2"}
    dom = max(names, key=lambda k: prof[k]["ms"])
    dp = prof[dom]
    avg_ms = dp["ms"] / max(1, dp["launches"])
    bytes_per_launch = dp["bytes"] / max(1, dp["launches"])
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    kernels = {names[k]: {"launches": prof[k]["launches"], "avg_us": 1e3 * prof[k]["ms"] / max(1, prof[k]["launches"]),
                          "GBps": prof[k]["bytes"] / max(1e-12, prof[k]["ms"] * 1e-3) / 1e9} for k in names}
    step_ms = 1e3 * el / args.steps
    value = nn * args.steps / el
    # whole-path roofline: algorithmic bytes of every kernel of a step over the step time
    step_bytes = sum(prof[k]["bytes"] for k in names) / args.steps
    path_gbs = step_bytes / (el / args.steps) / 1e9

    # the plain path: all-FP64, one node per launch, on the first nodes of the
    # grid, timed over several calls (median)
    sub = nodes[:args.plain_nodes]
    plan64 = fstat.Plan([fstat.SegmentSpec(x=x, dt=w.dt, n_days=w.days, nfft=nfft)], fstat.default_detector(),
                        fstat.Ephemeris(), interp=fstat.LINEAR_UP2, prec=fstat.FP64, max_batch=1)
    F64 = torch.empty((len(sub), width), dtype=torch.float64, device="cuda")
    plan64.grid_map(sub, 0, half, F64, interbin=ib)
    torch.cuda.synchronize()
    plain_runs = []
    for _ in range(max(1, args.plain_repeats)):
        t1 = time.perf_counter()
        plan64.grid_map(sub, 0, half, F64, interbin=ib)
        torch.cuda.synchronize()
        plain_runs.append(len(sub) / (time.perf_counter() - t1))
    plain = float(np.median(plain_runs))
    diff = (F[:len(sub)].double() - F64).abs() / torch.clamp(F64.abs(), min=1.0)
    err32 = float(diff.max().item())
    del F64, plan64
    log("plain FP64 path: %.1f nodes/s (median of %d calls of %d nodes); FP32 vs FP64 max |dF|/max(F,1) = %.2e"
        % (plain, len(plain_runs), len(sub), err32))

    out = {
        "metric": "F-stat grid nodes/sec (1 MI355X) at stated error; % HBM roofline vs plain path",
        "value": round(value, 1), "unit": "nodes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": ((w.name.replace("nfft=2^20", "nfft=2^19") + ", linear two-step resampling, "
                                 "interbinned F map on bins and half bins of [0, nfft/2)") if ib else
                                (w.name + ", linear two-step resampling, full F map on bins [0, nfft/2)"))
                               if lat is None else
                               ("2-day segment (N=%d, dt=%g s, nfft=%d), full-sky constrained A4* lattice of "
                                "Sec. IV (nu rule %s, C0=3/4, theta=%.4f), %d nodes, F map on bins [0, nfft/2) "
                                "with per-node bin offsets, written 16384 nodes at a time"
                                % (w.n, w.dt, nfft, args.lattice, lat.theta, nn)),
                   "nodes": nn, "n": w.n, "dt": w.dt, "nfft": nfft, "interbin": ib, "phase": "f64"},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_record(names[dom], sched, nfft, ib),
                     "avg_launch_us": round(1e3 * avg_ms, 2), "bytes_per_launch": bytes_per_launch,
                     "path_GBps": round(path_gbs, 1), "path_frac": round(path_gbs / HBM_PEAK_GBS, 4),
                     "path_bytes_per_node": round(step_bytes / nn)},
        "kernels": kernels,
        "schedule": sched,
        "plain_fp64_one_node_per_launch": {"value": round(plain, 1), "unit": "nodes/s",
                                           "nodes": len(sub), "calls": [round(v, 1) for v in plain_runs],
                                           "speedup": round(value / plain, 2)},
        "f32_vs_f64_max_rel_err": err32,
    }
    del F, plan
    torch.cuda.empty_cache()
    cp, cp_blocks = copy_probe_gbps()
    out["roofline"]["copy_probe_GBps"] = round(cp, 1)
    out["roofline"]["path_frac_of_copy"] = round(path_gbs / cp, 4)
    log("copy probe: %.1f GB/s (%d workgroups); path %.1f GB/s = %.1f %% of it" % (cp, cp_blocks, path_gbs,
                                                                                 100 * path_gbs / cp))
    if out["roofline"]["kernel"] == "k_pass1":
        b2 = sched["B2"] if sched["B2"] * 16 < 512 else 0   # the spill layout pass 1 writes (blocked or row-major)
        wp = spill_write_probe_gbps(sched["batch"], sched["R"], sched["C"], b2)
        out["roofline"]["spill_write_probe_GBps"] = round(wp, 1)
        out["roofline"]["frac_of_spill_write_probe"] = round(out["roofline"]["achieved"] / wp, 4)
        log("spill write probe: %.1f GB/s; k_pass1 %.1f GB/s = %.1f %% of it"
            % (wp, out["roofline"]["achieved"], 100 * out["roofline"]["achieved"] / wp))
    if not args.no_extra and lat is None and not ib:
        out["workloads"] = {"uneven_segments": uneven_leg(), "large6d": large6d_leg(), "refinement": refine_leg()}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, x, nodes, args.cpu_seconds, nfft, ib)
    if args.log:
        with open(args.log, "a") as f:
            for rec in chunk_log:
                n_c = rec["nodes"][1] - rec["nodes"][0]
                f.write(json.dumps(dict(rec, nodes_per_s=round(n_c / (rec["ms"] * 1e-3), 1),
                                        workload=out["config"]["workload"])) + "\n")
            f.write(json.dumps(out) + "\n")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
