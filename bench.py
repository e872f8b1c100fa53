"""Benchmark: TT-ICE stream throughput on one MI355X.

Headline workload (the largest single-GPU configuration): the high-order
reshaped stream.  4096 FP32 snapshots of a 256^3 scalar field (512 random
Fourier modes with integer k in [-16, 16]^3, amplitudes |k|^-3, phases
advancing linearly in time; seeded), each reshaped C-order to 8^8, arrive in
increments of 8 (512 increments); eps = 0.005; TT-ICE* (Algorithm 2, mean
skip rule) from empty cores.  Each increment (537 MB) is generated on the
device before its update, outside the timed region, so it is resident in
HBM when its update starts.

A step is one increment: one ttice_update call, the whole hot path over one
batch.  Every arm runs the whole 512-increment stream; exactly K of its
update calls (--steps, all 512 by default) are timed, at uniformly spaced
positions of the stream, each between device synchronisations (the call is
host-synchronous); value = 8 K / (their summed wall time).
full_stream_tensors_per_s = 4096 / (summed wall time of all 512 calls).
--warmup W runs the first W increments on a throwaway state first.

Arms: the chosen precision (--prec, default FP32 matrix-core level
products: the projections of the update, the TT-ICE* chain and the
next-level data; ||Y||, the residual's SVD, the re-orthogonalisation and
every rank decision stay FP64) and the plain FP64 path, same eps and
algorithm.  The video-shaped stream (2048 frames of 240x320x3 in increments
of 32, eps = 0.1, Algorithm 1) is reported beside it.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FIELD = dict(name="field256-8way", grid=256, modes=512, kmax=16, decay=3.0, snapshots=4096, batch=8, eps=0.005,
             seed=0, dims=(8,) * 8)
VIDEO = dict(name="video240", dims=(240, 320, 3), eps=0.1, frames=2048, batch=32, seed=0)
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=512,
                    help="timed update calls, spread uniformly over the stream (512 = all of them)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32", "bf16x3"],
                    help="arithmetic of the level products in the chosen arm")
    ap.add_argument("--snapshots", type=int, default=FIELD["snapshots"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-arm", action="store_true")
    ap.add_argument("--no-video", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--workload", default="field256", choices=["field256", "video240", "serving", "ablation", "gel"],
                    help="field256: the headline stream (default); video240: the video-shaped stream alone; "
                         "serving: the many-stream mix, reported as arrival-to-completion latency")
    ap.add_argument("--eps", type=float, default=None, help="ablation / gel: eps_des (default 0.1 / 0.01)")
    ap.add_argument("--seconds", type=float, default=10.0, help="serving: length of the arrival trace")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: Poisson arrivals per second")
    ap.add_argument("--streams", type=int, default=256, help="serving: number of streams")
    ap.add_argument("--workers", type=int, default=32, help="serving: worker threads of the server")
    ap.add_argument("--serving-prec", default="fp32", choices=["fp64", "fp32", "bf16x3"],
                    help="serving: the streams' precision")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, copy one increment device-to-device (a plain copy kernel of known "
                         "size whose FETCH_SIZE / WRITE_SIZE counters calibrate the projection kernel's)")
    return ap.parse_args()


def field_source():
    from paper_2211_12487_amd import synth
    w = FIELD
    gen = synth.DeviceFourierField(grid=w["grid"], components=1, n_modes=w["modes"], kmax=w["kmax"],
                                   decay=w["decay"], seed=w["seed"])
    N, dims = w["batch"], w["dims"]

    def increment(k):
        return gen.snapshots(k * N, N).reshape((N,) + dims).contiguous()
    return increment


def timed_positions(n_inc, k):
    """The K timed increments: all of them when K >= n_inc, else K uniformly
    spaced positions (the centres of K equal parts of the stream)."""
    if k >= n_inc:
        return set(range(n_inc))
    return {int((j + 0.5) * n_inc / k) for j in range(k)}


def run_field_arm(increment, n_inc, prec, steps, warmup):
    """One arm over the whole stream: per-increment update wall times, the
    timed subset, final ranks, skipped increments and the
    level-1 projection kernel's event timings."""
    import torch
    from paper_2211_12487_amd.ttice import TTICE
    w = FIELD
    if warmup > 0:
        g = TTICE(w["dims"], w["eps"], prec=prec, algo="star")
        for k in range(warmup):
            g.update(increment(k))
        g.close()
    g = TTICE(w["dims"], w["eps"], prec=prec, algo="star")
    g.profile(True)
    pos = timed_positions(n_inc, steps)
    lat, timed = [], []
    skipped = 0
    for k in range(n_inc):
        Y = increment(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = g.update(Y)
        dt = time.perf_counter() - t0
        lat.append(dt)
        if k in pos:
            timed.append(dt)
        skipped += int(info["skipped"])
        del Y
        if k % 64 == 63:
            print(f"  {prec}: {k + 1}/{n_inc} increments, {sum(lat):.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ks = g.kernel_stats()
    ranks = g.ranks()
    g.close()
    N = w["batch"]
    return dict(value=N * len(timed) / sum(timed), timed=len(timed), timed_seconds=sum(timed),
                full_stream_tensors_per_s=N * n_inc / sum(lat), seconds=sum(lat),
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                ranks=ranks, skipped=skipped, kstats=ks)


def run_video(prec):
    """The video-shaped stream once (Algorithm 1 from empty cores): tensors/s
    and final ranks."""
    import torch
    from paper_2211_12487_amd import synth
    from paper_2211_12487_amd.ttice import TTICE
    w = VIDEO
    Y = torch.from_numpy(np.concatenate(list(synth.video_stream(w["frames"], w["batch"], seed=w["seed"])))).cuda()
    for rep in range(2):  # the first pass loads and allocates
        g = TTICE(w["dims"], w["eps"], prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(0, w["frames"], w["batch"]):
            g.update(Y[k:k + w["batch"]])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ranks = g.ranks()
        g.close()
    return dict(tensors_per_s=w["frames"] / dt, seconds=dt, ranks=ranks)


# level-1 projection kernel of each arm: (name, source file)
# the level-1 projection kernel of each arm on the headline stream (8-row
# unfoldings: the short-column kernel in FP64 and FP32, the split-BF16
# matrix-core kernel otherwise) and its source file
PROJ_KERNEL = {
    "fp64": ("k_proj_short<float,double>", "proj_short.hip"),
    "fp32": ("k_proj_short<float,float>", "proj_short.hip"),
    "bf16x3": ("k_proj_bf3<float,4,1,1>", "proj_lp.hip"),
}


def measured_traffic(prec):
    """HBM bytes per launch of the arm's level-1 projection kernel on the
    headline stream from the committed counter summary, or None when that
    summary is missing or was taken on another revision of the kernel's
    source."""
    import hashlib
    name, src_file = PROJ_KERNEL[prec]
    path = os.path.join(ROOT, "profiles", f"{name.split('<')[0]}_{prec}_field256_traffic.txt")
    try:
        fields = dict(line.split(":", 1) for line in open(path).read().splitlines()
                      if ":" in line and not line.startswith("#"))
        src = os.path.join(ROOT, "paper_2211_12487_amd", "csrc", src_file)
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if fields.get("kernel_source_sha256", "").strip() != digest:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def roofline(kstats, prec):
    """Level-1 projection kernel (U_1^T Y and ||Y(b)||^2 in one pass over the
    increment): algorithmic bytes per launch = the increment read once + the
    r_1 coefficient rows and the per-column energies written (FP64);
    duration = mean of its launches' own start/end events over the stream."""
    n = kstats.get("launches", 0)
    if not n:
        return None
    avg_s = kstats["total_ms"] / n * 1e-3
    bytes_per_launch = kstats["bytes"] / n
    achieved = bytes_per_launch / avg_s / 1e9
    return dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=measured_traffic(prec),
                kernel=f"{PROJ_KERNEL[prec][0]} (level-1 projection, {prec} products)",
                launches=n, avg_us=avg_s * 1e6, bytes_per_launch=bytes_per_launch)


def cpu_baseline():
    """The FP64 NumPy oracle on a bounded sample of the headline stream: its
    first increment (8 snapshots) from empty cores, the same seeded field
    drawn on the host."""
    from oracle import TTICE as Oracle
    from paper_2211_12487_amd import synth
    w = FIELD
    Y = next(synth.fourier_field_stream(w["batch"], w["batch"], grid=w["grid"], components=1, n_modes=w["modes"],
                                        kmax=w["kmax"], decay=w["decay"], seed=w["seed"]))
    Y = Y.reshape((w["batch"],) + w["dims"])
    o = Oracle(w["dims"], w["eps"], algo="star")
    t0 = time.perf_counter()
    o.update(Y)
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        blas = ",".join(sorted({i.get("internal_api", "?") for i in threadpool_info()}))
    except Exception:  # pragma: no cover
        blas = "unknown"
    return dict(value=w["batch"] / dt, unit="tensors/s", cores=cores, kind="oracle", blas=blas,
                sample=f"first increment ({w['batch']} snapshots, 537 MB) of the stream from empty cores, NumPy FP64 "
                       f"+ LAPACK, BLAS threads up to {cores}", seconds=dt)


SERVING_SHAPES = [(32, 32, 3), (64, 64, 3), (128, 128, 3), (32, 32, 32)]
SERVING_EPS = [0.01, 0.05, 0.1]


def serving(a):
    """Many-stream serving mix: `streams` streams with shapes drawn from
    SERVING_SHAPES and eps from SERVING_EPS; Poisson arrivals at `rate` per
    second, each an increment of 1..64 tensors for a uniformly drawn stream.
    Every increment is generated on the device before the clock starts (a sum
    of five separable products of random cosine profiles with N(0,1) weights
    plus 1e-3 noise, FP32), so inputs are resident in HBM; at its arrival time
    it is submitted to the server.  Latency = completion - scheduled arrival
    (the driver's polling adds up to one loop period)."""
    import torch
    from paper_2211_12487_amd import synth
    from paper_2211_12487_amd.ttice import Server
    rng = np.random.default_rng(0)
    srv = Server(workers=a.workers, budget_bytes=200 << 30)
    kinds = [(SERVING_SHAPES[int(rng.integers(len(SERVING_SHAPES)))], SERVING_EPS[int(rng.integers(3))])
             for _ in range(a.streams)]
    n_req = int(rng.poisson(a.rate * a.seconds))
    times = np.sort(rng.uniform(0.0, a.seconds, n_req))
    who = rng.integers(0, a.streams, n_req)
    sizes = rng.integers(1, 65, n_req)
    # each stream declares its capacity (the tensors it will receive), which
    # bounds its reservation
    total = np.bincount(who, weights=sizes, minlength=a.streams).astype(np.int64)
    sids = [srv.add_stream(dims, eps, prec=a.serving_prec, max_batch=64, max_tensors=max(64, int(total[s])))
            for s, (dims, eps) in enumerate(kinds)]
    if srv.stats()["waiting_streams"]:
        raise RuntimeError("serving: the budget does not hold every stream")
    gen = torch.cuda.Stream()
    g = torch.Generator(device="cuda")
    g.manual_seed(0)

    def make(dims, n):
        with torch.cuda.stream(gen):
            Y = synth.device_separable(dims, n, g)
        gen.synchronize()
        return Y

    print(f"serving: generating {n_req} increments", file=sys.stderr, flush=True)
    data = []
    for k in range(n_req):
        data.append(make(kinds[int(who[k])][0], int(sizes[k])))
        if k % 2000 == 1999:
            print(f"serving: generated {k + 1}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    print(f"serving: {a.streams} streams, {n_req} increments over {a.seconds:.0f} s", file=sys.stderr, flush=True)
    outstanding = {}
    lag, arrivals = [], []
    lat, tensors = [], 0
    t0 = time.perf_counter()
    k = 0
    last_report = t0
    while k < n_req or outstanding:
        now = time.perf_counter() - t0
        busy = False
        while k < n_req and times[k] <= now:
            outstanding[srv.submit(sids[int(who[k])], data[k])] = (times[k], int(sizes[k]))
            lag.append(time.perf_counter() - t0 - times[k])
            data[k] = None  # the server's ticket keeps the tensor alive
            k += 1
            busy = True
        for t in list(outstanding):
            done, status, _ = srv.poll(t)
            if done:
                if status != 0:
                    raise RuntimeError(f"serving update failed with status {status}")
                arr, n = outstanding.pop(t)
                lat.append(time.perf_counter() - t0 - arr)
                arrivals.append(arr)
                tensors += n
                busy = True
        if time.perf_counter() - last_report > 5.0:
            last_report = time.perf_counter()
            print(f"serving: {k}/{n_req} submitted, {len(lat)} done", file=sys.stderr, flush=True)
        if not busy:
            time.sleep(50e-6)
    wall = time.perf_counter() - t0
    counters = srv.stats()
    srv.close()
    lat_ms = np.array(lat) * 1e3
    steady = lat_ms[np.array(arrivals) >= min(1.0, a.seconds / 2)]  # after the streams' first increments
    return dict(
        metric="serving arrival-to-completion latency p99", value=float(np.percentile(lat_ms, 99)), unit="ms",
        n_gpus=1, steps=1, warmup=0, ms_per_step=wall * 1e3, higher_is_better=False, scaling="weak",
        vs_baseline=None, dtype={"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[a.serving_prec], data="synthetic",
        config=dict(workload=f"serving: {a.streams} streams of {SERVING_SHAPES}, eps in {SERVING_EPS}, "
                             f"increments of 1..64 tensors, Poisson {a.rate:.0f}/s for {a.seconds:.0f} s, "
                             f"{a.workers} workers, {a.serving_prec}"),
        p50_ms=float(np.percentile(lat_ms, 50)), p99_ms=float(np.percentile(lat_ms, 99)),
        max_ms=float(lat_ms.max()), submit_lag_p99_ms=float(np.percentile(np.array(lag) * 1e3, 99)),
        steady_p50_ms=float(np.percentile(steady, 50)), steady_p99_ms=float(np.percentile(steady, 99)),
        increments=len(lat), tensors_per_s=tensors / wall, grouped_launches=counters["groups"],
        grouped_increments=counters["grouped_increments"],
        offered_tensors_per_s=float(sizes.sum()) / a.seconds)


# Algorithm 2 ablation on ATARI-shaped synthetic runs: 210x160x3 frames
# (background, moving sprites, noise) reshaped to 30x28x40x3 as in the
# experiments, streamed run by run (one run = one increment)
ABLATION = dict(name="atari-shaped", frame=(210, 160, 3), dims=(30, 28, 40, 3), runs=24, run_len=(64, 160),
                seed=5)
VARIANTS = [("TT-ICE", dict(algo="plain")),
            ("Subselect", dict(algo="star", skip_rule="none", tau=2.0)),
            ("SS", dict(algo="star", skip_rule="mean", tau=2.0)),
            ("TT-ICE*", dict(algo="star", skip_rule="mean", tau=0.8))]


def run_variants(Yd, starts, dims, eps, variants):
    """Each variant on the same increments (Yd[starts[k]:starts[k+1]]): wall
    time, tensors/s, tensors used in core updates, skipped increments, final
    ranks, compression ratio (eq:compressionratio) and mean relative
    reconstruction error over the stored tensors (eq:MRRE)."""
    import torch
    from paper_2211_12487_amd.ttice import TTICE
    total = int(starts[-1])
    n_inc = len(starts) - 1
    warm = TTICE(dims, eps)  # first-use allocations and module load, not timed
    warm.update(Yd[: starts[1]])
    warm.close()
    results = {}
    for name, kw in variants:
        print(f"variant {name}", file=sys.stderr, flush=True)
        g = TTICE(dims, eps, prec="fp64", **kw)
        used = skipped = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n_inc):
            info = g.update(Yd[starts[k]:starts[k + 1]])
            used += info["used"]
            skipped += int(info["skipped"])
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        ranks = g.ranks()
        rre = []
        for k in range(0, total, 256):
            cnt = min(256, total - k)
            rec = g.reconstruct(k, cnt)
            ref = Yd[k:k + cnt].double()
            rre.append(((rec - ref).flatten(1).norm(dim=1) / ref.flatten(1).norm(dim=1)).cpu().numpy())
        d = len(dims)
        stored = sum(ranks[i] * dims[i] * ranks[i + 1] for i in range(d)) + ranks[d] * total
        results[name] = dict(seconds=secs, tensors_per_s=total / secs, tensors_used=int(used),
                             skipped_increments=skipped, ranks=ranks,
                             compression_ratio=total * math.prod(dims) / stored,
                             mean_rre=float(np.concatenate(rre).mean()))
        g.close()
    return results


def ablation(a):
    """Every Algorithm 2 variant of the experiments on ATARI-shaped runs."""
    import torch
    from paper_2211_12487_amd import synth
    w = ABLATION
    eps = 0.1 if a.eps is None else a.eps
    rng = np.random.default_rng(w["seed"])
    lens = rng.integers(w["run_len"][0], w["run_len"][1] + 1, w["runs"])
    total = int(lens.sum())
    h, wd, c = w["frame"]
    print(f"generating {total} frames {w['frame']}", file=sys.stderr, flush=True)
    Y = np.concatenate(list(synth.video_stream(total, 256, height=h, width=wd, channels=c, seed=w["seed"])))
    dims = w["dims"]
    Yd = torch.from_numpy(Y.reshape((total,) + dims)).cuda()
    results = run_variants(Yd, np.concatenate([[0], np.cumsum(lens)]), dims, eps, VARIANTS)
    star = results["TT-ICE*"]
    return dict(
        metric="TT-ICE* tensors/s on ATARI-shaped runs (all Algorithm 2 variants reported)",
        value=star["tensors_per_s"], unit="tensors/s", n_gpus=1, steps=1, warmup=1,
        ms_per_step=star["seconds"] * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=f"{w['name']}: {w['runs']} runs of {w['run_len'][0]}-{w['run_len'][1]} frames "
                             f"{h}x{wd}x{c} as {dims}, fp32 input, eps={eps}, one run per increment",
                    frames=total, eps=eps),
        variants=results)


# gel-shaped simulations: one 7x13x37x3x10 tensor per increment (the
# experiments' per-simulation reshape); a family of simulations sharing
# structure stands in as an exactly low-rank TT stream plus relative noise
GEL = dict(name="gel-shaped", dims=(7, 13, 37, 3, 10), tensors=400, ranks=(5, 15, 30, 10, 12), noise=1e-3, seed=9)


def gel(a):
    """TT-ICE and TT-ICE* with tau = 1 (the experiments' setting for these
    simulations) on gel-shaped tensors, one per increment."""
    import torch
    from paper_2211_12487_amd import synth
    w = GEL
    eps = 0.01 if a.eps is None else a.eps
    print(f"generating {w['tensors']} tensors {w['dims']}", file=sys.stderr, flush=True)
    Y = np.concatenate(list(synth.tt_lowrank_stream(w["dims"], w["ranks"], w["tensors"], 64, seed=w["seed"])))
    rng = np.random.default_rng(w["seed"] + 1)
    Y = (Y + w["noise"] * Y.std() * rng.standard_normal(Y.shape)).astype(np.float32)
    Yd = torch.from_numpy(Y).cuda()
    variants = [("TT-ICE", dict(algo="plain")), ("TT-ICE*", dict(algo="star", skip_rule="mean", tau=1.0))]
    results = run_variants(Yd, np.arange(w["tensors"] + 1), w["dims"], eps, variants)
    star = results["TT-ICE*"]
    return dict(
        metric="TT-ICE* tensors/s on gel-shaped simulations, one per increment (TT-ICE reported beside it)",
        value=star["tensors_per_s"], unit="tensors/s", n_gpus=1, steps=1, warmup=1,
        ms_per_step=star["seconds"] * 1e3, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=f"{w['name']}: {w['tensors']} tensors {w['dims']} (TT ranks {w['ranks']}, "
                             f"relative noise {w['noise']}), fp32 input, eps={eps}, one per increment",
                    tensors=w["tensors"], eps=eps),
        variants=results)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps(dict(error="this benchmark runs on one GPU only; multi-GPU sharding is "
                                    "design-only (see DESIGN.md)", n_gpus=a.gpus)))
        sys.exit(2)
    import torch
    from paper_2211_12487_amd import ttice
    ttice.lib()
    if a.workload == "serving":
        print(json.dumps(serving(a)), flush=True)
        return
    if a.workload == "ablation":
        print(json.dumps(ablation(a)), flush=True)
        return
    if a.workload == "gel":
        print(json.dumps(gel(a)), flush=True)
        return
    if a.workload == "video240":
        print(json.dumps(dict(chosen=run_video(a.prec), fp64=run_video("fp64"))), flush=True)
        return
    w = FIELD
    n_inc = (a.snapshots + w["batch"] - 1) // w["batch"]
    increment = field_source()
    print(f"field256: {n_inc} increments of {w['batch']} snapshots, timing the {a.prec} arm", file=sys.stderr,
          flush=True)
    chosen = run_field_arm(increment, n_inc, a.prec, a.steps, a.warmup)
    if a.copy_calibration:
        inc = increment(0)
        dst = torch.empty_like(inc)
        for _ in range(3):
            dst.copy_(inc)
        torch.cuda.synchronize()
        print(f"copy calibration: 3 device copies of {inc.numel() * inc.element_size()} bytes", file=sys.stderr,
              flush=True)
        del inc, dst
    fp64 = None
    if not a.no_fp64_arm and a.prec != "fp64":
        print("timing the fp64 arm", file=sys.stderr, flush=True)
        fp64 = run_field_arm(increment, n_inc, "fp64", a.steps, a.warmup)
    video = None
    if not a.no_video:
        print("video240: both arms", file=sys.stderr, flush=True)
        video = dict(chosen=run_video(a.prec), fp64=run_video("fp64"))
    serve = None
    if not a.no_serving:
        print("serving mix", file=sys.stderr, flush=True)
        sa = argparse.Namespace(**vars(a))
        sa.seconds = min(a.seconds, 5.0)
        serve = serving(sa)
    cpu = None
    if not a.no_cpu_baseline:
        print("timing the cpu oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
    out = dict(
        metric="tensors/s at fixed eps (chosen precision vs plain FP64), % HBM roofline, p99 update latency",
        value=chosen["value"], unit="tensors/s", n_gpus=1, steps=chosen["timed"], warmup=a.warmup,
        ms_per_step=chosen["timed_seconds"] / chosen["timed"] * 1e3, higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype={"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[a.prec], data="synthetic",
        config=dict(workload=f"{w['name']}: {n_inc * w['batch']} fp32 snapshots of a 256^3 field (512 Fourier modes, "
                             f"|k|^-3, k in [-16,16]^3) reshaped to 8^8, increments of {w['batch']}, eps={w['eps']}, "
                             f"TT-ICE* (Algorithm 2, mean rule) from empty cores",
                    snapshots=n_inc * w["batch"], batch=w["batch"], eps=w["eps"], prec=a.prec),
        full_stream_tensors_per_s=chosen["full_stream_tensors_per_s"], stream_seconds=chosen["seconds"],
        final_ranks=chosen["ranks"], skipped_increments=chosen["skipped"],
        p50_update_ms=chosen["p50_ms"], p99_update_ms=chosen["p99_ms"],
        fp64_arm=(dict(value=fp64["value"], full_stream_tensors_per_s=fp64["full_stream_tensors_per_s"],
                       stream_seconds=fp64["seconds"], final_ranks=fp64["ranks"],
                       skipped_increments=fp64["skipped"], p50_update_ms=fp64["p50_ms"],
                       p99_update_ms=fp64["p99_ms"]) if fp64 else None),
        speedup_vs_fp64=(chosen["full_stream_tensors_per_s"] / fp64["full_stream_tensors_per_s"] if fp64 else None),
        video240=(dict(chosen_tensors_per_s=video["chosen"]["tensors_per_s"],
                       fp64_tensors_per_s=video["fp64"]["tensors_per_s"], ranks=video["chosen"]["ranks"],
                       fp64_ranks=video["fp64"]["ranks"]) if video else None),
        serving=(dict(p50_ms=serve["p50_ms"], p99_ms=serve["p99_ms"], steady_p99_ms=serve["steady_p99_ms"],
                      tensors_per_s=serve["tensors_per_s"], grouped_launches=serve["grouped_launches"],
                      grouped_increments=serve["grouped_increments"], increments=serve["increments"],
                      workload=serve["config"]["workload"])
                 if serve else None),
        roofline=roofline(chosen["kstats"], a.prec),
        cpu_baseline=cpu,
    )
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
