"""Benchmark: TT-ICE stream compression throughput on one MI355X.

Workload (the video-shaped stream): 2048 FP32 frames of 240x320x3 arriving
in increments of 32, eps = 0.1 (fixed rank-8 separable background, four
moving Gaussian blobs, N(0, 1e-2) noise; seeded).  One step = the whole
stream compressed from empty cores (64 ttice_update calls), with every
increment already resident in HBM.  value = tensors/s = 2048 * steps /
(summed wall time of the steps).

Both arms run at the same eps and must reach the same TT-ranks: the chosen
precision (--prec, default split-BF16 matrix-core projections; the residual
SVD is FP64 in every arm) and the plain FP64 path.
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

WORKLOAD = dict(name="video240", dims=(240, 320, 3), eps=0.1, frames=2048, batch=32, seed=0)
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3"],
                    help="arithmetic of the level projections in the chosen arm (the residual SVD is FP64)")
    ap.add_argument("--frames", type=int, default=WORKLOAD["frames"])
    ap.add_argument("--cpu-increments", type=int, default=6,
                    help="increments of the stream the CPU oracle baseline compresses")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-arm", action="store_true")
    ap.add_argument("--workload", default="video240", choices=["video240", "serving", "ablation", "gel"],
                    help="video240: the headline stream (default); serving: the many-stream mix, reported "
                         "as arrival-to-completion latency")
    ap.add_argument("--eps", type=float, default=None, help="ablation / gel: eps_des (default 0.1 / 0.01)")
    ap.add_argument("--seconds", type=float, default=10.0, help="serving: length of the arrival trace")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: Poisson arrivals per second")
    ap.add_argument("--streams", type=int, default=256, help="serving: number of streams")
    ap.add_argument("--workers", type=int, default=32, help="serving: worker threads of the server")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, copy one increment device-to-device (a plain copy kernel of known "
                         "size whose FETCH_SIZE / WRITE_SIZE counters calibrate the projection kernel's)")
    return ap.parse_args()


def gen_stream(frames):
    from paper_2211_12487_amd import synth
    w = WORKLOAD
    return np.concatenate(list(synth.video_stream(frames, w["batch"], seed=w["seed"])))


def run_stream(Yd, prec, batch, eps, dims, lat=None, kstats=None):
    from paper_2211_12487_amd.ttice import TTICE
    g = TTICE(dims, eps, prec=prec)
    if kstats is not None:
        g.profile(True)
    info = None
    for k in range(0, Yd.shape[0], batch):
        t0 = time.perf_counter()
        info = g.update(Yd[k:k + batch])
        if lat is not None:
            lat.append(time.perf_counter() - t0)
    ranks = g.ranks()
    if kstats is not None:
        ks = g.kernel_stats()
        for key in ks:
            kstats[key] = kstats.get(key, 0) + ks[key]
    g.close()
    return ranks, info


def time_arm(Yd, prec, steps, warmup):
    import torch
    w = WORKLOAD
    for _ in range(warmup):
        run_stream(Yd, prec, w["batch"], w["eps"], w["dims"])
    lat = []
    kstats = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ranks = None
    for _ in range(steps):
        ranks, _ = run_stream(Yd, prec, w["batch"], w["eps"], w["dims"], lat, kstats)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total = t1 - t0
    return dict(seconds=total, tensors_per_s=Yd.shape[0] * steps / total, ranks=ranks,
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                kstats=kstats)


# level-1 projection kernel of each arm: (name, source file)
PROJ_KERNEL = {
    "fp64": ("k_proj_mfma", "proj.hip"),
    "fp32": ("k_proj_f32", "proj_lp.hip"),
    "bf16x3": ("k_proj_bf3", "proj_lp.hip"),
}


def measured_traffic(prec):
    """HBM bytes per launch of the arm's projection kernel from the committed
    counter summary, or None when that summary is missing or was taken on
    another revision of the kernel's source."""
    import hashlib
    name, src_file = PROJ_KERNEL[prec]
    path = os.path.join(ROOT, "profiles", f"{name}_video240_traffic.txt")
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
    """Level-1 fused projection kernel (U_1^T Y, ||Y(b)||^2 and the residual
    energy in one pass): algorithmic bytes per launch = the increment read
    once + the r_1 coefficient rows written; duration = mean of its HIP-event
    timed launches in the timed region."""
    n = kstats.get("launches", 0)
    if not n:
        return None
    avg_s = kstats["total_ms"] / n * 1e-3
    bytes_per_launch = kstats["bytes"] / n
    achieved = bytes_per_launch / avg_s / 1e9
    return dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=measured_traffic(prec),
                kernel=f"{PROJ_KERNEL[prec][0]} (level-1 projection + residual energy, {prec} products)",
                launches=n, avg_us=avg_s * 1e6, bytes_per_launch=bytes_per_launch)


def cpu_baseline(Y, n_inc):
    """The FP64 NumPy oracle on the first n_inc increments of the same stream."""
    from oracle import TTICE as Oracle
    w = WORKLOAD
    o = Oracle(w["dims"], w["eps"])
    t0 = time.perf_counter()
    for k in range(n_inc):
        o.update(Y[k * w["batch"]:(k + 1) * w["batch"]])
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    return dict(value=n_inc * w["batch"] / dt, unit="tensors/s", cores=cores, kind="oracle",
                sample=f"first {n_inc} increments ({n_inc * w['batch']} frames) of the stream, "
                       f"NumPy FP64 + LAPACK, BLAS threads up to {cores}", seconds=dt)


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
    from paper_2211_12487_amd.ttice import Server
    rng = np.random.default_rng(0)
    srv = Server(workers=a.workers, budget_bytes=200 << 30)
    kinds = [(SERVING_SHAPES[int(rng.integers(len(SERVING_SHAPES)))], SERVING_EPS[int(rng.integers(3))])
             for _ in range(a.streams)]
    sids = [srv.add_stream(dims, eps, max_batch=64) for dims, eps in kinds]
    n_req = int(rng.poisson(a.rate * a.seconds))
    times = np.sort(rng.uniform(0.0, a.seconds, n_req))
    who = rng.integers(0, a.streams, n_req)
    sizes = rng.integers(1, 65, n_req)
    gen = torch.cuda.Stream()
    g = torch.Generator(device="cuda")
    g.manual_seed(0)

    def make(dims, n):
        with torch.cuda.stream(gen):
            parts = []
            for ax, nn in enumerate(dims):
                t = torch.arange(nn, device="cuda", dtype=torch.float32) / max(nn - 1, 1)
                w = torch.rand((n, 5, 1), device="cuda", generator=g) * 3.0
                ph = torch.rand((n, 5, 1), device="cuda", generator=g) * (2 * math.pi)
                parts.append(torch.cos(math.pi * w * t + ph))
            wt = torch.randn((n, 5), device="cuda", generator=g)
            Y = (wt[:, :, None, None, None] * parts[0][:, :, :, None, None] * parts[1][:, :, None, :, None]
                 * parts[2][:, :, None, None, :]).sum(1)
            Y += 1e-3 * torch.randn(Y.shape, device="cuda", generator=g)
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
    srv.close()
    lat_ms = np.array(lat) * 1e3
    steady = lat_ms[np.array(arrivals) >= min(1.0, a.seconds / 2)]  # after the streams' first increments
    return dict(
        metric="serving arrival-to-completion latency p99", value=float(np.percentile(lat_ms, 99)), unit="ms",
        n_gpus=1, steps=1, warmup=0, ms_per_step=wall * 1e3, higher_is_better=False, scaling="weak",
        vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=f"serving: {a.streams} streams of {SERVING_SHAPES}, eps in {SERVING_EPS}, "
                             f"increments of 1..64 tensors, Poisson {a.rate:.0f}/s for {a.seconds:.0f} s, "
                             f"{a.workers} workers"),
        p50_ms=float(np.percentile(lat_ms, 50)), p99_ms=float(np.percentile(lat_ms, 99)),
        max_ms=float(lat_ms.max()), submit_lag_p99_ms=float(np.percentile(np.array(lag) * 1e3, 99)),
        steady_p50_ms=float(np.percentile(steady, 50)), steady_p99_ms=float(np.percentile(steady, 99)),
        increments=len(lat), tensors_per_s=tensors / wall,
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
    w = WORKLOAD
    print(f"generating {a.frames} frames", file=sys.stderr, flush=True)
    Y = gen_stream(a.frames)
    Yd = torch.from_numpy(Y).cuda()
    torch.cuda.synchronize()
    print("timing chosen arm", file=sys.stderr, flush=True)
    chosen = time_arm(Yd, a.prec, a.steps, a.warmup)
    if a.copy_calibration:
        inc = Yd[:w["batch"]]
        dst = torch.empty_like(inc)
        for _ in range(3):
            dst.copy_(inc)
        torch.cuda.synchronize()
        print(f"copy calibration: 3 device copies of {inc.numel() * inc.element_size()} bytes", file=sys.stderr,
              flush=True)
    fp64 = None
    if not a.no_fp64_arm and a.prec != "fp64":
        print("timing fp64 arm", file=sys.stderr, flush=True)
        fp64 = time_arm(Yd, "fp64", a.steps, a.warmup)
        assert fp64["ranks"] == chosen["ranks"], (fp64["ranks"], chosen["ranks"])
    cpu = None
    if not a.no_cpu_baseline:
        print("timing cpu oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(Y, a.cpu_increments)
    ms_per_step = chosen["seconds"] / a.steps * 1e3
    out = dict(
        metric="tensors/s at fixed eps (chosen precision vs plain FP64), % HBM roofline, p99 update latency",
        value=chosen["tensors_per_s"], unit="tensors/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
        ms_per_step=ms_per_step, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype={"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[a.prec], data="synthetic",
        config=dict(workload=f"{w['name']}: {a.frames} frames 240x320x3 fp32, increments of {w['batch']}, "
                             f"eps={w['eps']}, TT-ICE (Algorithm 1) from empty cores",
                    frames=a.frames, batch=w["batch"], eps=w["eps"], prec=a.prec),
        final_ranks=chosen["ranks"], p50_update_ms=chosen["p50_ms"], p99_update_ms=chosen["p99_ms"],
        fp64_arm=(dict(value=fp64["tensors_per_s"], p50_update_ms=fp64["p50_ms"], p99_update_ms=fp64["p99_ms"])
                  if fp64 else None),
        roofline=roofline(chosen["kstats"], a.prec),
        cpu_baseline=cpu,
    )
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
