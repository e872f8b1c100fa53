"""Shared helpers of the GPU parity tests: run the HIP library and the CPU
oracle on the same seeded stream and compare them increment by increment."""
import math
import sys

import numpy as np
import torch

from oracle import TTICE as Oracle


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# The benchmark spec's bars: exact ranks on increments whose rank decisions are
# well separated from the threshold, reconstructions within 1e-10 relative on
# the FP64 path (1e-5 reduced precision), achieved error <= eps, orthonormal
# cores to 1e-12.
MARGIN_FP64 = 1e-8
MARGIN_REDUCED = 1e-3


def to_dev(Y, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(Y))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def compare_stream(gpu, ora, batches, rtol, margin_floor, check_every=1, label=""):
    """Feed every batch to both; assert equal ranks (when the oracle's
    decision margins clear margin_floor), equal reconstructions of the newest
    increment, and return the list of (gpu_info, oracle_info)."""
    infos = []
    for k, Y in enumerate(batches):
        gi = gpu.update(to_dev(Y))
        oi = ora.update(Y.astype(np.float64))
        infos.append((gi, oi))
        margins = [m for m in oi["margin"] if m == m]
        decisive = all(m > margin_floor for m in margins) if margins else True
        if decisive:
            assert gi["ranks"][1:-1] == oi["ranks"][1:-1], (label, k, gi["ranks"], oi["ranks"], oi["margin"])
        else:
            log(f"{label} increment {k}: oracle margin {min(margins):.2e} below {margin_floor}, ranks not compared")
            if gi["ranks"][1:-1] != oi["ranks"][1:-1]:
                return infos, False
        if k % check_every == 0:
            n = Y.shape[0]
            first = gpu.n_total - n
            g = gpu.reconstruct(first, n).cpu().numpy()
            o = ora.reconstruct(first, n)
            for b in range(n):
                den = max(np.linalg.norm(o[b]), 1e-300)
                rel = np.linalg.norm(g[b] - o[b]) / den
                assert rel <= rtol, (label, k, b, rel)
    return infos, True


def full_reconstruction_error(gpu, ora, rtol):
    g = gpu.reconstruct().cpu().numpy()
    o = ora.reconstruct()
    worst = 0.0
    for b in range(o.shape[0]):
        den = max(np.linalg.norm(o[b]), 1e-300)
        worst = max(worst, np.linalg.norm(g[b] - o[b]) / den)
    assert worst <= rtol, worst
    return worst


def orthogonality(gpu):
    worst = 0.0
    for i in range(gpu.d):
        U = gpu.core(i)
        if U.shape[1]:
            E = U.T @ U - torch.eye(U.shape[1], dtype=U.dtype, device=U.device)
            worst = max(worst, float(E.abs().max()))
    return worst
