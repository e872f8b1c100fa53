"""GPU <-> oracle parity of the reduced-precision projections (FP32 matrix
cores, and split BF16: hi + lo bf16 operands with three products and FP32
accumulation), through the C ABI.

These modes change the level projections C = U^T Z (the one-pass projection
of narrow cores and the large matrix-core products); the norm test's
residual is formed in FP64 from the rounded coefficients (never below the
exact energy), and the residual SVD, re-orthogonalisation and all rank
decisions stay FP64.  Bars: equal TT-ranks wherever the oracle's decision
margins clear the reduced-precision floor, reconstructions within 1e-5
relative (FP32) or 3e-4 (split BF16, see RTOL), achieved error <= eps per
increment, orthonormal cores to 1e-12.  The shapes put more than 8192
columns at level 1 (the fused path) and reach every kernel variant: 4, 2
and 1 columns per lane, FP64 and FP32 input, and level-1 ranks in each
16-wide tile count (<= 16, <= 32, <= 64)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import TTICE as Oracle
from paper_2211_12487_amd import synth

from gpu_helpers import MARGIN_REDUCED, compare_stream, full_reconstruction_error, log, orthogonality

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16x3"]
# Reconstruction bars against the FP64 oracle: 1e-5 for FP32 (operands to
# 2^-24, the reduced path's bar).  Split BF16 keeps 16 significant bits of
# each operand (hi + lo): coefficient j is off by up to 2^-16 ||z|| even for
# data in the cores' span, so the r coefficients of a column by up to
# sqrt(r) 2^-16 ||z||, 1.2e-4 relative at the largest level-1 rank here
# (r = 64): 3e-4 (a factor 2.5 above).
RTOL = {"fp32": 1e-5, "bf16x3": 3e-4}


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12487_amd import ttice
    ttice.lib()
    yield


def make(dims, eps, **kw):
    from paper_2211_12487_amd.ttice import TTICE
    return TTICE(dims, eps, **kw)


def check(dims, eps, batches, prec, label):
    g, o = make(dims, eps, prec=prec), Oracle(dims, eps)
    infos, ok = compare_stream(g, o, batches, RTOL[prec], MARGIN_REDUCED, label=label)
    assert ok, label
    for gi, oi in infos:
        assert gi["achieved2"] <= eps ** 2 * gi["normY2"] * (1 + 1e-6), (label, gi["achieved2"])
    full_reconstruction_error(g, o, RTOL[prec])
    assert orthogonality(g) <= 1e-12
    g.close()


@pytest.mark.parametrize("prec", PRECS)
def test_video_prefix(prec):
    """240x320x3 FP32 frames in increments of 32 (30720 columns, four per
    lane), eps = 0.1: the benchmark's shapes."""
    log(f"case video240 prefix, prec={prec}")
    check((240, 320, 3), 0.1, list(synth.video_stream(128, 32, seed=2)), prec, f"video-{prec}")


@pytest.mark.parametrize("prec", PRECS)
def test_fp64_input_four_columns_per_lane(prec):
    """12 x 40 x 50, FP64 input, batches of 5 (10000 columns)."""
    log(f"case 12x40x50 f64 input, prec={prec}")
    batches = list(synth.smooth_separable_stream(25, (12, 40, 50), 4, 1e-3, 5, 4, dtype=np.float64))
    check((12, 40, 50), 0.02, batches, prec, f"f64in-{prec}")


@pytest.mark.parametrize("prec", PRECS)
def test_two_columns_per_lane(prec):
    """24 x 50 x 41: 2050 columns per frame (two per lane), batches of 5."""
    log(f"case 24x50x41, prec={prec}")
    batches = list(synth.smooth_separable_stream(20, (24, 50, 41), 4, 1e-3, 5, 5, dtype=np.float32))
    check((24, 50, 41), 0.02, batches, prec, f"vec2-{prec}")


@pytest.mark.parametrize("prec", PRECS)
def test_one_column_per_lane(prec):
    """20 x 33 x 31: 1023 columns per frame (odd: one per lane), batches of 9."""
    log(f"case 20x33x31, prec={prec}")
    batches = list(synth.smooth_separable_stream(27, (20, 33, 31), 4, 1e-3, 9, 6, dtype=np.float32))
    check((20, 33, 31), 0.02, batches, prec, f"vec1-{prec}")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("r1", [20, 40])
def test_wide_level_one_core(prec, r1):
    """Exactly low-rank TT stream on 48 x 32 x 32 with r_1 = 20 or 40, so the
    level-1 core spans two or three 16-wide tiles; batches of 8 (8192
    columns), eps = 1e-3."""
    log(f"case lowrank 48x32x32 r1={r1}, prec={prec}")
    dims = (48, 32, 32)
    ys = list(synth.tt_lowrank_stream(dims, (r1, 24, 16), 32, 8, seed=8))
    batches = [y.astype(np.float32) for y in ys]
    check(dims, 1e-3, batches, prec, f"rt-{r1}-{prec}")
