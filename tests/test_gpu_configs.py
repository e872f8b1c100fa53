"""GPU <-> oracle parity on the higher-order workloads, through the C ABI.

* Order 4, simulation-shaped snapshots (random Fourier fields, |k|^-2,
  three components, eps = 0.01, increments of 16): a reduced 16^3 x 3 grid
  over several increments, and the full 64^3 x 3 grid on its first increment.
* Order 8, a scalar 64^3 field reshaped to 8 x 8 x 4^6 and the full 256^3
  field reshaped to 8^8 (|k|^-3, eps = 0.005, increments of 8, Algorithm 2
  with the mean skip rule).

Bars: equal TT-ranks where the oracle's decision margins clear the FP64
floor, reconstructions within 1e-10 relative, orthonormal cores to 1e-12,
and the error of each increment equal to its discarded energy (P1) and
within eps (Algorithm 1, and Algorithm 2's first increment, where every frame
is updated)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import TTICE as Oracle
from paper_2211_12487_amd import synth

from gpu_helpers import MARGIN_FP64, compare_stream, full_reconstruction_error, log, orthogonality

pytestmark = pytest.mark.gpu


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


def discarded_energy_is_the_error(g, Y, info, eps, label):
    """P1 on the device: ||Y - Yhat||^2 of the newest increment equals the
    reported discarded energy, and is within eps^2 ||Y||^2."""
    n = Y.shape[0]
    rec = g.reconstruct(g.n_total - n, n)
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).to(torch.float64).cuda()
    err2 = float(((Yd - rec) ** 2).sum())
    if info["achieved2"] is not None:  # Algorithm 1 reports the discarded energy
        assert err2 == pytest.approx(info["achieved2"], rel=1e-6, abs=1e-12 * info["normY2"]), label
    assert err2 <= eps ** 2 * info["normY2"] * (1 + 1e-9), label


def test_order4_reduced_grid_stream():
    log("case order-4 field 16^3 x 3, 4 increments of 16")
    dims, eps = (16, 16, 16, 3), 0.01
    batches = list(synth.fourier_field_stream(64, 16, grid=16, components=3, seed=1))
    g, o = make(dims, eps), Oracle(dims, eps)
    infos, ok = compare_stream(g, o, batches, 1e-10, MARGIN_FP64, label="field16")
    assert ok
    for (gi, _), Y in zip(infos, batches):
        assert gi["achieved2"] <= eps ** 2 * gi["normY2"] * (1 + 1e-9)
    full_reconstruction_error(g, o, 1e-10)
    assert orthogonality(g) <= 1e-12


def test_order4_full_grid_first_increment():
    log("case order-4 field 64^3 x 3, first increment of 16 (oracle at full size)")
    dims, eps = (64, 64, 64, 3), 0.01
    Y = next(synth.fourier_field_stream(16, 16, grid=64, components=3, seed=3))
    g, o = make(dims, eps), Oracle(dims, eps)
    infos, ok = compare_stream(g, o, [Y], 1e-10, MARGIN_FP64, label="field64")
    assert ok
    discarded_energy_is_the_error(g, Y, infos[0][0], eps, "field64")
    assert orthogonality(g) <= 1e-12


def test_order8_reduced_star_stream():
    log("case order-8 field 64^3 as 8x8x4^6, Algorithm 2, 3 increments of 8")
    dims, eps = (8, 8, 4, 4, 4, 4, 4, 4), 0.005
    raw = synth.fourier_field_stream(24, 8, grid=64, components=1, kmax=16, decay=3.0, seed=4)
    batches = [b.reshape((b.shape[0],) + dims) for b in raw]
    g, o = make(dims, eps, algo="star"), Oracle(dims, eps, algo="star")
    infos, ok = compare_stream(g, o, batches, 1e-10, MARGIN_FP64, label="order8-small")
    assert ok
    for gi, oi in infos:
        assert gi["skipped"] == oi["skipped"] and gi["used"] == oi["used"]
    full_reconstruction_error(g, o, 1e-10)
    assert orthogonality(g) <= 1e-12


def test_order8_full_field_first_increment():
    log("case order-8 field 256^3 as 8^8, Algorithm 2, first increment of 8 (oracle at full size)")
    dims, eps = (8,) * 8, 0.005
    raw = next(synth.fourier_field_stream(8, 8, grid=256, components=1, kmax=16, decay=3.0, seed=5))
    Y = raw.reshape((8,) + dims)
    g, o = make(dims, eps, algo="star"), Oracle(dims, eps, algo="star")
    infos, ok = compare_stream(g, o, [Y], 1e-10, MARGIN_FP64, label="order8-full")
    assert ok
    gi = infos[0][0]
    assert not gi["skipped"] and gi["used"] == 8  # empty cores: every frame is updated (P8)
    discarded_energy_is_the_error(g, Y, gi, eps, "order8-full")
    assert orthogonality(g) <= 1e-12
