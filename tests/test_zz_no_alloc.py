"""The allocation-free projection (ttice_project_noalloc) against
ttice_project, through the C ABI: two calls in a row on the same state (the
second with fewer tensors, so the fixed device scratch is reused with a
different layout), coefficients, per-tensor residual energies and norms
within FP64 rounding of the allocating call; a request larger than the
fixed scratch is refused with TTICE_ESCRATCH and leaves the outputs alone."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2211_12487_amd import synth

pytestmark = pytest.mark.gpu

ESCRATCH = -5


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12487_amd import ttice
    ttice.lib()
    yield


def _state(dims, eps, n_inc, batch, seed):
    from paper_2211_12487_amd.ttice import TTICE
    g = TTICE(dims, eps)
    for Y in synth.smooth_separable_stream(n_inc * batch, dims, 5, 1e-3, batch, seed, dtype=np.float32):
        g.update(torch.from_numpy(Y).cuda())
    return g


def _compare(g, Y):
    coef_ref, err2_ref, y2_ref = g.project(Y)
    n = Y.shape[0]
    rd = max(g.ranks()[g.d], 1)
    coef = torch.full((n, rd), float("nan"), dtype=torch.float64, device="cuda")
    err2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    y2 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    g.project_noalloc(Y, coef, err2, y2)
    torch.cuda.synchronize()
    rdk = g.ranks()[g.d]
    scale = float(coef_ref.abs().max())
    assert float((coef[:, :rdk] - coef_ref).abs().max()) <= 1e-12 * scale
    assert torch.allclose(y2, y2_ref, rtol=1e-12, atol=0.0)
    # residual energies: relative to the tensors' energies (they are small
    # differences of large sums)
    assert float((err2 - err2_ref).abs().max()) <= 1e-12 * float(y2_ref.max())


@pytest.mark.parametrize("dims,batch", [((40, 36, 6), 4), ((16, 16, 3), 1)])
def test_noalloc_matches_project_twice(dims, batch):
    print(f"case noalloc {dims}", flush=True)
    g = _state(dims, 0.02, 5, batch, 3)
    big = next(synth.smooth_separable_stream(12, dims, 5, 1e-3, 12, 77, dtype=np.float32))
    small = next(synth.smooth_separable_stream(5, dims, 5, 1e-3, 5, 78, dtype=np.float32))
    _compare(g, torch.from_numpy(big).cuda())
    _compare(g, torch.from_numpy(small).cuda())
    g.close()


def test_noalloc_wide_level_and_fp64_input():
    """A level wide enough for the fused projection (>= 8192 columns) and
    FP64 input, then a smaller call."""
    print("case noalloc wide", flush=True)
    dims = (12, 40, 50)
    g = _state(dims, 0.02, 3, 5, 4)
    a = next(synth.smooth_separable_stream(6, dims, 4, 1e-3, 6, 81))
    b = next(synth.smooth_separable_stream(2, dims, 4, 1e-3, 2, 82))
    _compare(g, torch.from_numpy(a).cuda())
    _compare(g, torch.from_numpy(b).cuda())
    g.close()


def test_noalloc_refuses_requests_beyond_its_scratch():
    from paper_2211_12487_amd.ttice import TTICEError
    print("case noalloc too large", flush=True)
    dims = (64, 64, 64)
    g = _state(dims, 0.05, 1, 2, 5)
    n = 8  # 2 * 8 * 262144 doubles of level buffers alone exceed 32 MiB
    Y = torch.zeros((n,) + dims, dtype=torch.float32, device="cuda")
    coef = torch.full((n, max(g.ranks()[g.d], 1)), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(TTICEError) as ei:
        g.project_noalloc(Y, coef)
    assert ei.value.code == ESCRATCH
    assert bool((coef == 7.0).all())
    g.close()
