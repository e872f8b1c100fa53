"""Checkpoint / resume on the GPU, through the C ABI (ttice_save /
ttice_load): a stream saved part-way, loaded into a new state and continued
equals the stream run without interruption, bit for bit (ranks, every core,
the last core), in every precision mode and for Algorithm 2; the resumed
stream also matches the FP64 oracle (equal ranks, reconstructions within
1e-10); a corrupted image is refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import TTICE as Oracle
from paper_2211_12487_amd import synth

from gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12487_amd import ttice
    ttice.lib()
    yield


def stream(dims, n, batch, seed):
    return [torch.from_numpy(y).cuda()
            for y in synth.smooth_separable_stream(n, dims, 4, 1e-3, batch, seed, dtype=np.float32)]


@pytest.mark.parametrize("prec,algo", [("fp64", "plain"), ("fp32", "plain"), ("bf16x3", "plain"), ("fp64", "star")])
def test_resume_equals_uninterrupted(prec, algo):
    from paper_2211_12487_amd.ttice import TTICE
    dims, eps = (32, 24, 3), 0.02
    log(f"case checkpoint {prec} {algo} {dims}")
    batches = stream(dims, 48, 6, 11)
    full = TTICE(dims, eps, prec=prec, algo=algo)
    for Y in batches:
        full.update(Y)
    for cut in (0, 3, 6):
        a = TTICE(dims, eps, prec=prec, algo=algo)
        for Y in batches[:cut]:
            a.update(Y)
        img = a.save()
        a.close()
        b = TTICE.load(img)
        assert b.dims == dims and b.eps == eps
        for Y in batches[cut:]:
            b.update(Y)
        assert b.ranks() == full.ranks(), (cut, b.ranks(), full.ranks())
        for i in range(len(dims) + 1):
            assert torch.equal(b.core(i), full.core(i)), (cut, i)
        assert b.save() == full.save()
        b.close()
    full.close()


def test_resumed_stream_matches_oracle():
    from paper_2211_12487_amd.ttice import TTICE
    dims, eps = (40, 30, 3), 0.01
    log("case checkpoint vs oracle")
    batches = stream(dims, 40, 5, 12)
    o = Oracle(dims, eps)
    a = TTICE(dims, eps)
    for Y in batches[:4]:
        a.update(Y)
        o.update(Y.cpu().numpy().astype(np.float64))
    b = TTICE.load(a.save())
    a.close()
    for Y in batches[4:]:
        gi = b.update(Y)
        oi = o.update(Y.cpu().numpy().astype(np.float64))
        assert gi["ranks"] == oi["ranks"]
    g = b.reconstruct().cpu().numpy()
    r = o.reconstruct()
    rel = max(np.linalg.norm(g[k] - r[k]) / np.linalg.norm(r[k]) for k in range(r.shape[0]))
    assert rel <= 1e-10, rel
    b.close()


def test_corrupted_image_is_refused():
    from paper_2211_12487_amd.ttice import TTICE, TTICEError
    dims = (16, 16, 3)
    log("case checkpoint corrupted image")
    a = TTICE(dims, 0.05)
    for Y in stream(dims, 8, 4, 13):
        a.update(Y)
    img = bytearray(a.save())
    img[len(img) // 3] ^= 0x10
    with pytest.raises(TTICEError):
        TTICE.load(bytes(img))
    with pytest.raises(TTICEError):
        TTICE.load(a.save()[:-3])
    a.close()
