"""The serving layer on the GPU (ttice_server_*), through the C ABI: many
streams of the serving mix updated concurrently by several workers.

Checks: every stream's cores and reconstructions are bit-identical to the
same stream run alone (fixed-order reductions make a stream's result
independent of the mix); two streams against the FP64 oracle (equal ranks,
reconstructions within 1e-10); an invalid batch fails only its own ticket
and leaves its stream usable; admission refuses a stream beyond the budget."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import TTICE as Oracle
from paper_2211_12487_amd import synth

from gpu_helpers import log

pytestmark = pytest.mark.gpu

SHAPES = [(32, 32, 3), (64, 64, 3), (32, 32, 32), (48, 40, 3)]
EPS = [0.01, 0.05, 0.1]


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_12487_amd import ttice
    ttice.lib()
    yield


def streams(n_streams, incs, seed):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_streams):
        dims = SHAPES[s % len(SHAPES)]
        eps = EPS[int(rng.integers(len(EPS)))]
        sizes = [int(x) for x in rng.integers(1, 9, size=incs)]
        ys = list(synth.smooth_separable_stream(sum(sizes), dims, 4, 1e-3, 1, 100 + s, dtype=np.float32))
        batches, k = [], 0
        for n in sizes:
            batches.append(np.concatenate(ys[k:k + n]))
            k += n
        out.append((dims, eps, batches))
    return out


def test_mix_is_bit_identical_to_alone():
    from paper_2211_12487_amd.ttice import TTICE, Server
    log("case server: 12 streams x 6 increments on 4 workers, alone vs mix")
    spec = streams(12, 6, 0)
    srv = Server(workers=4, budget_bytes=32 << 30)
    sids = [srv.add_stream(dims, eps, max_batch=8) for dims, eps, _ in spec]
    dev = [[torch.from_numpy(b).cuda() for b in batches] for _, _, batches in spec]
    torch.cuda.synchronize()
    tickets = []
    for j in range(6):
        for s, sid in enumerate(sids):
            tickets.append(srv.submit(sid, dev[s][j]))
    for t in tickets:
        status, info = srv.wait(t)
        assert status == 0, status
    assert srv.stats()["pending"] == 0
    for s, sid in enumerate(sids):
        dims, eps, _ = spec[s]
        mixed = srv.stream(sid)
        alone = TTICE(dims, eps)
        for Y in dev[s]:
            alone.update(Y)
        assert mixed.ranks() == alone.ranks(), s
        assert torch.equal(mixed.reconstruct(), alone.reconstruct()), s
        for i in range(len(dims) + 1):
            assert torch.equal(mixed.core(i), alone.core(i)), (s, i)
        alone.close()
    srv.close()


def test_server_streams_match_oracle():
    from paper_2211_12487_amd.ttice import Server
    log("case server: oracle parity of two streams")
    spec = streams(2, 5, 1)
    srv = Server(workers=2, budget_bytes=8 << 30)
    sids = [srv.add_stream(dims, eps, max_batch=8) for dims, eps, _ in spec]
    oracles = [Oracle(dims, eps) for dims, eps, _ in spec]
    for j in range(5):
        ts = [srv.submit(sid, torch.from_numpy(spec[s][2][j]).cuda()) for s, sid in enumerate(sids)]
        for s, t in enumerate(ts):
            status, info = srv.wait(t)
            assert status == 0
            oi = oracles[s].update(spec[s][2][j].astype(np.float64))
            assert info["ranks"] == oi["ranks"], (s, j)
    for s, sid in enumerate(sids):
        g = srv.stream(sid).reconstruct().cpu().numpy()
        o = oracles[s].reconstruct()
        rel = max(np.linalg.norm(g[b] - o[b]) / np.linalg.norm(o[b]) for b in range(o.shape[0]))
        assert rel <= 1e-10, (s, rel)
    srv.close()


def test_bad_batch_fails_only_its_ticket():
    from paper_2211_12487_amd.ttice import Server
    log("case server: invalid batch")
    dims = (16, 16, 3)
    srv = Server(workers=2, budget_bytes=1 << 30)
    a, b = srv.add_stream(dims, 0.05, max_batch=4), srv.add_stream(dims, 0.05, max_batch=4)
    good = [torch.from_numpy(y).cuda() for y in synth.smooth_separable_stream(6, dims, 4, 1e-3, 2, 5)]
    bad = torch.full((2,) + dims, float("nan"), dtype=torch.float64, device="cuda")
    t0 = srv.submit(a, good[0])
    t1 = srv.submit(a, bad)
    t2 = srv.submit(b, good[1])
    t3 = srv.submit(a, good[2])
    assert srv.wait(t0)[0] == 0
    assert srv.wait(t1)[0] == -1
    assert srv.wait(t2)[0] == 0
    assert srv.wait(t3)[0] == 0
    assert srv.stream(a).n_total == 4
    # admission: a stream beyond the remaining budget is refused
    from paper_2211_12487_amd.ttice import TTICEError
    with pytest.raises(TTICEError):
        srv.add_stream((512, 512, 512), 0.1, max_batch=64)
    srv.close()
