"""The serving layer on the GPU (ttice_server_*), through the C ABI: many
streams of the serving mix updated concurrently by several workers.

Checks: 64 streams of the serving mix (every shape, eps and precision),
grouped level-1 launches included, give cores bit-identical to the same
streams served alone (the grouped kernel computes each stream's own blocks,
and every reduction has a fixed order); a batch still being written on a
side stream is read only after that work; two streams against the FP64
oracle (equal ranks, reconstructions within 1e-10); an invalid batch fails
only its own ticket and leaves its stream usable; a reservation above the
budget is refused (queued admission: the emulated cases)."""
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


# the serving mix's shapes, tolerances and precisions
MIX_SHAPES = [(32, 32, 3), (64, 64, 3), (128, 128, 3), (32, 32, 32)]
MIX_PREC = ["fp64", "fp32", "bf16x3"]


def mix_streams(n_streams, incs, seed):
    """n_streams streams of the serving mix: shapes cycling through
    MIX_SHAPES, eps drawn from EPS, precisions cycling through MIX_PREC,
    increments of 1..64 tensors drawn on the device."""
    rng = np.random.default_rng(seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    out = []
    for s in range(n_streams):
        dims = MIX_SHAPES[s % len(MIX_SHAPES)]
        eps = EPS[int(rng.integers(len(EPS)))]
        sizes = [int(x) for x in rng.integers(1, 65, size=incs)]
        out.append(dict(dims=dims, eps=eps, prec=MIX_PREC[s % len(MIX_PREC)],
                        batches=[synth.device_separable(dims, n, g) for n in sizes]))
    torch.cuda.synchronize()
    return out


def cores_of(st, d):
    return [st.core(i) for i in range(d + 1)]


def test_config4_mix_is_bit_identical_to_alone():
    """64 streams of the serving mix, every increment submitted before any
    completes (so workers find many streams waiting and group their level-1
    projections), against each stream served alone: equal ranks and
    bit-identical cores, in every precision."""
    from paper_2211_12487_amd.ttice import Server
    n_streams, incs = 64, 3
    log(f"case server: {n_streams} serving-mix streams x {incs} increments on 8 workers, alone vs mix")
    spec = mix_streams(n_streams, incs, 0)
    srv = Server(workers=8, budget_bytes=64 << 30)
    cap = [max(64, sum(b.shape[0] for b in x["batches"])) for x in spec]
    sids = [srv.add_stream(x["dims"], x["eps"], prec=x["prec"], max_batch=64, max_tensors=cap[s])
            for s, x in enumerate(spec)]
    tickets = []
    for j in range(incs):
        for s, sid in enumerate(sids):
            tickets.append(srv.submit(sid, spec[s]["batches"][j]))
    for t in tickets:
        status, info = srv.wait(t)
        assert status == 0, status
    c = srv.stats()
    log(f"grouped launches {c['groups']}, grouped increments {c['grouped_increments']} of {len(tickets)}")
    assert c["pending"] == 0 and c["waiting_streams"] == 0
    assert c["groups"] > 0 and c["grouped_increments"] > c["groups"], c
    alone = Server(workers=1, budget_bytes=64 << 30)
    for s, sid in enumerate(sids):
        x = spec[s]
        aid = alone.add_stream(x["dims"], x["eps"], prec=x["prec"], max_batch=64, max_tensors=cap[s])
        for Y in x["batches"]:
            status, _ = alone.wait(alone.submit(aid, Y))
            assert status == 0
        mixed, single = srv.stream(sid), alone.stream(aid)
        assert mixed.ranks() == single.ranks(), s
        for i, (a, b) in enumerate(zip(cores_of(mixed, len(x["dims"])), cores_of(single, len(x["dims"])))):
            if not torch.equal(a, b):
                dd = (a - b).abs()
                raise AssertionError(f"stream {s} {x['dims']} {x['prec']} core {i}: {int((dd > 0).sum())} entries "
                                     f"differ, max |diff| {float(dd.max()):.3e} of max |entry| "
                                     f"{float(a.abs().max()):.3e}")
        alone.remove_stream(aid)
    alone.close()
    srv.close()


def test_producer_stream_orders_the_update():
    """A batch written by work still running on a side stream: the update
    reads it only after that work (the submission's producer event, and the
    state's stream for a plain update), so no NaN of the stale contents is
    seen and the results equal those of the synchronised batch."""
    from paper_2211_12487_amd.ttice import TTICE, Server
    log("case server: batch produced on a side stream without a global synchronise")
    dims, eps = (64, 64, 3), 0.05
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    src = [synth.device_separable(dims, 16, g) for _ in range(3)]
    A = torch.randn(4096, 4096, device="cuda", generator=g)
    torch.cuda.synchronize()
    srv = Server(workers=2, budget_bytes=8 << 30)
    sid = srv.add_stream(dims, eps, max_batch=16, max_tensors=64)
    ref = srv.add_stream(dims, eps, max_batch=16, max_tensors=64)
    plain, plain_ref = TTICE(dims, eps), TTICE(dims, eps)
    side = torch.cuda.Stream()
    for Y in src:
        with torch.cuda.stream(side):
            late = torch.full_like(Y, float("nan"))
            B = A
            for _ in range(24):  # keeps the side stream busy for several milliseconds
                B = (B @ A) * (1.0 / 64.0)
            late.copy_(Y + 0.0 * B[0, 0])
            t = srv.submit(sid, late)
            info = plain.update(late)
        assert srv.wait(t)[0] == 0
        assert srv.wait(srv.submit(ref, Y))[0] == 0
        plain_ref.update(Y)
        assert info["ranks"] == plain_ref.ranks()
    side.synchronize()
    a, b = srv.stream(sid), srv.stream(ref)
    assert a.ranks() == b.ranks()
    for i in range(len(dims) + 1):
        assert torch.equal(a.core(i), b.core(i)), i
        assert torch.equal(plain.core(i), plain_ref.core(i)), i
    plain.close()
    plain_ref.close()
    srv.close()


def test_server_streams_match_oracle():
    from paper_2211_12487_amd.ttice import Server
    log("case server: oracle parity of two streams")
    spec = streams(2, 5, 1)
    srv = Server(workers=2, budget_bytes=8 << 30)
    sids = [srv.add_stream(dims, eps, max_batch=8, max_tensors=64) for dims, eps, _ in spec]
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
    a, b = (srv.add_stream(dims, 0.05, max_batch=4, max_tensors=16),
            srv.add_stream(dims, 0.05, max_batch=4, max_tensors=16))
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
    # admission: a reservation above the whole budget is refused
    from paper_2211_12487_amd.ttice import TTICEError
    with pytest.raises(TTICEError):
        srv.add_stream((512, 512, 512), 0.1, max_batch=64, max_tensors=64)
    srv.close()
