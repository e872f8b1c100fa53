"""Parity cases run against the host-emulation build (tests only).

Invoked by tests/test_emu.py in a subprocess that preloads the
AddressSanitizer runtime: argv[1] = path of libttice_emu.so, argv[2:] =
case names (default: all).  Exits non-zero on the first failure."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

from emu_ttice import EmuError, EmuTTICE, ServerCounters, UpdateInfo, load  # noqa: E402
from oracle import TTICE as Oracle  # noqa: E402
from paper_2211_12487_amd import synth  # noqa: E402

L = None


def sep(n, dims, batch, seed, terms=4, noise=1e-3, dtype=np.float64):
    return list(synth.smooth_separable_stream(n, dims, terms, noise, batch, seed, dtype=dtype))


def check_stream(g, o, batches, rtol=1e-10, label=""):
    for k, Y in enumerate(batches):
        gi = g.update(Y)
        oi = o.update(Y.astype(np.float64))
        assert gi["ranks"][1:-1] == oi["ranks"][1:-1], (label, k, gi["ranks"], oi["ranks"], oi["margin"])
        if oi.get("achieved2") is not None and gi["achieved2"] is not None:
            assert abs(gi["achieved2"] - oi["achieved2"]) <= 1e-6 * oi["achieved2"] + 1e-20, (label, k)
    rg, ro = g.reconstruct(), o.reconstruct()
    for b in range(ro.shape[0]):
        rel = np.linalg.norm(rg[b] - ro[b]) / max(np.linalg.norm(ro[b]), 1e-300)
        assert rel <= rtol, (label, b, rel)
    for i in range(g.d):
        U = g.core(i)
        if U.shape[1]:
            assert np.abs(U.T @ U - np.eye(U.shape[1])).max() <= 1e-12, (label, i)


def case_separable():
    dims, eps = (16, 16, 3), 0.05
    check_stream(EmuTTICE(L, dims, eps), Oracle(dims, eps), sep(12, dims, 2, 0, terms=5), label="sep")


def case_ragged_f32():
    dims, eps = (37, 29, 5), 0.02
    rng = np.random.default_rng(3)
    sizes = [int(x) for x in rng.integers(1, 6, 5)]
    flat = sep(sum(sizes), dims, 1, 4, terms=6, dtype=np.float32)
    batches, k = [], 0
    for s in sizes:
        batches.append(np.concatenate(flat[k:k + s]))
        k += s
    check_stream(EmuTTICE(L, dims, eps), Oracle(dims, eps), batches, rtol=1e-9, label="ragged")


def case_wide_level():
    """Level 1 wide enough (>= 8192 columns) for the fused one-pass projection."""
    dims, eps = (12, 40, 50), 0.05
    check_stream(EmuTTICE(L, dims, eps), Oracle(dims, eps), sep(15, dims, 5, 21, terms=4), label="wide")


def case_order4():
    dims, eps = (9, 7, 11, 3), 0.03
    check_stream(EmuTTICE(L, dims, eps), Oracle(dims, eps), sep(12, dims, 4, 5, terms=5), label="order4")


def case_order1_order2():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((70, 5))
    batches = [(A @ rng.standard_normal((5, b))).T + 1e-3 * rng.standard_normal((b, 70)) for b in (50, 3, 9)]
    check_stream(EmuTTICE(L, (70,), 0.05), Oracle((70,), 0.05), batches, label="order1")
    check_stream(EmuTTICE(L, (40, 90), 0.05), Oracle((40, 90), 0.05), sep(12, (40, 90), 6, 7), label="order2")


def case_lanczos():
    """The block-Lanczos truncated SVD (forced for every Gram matrix wider
    than its 128-vector Krylov basis): a left Gram matrix 150 wide and a
    right one 180 wide; ranks and reconstructions as the oracle and as the
    dense solver of the same library, and the solver reported per core."""
    for dims, batch, n in (((150, 12, 14), 1, 3), ((300, 10, 3), 6, 18)):
        batches = sep(n, dims, batch, 31, terms=4)
        g, o = EmuTTICE(L, dims, 0.02, svd=2), Oracle(dims, 0.02)
        dense = EmuTTICE(L, dims, 0.02, svd=0)
        used = 0
        for Y in batches:
            gi = g.update(Y)
            di = dense.update(Y)
            oi = o.update(Y)
            used += sum(1 for s in gi["solver"] if s == 2)
            assert all(s != 2 for s in di["solver"])
            assert gi["ranks"] == di["ranks"] == oi["ranks"], (dims, gi["ranks"], di["ranks"], oi["ranks"])
        assert used > 0, dims
        rg, rd, ro = g.reconstruct(), dense.reconstruct(), o.reconstruct()
        assert np.abs(rg - rd).max() <= 1e-10 * np.abs(rd).max(), dims
        for b in range(ro.shape[0]):
            assert np.linalg.norm(rg[b] - ro[b]) <= 1e-10 * np.linalg.norm(ro[b]), (dims, b)
        for i in range(g.d):
            U = g.core(i)
            if U.shape[1]:
                assert np.abs(U.T @ U - np.eye(U.shape[1])).max() <= 1e-12, (dims, i)


def case_star():
    dims, eps = (12, 10, 6), 0.05
    g, o = EmuTTICE(L, dims, eps, algo=1), Oracle(dims, eps, algo="star")
    skipped = 0
    rng = np.random.default_rng(8)
    batches = [Y + 1e-3 * rng.standard_normal(Y.shape)
               for Y in synth.tt_lowrank_stream(dims, (3, 4, 4), 40, 4, seed=8)]
    for k, Y in enumerate(batches):
        gi, oi = g.update(Y), o.update(Y)
        assert gi["skipped"] == oi["skipped"] and gi["used"] == oi["used"], k
        assert gi["ranks"][1:-1] == oi["ranks"][1:-1], (k, gi["ranks"], oi["ranks"])
        skipped += gi["skipped"]
    assert skipped > 0
    rg, ro = g.reconstruct(), o.reconstruct()
    assert np.abs(rg - ro).max() <= 1e-10 * np.abs(ro).max()


def case_project():
    dims, eps = (12, 10, 6), 0.05
    g, o = EmuTTICE(L, dims, eps), Oracle(dims, eps)
    for Y in sep(8, dims, 2, 9):
        g.update(Y)
        o.update(Y)
    Yn = sep(5, dims, 5, 99)[0]
    coef, err2, y2 = g.project(Yn)
    oc, ot = o.project(Yn)
    assert np.abs(coef - oc).max() <= 1e-10 * np.abs(oc).max()
    brute = np.array([np.sum((Yn[b] - ot[b]) ** 2) for b in range(5)])
    assert np.allclose(err2, brute, rtol=1e-8)


def case_errors_and_degenerate():
    dims, eps = (4, 3, 5), 0.1
    g = EmuTTICE(L, dims, eps)
    g.update(np.zeros((0,) + dims))
    g.update(np.zeros((2,) + dims))
    r, n = g.ranks()
    assert r == [1, 0, 0, 0, 1] and n == 2
    assert np.all(g.reconstruct() == 0)
    Y = sep(3, dims, 3, 10)[0]
    g.update(Y)
    r0, n0 = g.ranks()
    rec0 = g.reconstruct()
    bad = Y.copy()
    bad[1, 2, 1, 3] = np.nan
    try:
        g.update(bad)
        raise AssertionError("NaN accepted")
    except EmuError as e:
        assert e.code == -1
    assert g.ranks() == (r0, n0) and np.array_equal(g.reconstruct(), rec0)


def case_alloc_failure_leaves_state():
    """Failure injection: the k-th device allocation fails -> ENOMEM and the
    state (ranks, stored tensors, reconstructions) is unchanged."""
    dims, eps = (12, 10, 6), 0.02
    data = sep(9, dims, 3, 11, terms=6) + sep(9, dims, 9, 12, terms=6)   # last increment is larger
    ref = EmuTTICE(L, dims, eps)
    for Y in data:
        ref.update(Y)
    hits = 0
    for k in range(0, 12):
        g = EmuTTICE(L, dims, eps)
        for Y in data[:-1]:
            g.update(Y)
        r0, n0 = g.ranks()
        rec0 = g.reconstruct()
        L.hipemu_fail_alloc_after(k)
        try:
            g.update(data[-1])
            ok = True
        except EmuError as e:
            assert e.code == -2, e.code
            ok = False
        finally:
            L.hipemu_fail_alloc_after(-1)
        if not ok:
            hits += 1
            assert g.ranks() == (r0, n0)
            assert np.array_equal(g.reconstruct(), rec0)
            g.update(data[-1])  # and it recovers
        assert g.ranks() == ref.ranks()
        assert np.allclose(g.reconstruct(), ref.reconstruct(), atol=1e-12)
        g.close()
    assert hits > 0


def case_lowrank():
    """Exactly low-rank stream at the paper's eps = 1e-8 (App. B): the Gram
    matrix cannot resolve that cut, so the rank comes from the explicit
    residual energies; the ranks are the stream's TT-ranks."""
    dims = (10, 15, 20)
    g = EmuTTICE(L, dims, 1e-8)
    o = Oracle(dims, 1e-8)
    for k, Y in enumerate(synth.tt_lowrank_stream(dims, (2, 3, 5), 7, 1, seed=7), start=1):
        gi = g.update(Y)
        oi = o.update(Y)
        assert g.ranks()[0][1:-1] == [2, 3, min(k, 5)] == oi["ranks"][1:-1], (k, g.ranks(), oi["ranks"])
    rg, ro = g.reconstruct(), o.reconstruct()
    assert np.abs(rg - ro).max() <= 1e-10 * np.abs(ro).max()


def case_graded_spectrum():
    """Singular values falling 30x per term over 12 terms at eps = 1e-9: the
    kept directions reach below what the first Gram matrix resolves, so the
    level runs again on the deflated residual.  Ranks as the oracle's; each
    increment within eps (eq:ttsvd_error) and within 2x the oracle's
    error; reconstructions within eps/2 of the oracle's (directions near the
    first Gram matrix's resolution differ from the exact SVD's by angles of
    order u sigma_1^2 / (sigma_j^2 - sigma_{j+1}^2))."""
    dims, eps = (12, 10, 8), 1e-9
    batches = list(synth.graded_stream(dims, 12, 1.0 / 30.0, 3, 2, seed=41))
    g, o = EmuTTICE(L, dims, eps), Oracle(dims, eps)
    for k, Y in enumerate(batches):
        gi = g.update(Y)
        oi = o.update(Y)
        assert gi["ranks"] == oi["ranks"], (k, gi["ranks"], oi["ranks"], oi["margin"])
    assert max(g.ranks()[0][1:-1]) >= 7, g.ranks()
    rg, ro = g.reconstruct(), o.reconstruct()
    Yall = np.concatenate(batches)
    for k in range(len(batches)):
        s = slice(2 * k, 2 * k + 2)
        eg = np.linalg.norm(rg[s] - Yall[s]) / np.linalg.norm(Yall[s])
        eo = np.linalg.norm(ro[s] - Yall[s]) / np.linalg.norm(Yall[s])
        assert eg <= eps and eg <= 2.0 * eo + 1e-15, (k, eg, eo)
    for b in range(ro.shape[0]):
        assert np.linalg.norm(rg[b] - ro[b]) <= 0.5 * eps * np.linalg.norm(ro[b]), b
    for i in range(g.d):
        U = g.core(i)
        if U.shape[1]:
            assert np.abs(U.T @ U - np.eye(U.shape[1])).max() <= 1e-12, i


def case_checkpoint():
    """Checkpoint / resume: a stream saved after some increments, loaded into
    a new state and continued gives the same ranks, cores and last core, bit
    for bit, as the stream run without interruption (Algorithm 1 and 2, non-
    default options); the image carries the options; corrupted, truncated,
    resized or impossible images are refused with EINVAL."""
    import ctypes
    from emu_ttice import EmuError
    for algo, dims, eps in ((0, (12, 10, 6), 0.05), (1, (9, 7, 11, 3), 0.03)):
        batches = list(synth.smooth_separable_stream(14, dims, 3, 1e-3, 2, 40 + algo, dtype=np.float32))
        full = EmuTTICE(L, dims, eps, algo=algo, prec=0, tau=0.8 if algo else None, skip_rule=1 if algo else None)
        for Y in batches:
            full.update(Y)
        for cut in (0, 1, 4):
            a = EmuTTICE(L, dims, eps, algo=algo, prec=0, tau=0.8 if algo else None,
                         skip_rule=1 if algo else None)
            for Y in batches[:cut]:
                a.update(Y)
            img = a.save()
            assert img == a.save()  # saving does not change the state
            b = EmuTTICE.load(L, img)
            assert b.dims == tuple(dims) and b.eps == eps
            assert b.ranks() == a.ranks()
            a.close()
            for Y in batches[cut:]:
                b.update(Y)
            assert b.ranks() == full.ranks(), (algo, cut)
            for i in range(len(dims) + 1):
                assert np.array_equal(b.core(i), full.core(i)), (algo, cut, i)
            assert b.save() == full.save()
            b.close()
        img = full.save()
        bad = bytearray(img)
        bad[len(img) // 2] ^= 1
        for broken in (bytes(bad), img[:-1], img + b"\0", b"XXXXXXXX" + img[8:], b""):
            h = ctypes.c_void_p()
            assert L.ttice_load(broken, len(broken), ctypes.byref(h)) == -1 and not h.value
        # a rank larger than r_{i-1} n_i, with a matching hash, is still refused
        d = len(dims)
        off = 48 + 8 * d + 8
        forged = bytearray(img[:-8])
        forged[off:off + 8] = (dims[0] + 1).to_bytes(8, "little", signed=True)
        h = 1469598103934665603
        for byte in forged:
            h = ((h ^ byte) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
        forged = bytes(forged) + h.to_bytes(8, "little")
        hh = ctypes.c_void_p()
        assert L.ttice_load(forged, len(forged), ctypes.byref(hh)) == -1
        n = ctypes.c_int64()
        small = ctypes.create_string_buffer(16)
        assert L.ttice_save(full.h, small, 16, ctypes.byref(n)) == -1 and n.value == len(img)
        full.close()


def case_eigensolver():
    """The library's eigensolver kernels (tridiagonalisation, bisection,
    inverse iteration) against LAPACK on random, clustered and
    rank-deficient PSD matrices, on both the LDS and the global-memory path."""
    import ctypes
    L.hipemu_sym_eig.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    rng = np.random.default_rng(0)

    def run(G, r):
        m = G.shape[0]
        G = np.ascontiguousarray(G)
        w = np.zeros(m)
        X = np.zeros((m, max(r, 1)))
        assert L.hipemu_sym_eig(m, G.ctypes.data, w.ctypes.data, r, X.ctypes.data) == 0
        return w, X[:, :r]

    for m in (1, 2, 3, 5, 16, 32, 33, 40, 64, 65, 96, 124, 125, 128, 129, 131, 230):
        B = rng.standard_normal((m, m + 3))
        G = B @ B.T
        w, X = run(G, min(m, 5))
        ev, EV = np.linalg.eigh(G)
        ev, EV = ev[::-1], EV[:, ::-1]
        assert np.abs(w - ev).max() <= 1e-13 * ev[0], m
        for c in range(X.shape[1]):
            assert min(np.linalg.norm(X[:, c] - EV[:, c]), np.linalg.norm(X[:, c] + EV[:, c])) <= 1e-10, (m, c)
    # many kept vectors (the back-transformation with several columns per
    # wave): separated spectrum, every vector against LAPACK's
    for m, r in ((40, 12), (96, 40), (128, 70), (200, 40), (300, 40), (331, 3)):
        Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
        lam = np.linspace(10.0, 1.0, m)
        G = (Q * lam) @ Q.T
        w, X = run(G, r)
        assert np.abs(w - lam).max() <= 1e-13 * 10.0, m
        for c in range(r):
            q = Q[:, c]
            assert min(np.linalg.norm(X[:, c] - q), np.linalg.norm(X[:, c] + q)) <= 1e-10, (m, r, c)
        assert np.abs(X.T @ X - np.eye(r)).max() <= 1e-12, (m, r)
    # clustered spectrum: compare the kept subspace through its projector
    for m in (12, 140):
        Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
        lam = np.concatenate([[9.0, 5.0, 5.0, 5.0 + 1e-9, 2.0], np.linspace(1.0, 0.1, m - 5)])
        G = (Q * lam) @ Q.T
        w, X = run(G, 4)
        assert np.abs(w - np.sort(lam)[::-1]).max() <= 1e-13 * 9.0
        P = X @ X.T
        Pref = Q[:, :4] @ Q[:, :4].T
        assert np.abs(P - Pref).max() <= 1e-9, m
        assert np.abs(X.T @ X - np.eye(4)).max() <= 1e-12
    # a non-finite matrix gives NaN eigenvalues (which the rank selection
    # reports as a device error), never a finite spectrum
    for m in (12, 96, 140):
        G = np.eye(m)
        G[3, 5] = G[5, 3] = np.nan
        w, _ = run(G, 0)
        assert np.isnan(w).all(), (m, w[:4])
    # one large cluster inside the kept set (a Gram matrix's small eigenvalues
    # within 1e-3 ||T|| of each other): the kept subspace against LAPACK's
    for m, r in ((120, 41), (300, 41)):
        Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
        lam = np.concatenate([[1.0], np.linspace(1.1e-4, 1e-4, 40), np.linspace(1e-8, 1e-9, m - 41)])
        G = (Q * lam) @ Q.T
        w, X = run(G, r)
        assert np.abs(w - lam).max() <= 1e-13, m
        P = X @ X.T
        Pref = Q[:, :r] @ Q[:, :r].T
        assert np.abs(P - Pref).max() <= 1e-9, (m, np.abs(P - Pref).max())
        assert np.abs(X.T @ X - np.eye(r)).max() <= 1e-12, (m, np.abs(X.T @ X - np.eye(r)).max())
    # rank deficient
    B = rng.standard_normal((30, 2))
    w, X = run(B @ B.T, 2)
    ev = np.linalg.eigvalsh(B @ B.T)[::-1]
    assert np.abs(w - ev).max() <= 1e-13 * ev[0]


def case_gemm_mx():
    """The matrix-core tiled product (FP64) on its own, against NumPy:
    ragged sizes off the 128 x 64 tile and the 32-deep K tile, A given
    row-major or transposed, framed B columns, beta E, and the column
    energies per 64-row block."""
    import ctypes
    vp, c_int, c_dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.hipemu_gemm_mx.argtypes = [c_int, c_int, c_int, c_dbl, vp, c_int, vp, c_int, ctypes.c_long, c_dbl, vp, vp, vp]
    rng = np.random.default_rng(12)
    for M, N, K, nf, a_trans, beta in ((130, 70, 45, 1, 0, 0.0), (200, 96, 33, 3, 1, -1.0), (64, 64, 32, 2, 0, 0.5),
                                       (7, 5, 3, 1, 1, 1.0)):
        A = rng.standard_normal((M, K))
        cpf = N // nf
        fs = K * cpf + 7
        Bf = rng.standard_normal(nf * fs)
        B = np.concatenate([Bf[f * fs:f * fs + K * cpf].reshape(K, cpf) for f in range(nf)], axis=1)
        E = rng.standard_normal((M, N))
        D = np.zeros((M, N))
        MB = (M + 63) // 64
        cp = np.zeros((MB, N))
        Ain = np.ascontiguousarray(A.T) if a_trans else A
        assert L.hipemu_gemm_mx(M, N, K, 0.75, Ain.ctypes.data, a_trans, Bf.ctypes.data, nf, fs, beta,
                                E.ctypes.data, D.ctypes.data, cp.ctypes.data) == 0
        ref = 0.75 * A @ B + beta * E
        assert np.abs(D - ref).max() <= 1e-12 * np.abs(ref).max(), (M, N, K)
        cref = np.array([(ref[64 * b:64 * (b + 1)] ** 2).sum(0) for b in range(MB)])
        assert np.abs(cp - cref).max() <= 1e-12 * np.abs(cref).max(), (M, N, K)
    # few output tiles and a long K: FP64 partials of K slices, their
    # fixed-order sum and the epilogue (beta E, column energies)
    L.hipemu_gemm_ws.argtypes = [c_int, c_int, c_int, c_dbl, vp, vp, c_dbl, vp, vp, vp, vp, ctypes.c_long, vp]
    L.hipemu_gemm_split_slices.argtypes = [c_int, c_int, c_int, ctypes.c_long]
    M, N, K = 200, 256, 2630
    ws_len = 1 << 20
    assert L.hipemu_gemm_split_slices(M, N, K, ws_len) == 2
    assert L.hipemu_gemm_split_slices(M, N, K, M * N) == 0  # workspace for one slice only: unsplit
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    E = rng.standard_normal((M, N))
    D = np.zeros((M, N))
    MB = (M + 63) // 64
    cp = np.zeros((MB, N))
    ws = np.zeros(ws_len)
    cnt = np.zeros(256, dtype=np.int32)
    assert L.hipemu_gemm_ws(M, N, K, -1.0, A.ctypes.data, B.ctypes.data, 1.0, E.ctypes.data, D.ctypes.data,
                            cp.ctypes.data, ws.ctypes.data, ws_len, cnt.ctypes.data) == 0
    ref = E - A @ B
    assert np.abs(D - ref).max() <= 1e-12 * np.abs(ref).max()
    cref = np.array([(ref[64 * b:64 * (b + 1)] ** 2).sum(0) for b in range(MB)])
    assert np.abs(cp - cref).max() <= 1e-12 * np.abs(cref).max()


def case_proj_kernel():
    """The fused column-projection kernel on its own, against NumPy FP64:
    every vector width (4, 2, 1 columns per lane, and 1 for a misaligned
    base), every U tile count (r <= 16, <= 32, <= 64), both input types,
    ragged row quads and idle waves, and the short-column kernel (at most 8
    rows) in FP64 and FP32.  U is allocated with exactly the
    documented over-read tail, so AddressSanitizer flags any read past it."""
    import ctypes
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong
    L.hipemu_proj.argtypes = [i32, i32, i32, i32, i64, i32, vp, vp, i64, vp, i64, vp, vp, i32]
    rng = np.random.default_rng(3)
    tail = 64
    # (prec, shapes): FP64 everywhere; FP32 on the short-column kernel (at
    # most 8 rows and core columns, four aligned columns: cols = 8, no
    # shift), the only FP32 form the emulation models
    cases = [(0, (13, 5)), (0, (37, 20)), (0, (45, 40)), (0, (70, 16)), (0, (2, 0)), (0, (8, 8)), (0, (5, 3)),
             (0, (8, 0)), (1, (8, 8)), (1, (3, 2)), (1, (8, 0))]
    for dt, code in ((np.float32, 0), (np.float64, 1)):
        for cols, shift in ((8, 0), (6, 0), (3, 0), (8, 1)):
            for prec, (rows, r) in cases:
                if prec == 1 and (cols, shift) != (8, 0):
                    continue
                N = 5
                fs = rows * cols + 4
                buf = rng.standard_normal(N * fs + shift).astype(dt)
                Zb = buf[shift:]
                Ufull = np.zeros(rows * max(r, 1) + tail)
                Ufull[:rows * max(r, 1)] = rng.standard_normal(rows * max(r, 1)) / np.sqrt(rows)
                Ufull[rows * max(r, 1):] = np.nan  # over-read values are never used
                ldu = max(r, 1)
                fs_c = max(r, 1) * cols
                C = np.zeros(N * fs_c)
                zn = np.zeros(N * cols)
                rh = np.zeros(N * cols)
                rc = L.hipemu_proj(rows, r, N, cols, fs, code, Zb.ctypes.data, Ufull.ctypes.data, ldu,
                                   C.ctypes.data, fs_c, zn.ctypes.data, rh.ctypes.data, prec)
                assert rc == 0
                # FP32 products: operands and sums rounded to 24 bits
                tol_c, tol_r = (1e-13, 1e-12) if prec == 0 else (1e-6, 1e-6)
                U = Ufull[:rows * ldu].reshape(rows, ldu)[:, :r]
                for b in range(N):
                    Zf = Zb[b * fs: b * fs + rows * cols].astype(np.float64).reshape(rows, cols)
                    Cref = U.T @ Zf
                    z2 = (Zf * Zf).sum(axis=0)
                    got = C[b * fs_c: b * fs_c + r * cols].reshape(r, cols)
                    scale = np.sqrt(z2.max())
                    if r:
                        assert np.abs(got - Cref).max() <= tol_c * scale, (dt, cols, shift, rows, r, prec)
                    assert np.abs(zn[b * cols:(b + 1) * cols] - z2).max() <= 1e-13 * z2.max()
                    # the residual energy from the coefficients as computed: by
                    # Pythagoras, or explicitly in the short-column kernel (8
                    # rows and columns at most, four aligned columns per thread)
                    if rows <= 8 and r <= 8 and (cols, shift) == (8, 0):
                        res = ((Zf - U @ got) ** 2).sum(axis=0)
                    else:
                        res = z2 - (got * got).sum(axis=0)
                    assert np.abs(rh[b * cols:(b + 1) * cols] - res).max() <= 1e-12 * z2.max()
                    if not (rows <= 8 and r <= 8 and (cols, shift) == (8, 0)):
                        res_exact = z2 - (Cref * Cref).sum(axis=0)
                        assert np.abs(rh[b * cols:(b + 1) * cols] - res_exact).max() <= tol_r * z2.max()


def _server_run(specs, data, workers, budget):
    """Runs every stream's increments through one server (all submitted
    before any is waited for); returns the server and the stream ids."""
    import ctypes
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    srv = vp()
    assert L.ttice_server_create(workers, budget, ctypes.byref(srv)) == 0
    sids = []
    for dims, eps, algo in specs:
        sid = i32()
        arr = (ctypes.c_int64 * len(dims))(*dims)
        assert L.ttice_server_add_stream(srv, len(dims), arr, eps, 0, algo, 4, 64, ctypes.byref(sid)) == 0
        sids.append(sid.value)
    return srv, sids


def case_server():
    """The serving layer (one worker thread: the emulation runs one launch at
    a time): per-stream FIFO order, tickets and statuses, an error that
    leaves its stream usable, grouped level-1 launches, queued admission
    against the byte budget, removal, and alone-vs-mix: every stream's cores
    and reconstructions are bit-identical to the same stream served alone."""
    import ctypes
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    specs = [((16, 16, 3), 0.05, 0), ((12, 9, 4), 0.02, 0), ((8, 8, 8), 0.05, 1), ((16, 16, 3), 0.1, 0)]
    data = [list(synth.smooth_separable_stream(10, dims, 3, 1e-3, 1 + k, 40 + k, dtype=np.float64))
            for k, (dims, _, _) in enumerate(specs)]
    srv, sids = _server_run(specs, data, 1, 1 << 30)
    # interleave the increments of the streams; one bad batch on stream 1
    bad = np.full((2,) + specs[1][0], np.nan)
    tickets = []  # (stream index, increment index or -1, ticket)
    keep = []
    for j in range(max(len(x) for x in data)):
        for k, sid in enumerate(sids):
            if j < len(data[k]):
                Y = np.ascontiguousarray(data[k][j])
                keep.append(Y)
                t = i64()
                assert L.ttice_server_submit(srv, sid, Y.ctypes.data, Y.shape[0], 1, None, ctypes.byref(t)) == 0
                tickets.append((k, j, t.value))
            if k == 1 and j == 2:
                t = i64()
                assert L.ttice_server_submit(srv, sid, bad.ctypes.data, 2, 1, None, ctypes.byref(t)) == 0
                tickets.append((k, -1, t.value))
    for k, j, t in tickets:
        status, info = i32(), UpdateInfo()
        assert L.ttice_server_wait(srv, t, ctypes.byref(status), ctypes.byref(info)) == 0
        assert status.value == (-1 if j < 0 else 0), (k, j, status.value)
        done = i32()
        assert L.ttice_server_poll(srv, t, ctypes.byref(done), None, None) == -1  # released
    c = ServerCounters()
    assert L.ttice_server_stats(srv, ctypes.byref(c)) == 0
    assert c.pending == 0 and 0 < c.reserved_bytes <= c.budget_bytes and c.waiting_streams == 0
    # the worker found several Algorithm 1 streams waiting after its first update
    assert c.groups > 0 and c.grouped_increments > c.groups, (c.groups, c.grouped_increments)
    for k, sid in enumerate(sids):
        h = vp()
        assert L.ttice_server_stream_state(srv, sid, ctypes.byref(h)) == 0
        mixed = EmuTTICE.borrowed(L, h, specs[k][0])
        # the same stream served alone (its bad batch included)
        alone_srv, (asid,) = _server_run([specs[k]], [data[k]], 1, 1 << 30)
        for j, Y in enumerate(data[k]):
            Y = np.ascontiguousarray(Y)
            t, status = i64(), i32()
            assert L.ttice_server_submit(alone_srv, asid, Y.ctypes.data, Y.shape[0], 1, None, ctypes.byref(t)) == 0
            assert L.ttice_server_wait(alone_srv, t.value, ctypes.byref(status), None) == 0 and status.value == 0
        ha = vp()
        assert L.ttice_server_stream_state(alone_srv, asid, ctypes.byref(ha)) == 0
        alone = EmuTTICE.borrowed(L, ha, specs[k][0])
        assert mixed.ranks() == alone.ranks(), k
        assert np.array_equal(mixed.reconstruct(), alone.reconstruct()), k
        for i in range(len(specs[k][0]) + 1):
            assert np.array_equal(mixed.core(i), alone.core(i)), (k, i)
        L.ttice_server_destroy(alone_srv)
    # a reservation above the whole budget is refused
    big = (ctypes.c_int64 * 3)(512, 512, 512)
    sid = i32()
    assert L.ttice_server_add_stream(srv, 3, big, 0.1, 0, 0, 64, 64, ctypes.byref(sid)) == -2
    assert L.ttice_server_add_stream(srv, 3, big, 0.1, 0, 0, 64, 32, ctypes.byref(sid)) == -1  # max_tensors < max_batch
    # removal returns the reservation; the id is then unknown
    before = c.reserved_bytes
    assert L.ttice_server_remove_stream(srv, sids[0]) == 0
    assert L.ttice_server_stats(srv, ctypes.byref(c)) == 0
    assert c.reserved_bytes < before
    t = i64()
    Y = keep[0]
    assert L.ttice_server_submit(srv, sids[0], Y.ctypes.data, Y.shape[0], 1, None, ctypes.byref(t)) == -1
    assert L.ttice_server_submit(srv, sids[1], None, 5, 1, None, ctypes.byref(t)) == -1  # null batch / over max_batch
    # the tensor limit: stream 3 has taken 10 of its 64 tensors
    zeros = np.zeros((4,) + specs[3][0])
    for _ in range(13):
        assert L.ttice_server_submit(srv, sids[3], zeros.ctypes.data, 4, 1, None, ctypes.byref(t)) == 0
        assert L.ttice_server_wait(srv, t.value, None, None) == 0
    assert L.ttice_server_submit(srv, sids[3], zeros.ctypes.data, 3, 1, None, ctypes.byref(t)) == -1  # 65 > 64
    assert L.ttice_server_submit(srv, sids[3], zeros.ctypes.data, 2, 1, None, ctypes.byref(t)) == 0
    assert L.ttice_server_wait(srv, t.value, None, None) == 0
    L.ttice_server_destroy(srv)


def case_server_admission():
    """Queued admission: with a budget that holds two streams, a third waits
    (its increments queue) and is admitted when a stream is removed; its
    results equal the same stream served alone."""
    import ctypes
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    dims, eps = (16, 16, 3), 0.05
    arr = (ctypes.c_int64 * 3)(*dims)
    # the footprint of one stream, measured on a server of ample budget
    probe, sid = vp(), i32()
    assert L.ttice_server_create(1, 1 << 40, ctypes.byref(probe)) == 0
    assert L.ttice_server_add_stream(probe, 3, arr, eps, 0, 0, 4, 64, ctypes.byref(sid)) == 0
    c = ServerCounters()
    assert L.ttice_server_stats(probe, ctypes.byref(c)) == 0
    one = c.reserved_bytes
    L.ttice_server_destroy(probe)
    srv = vp()
    assert L.ttice_server_create(1, 2 * one + one // 2, ctypes.byref(srv)) == 0
    sids = []
    for _ in range(3):
        assert L.ttice_server_add_stream(srv, 3, arr, eps, 0, 0, 4, 64, ctypes.byref(sid)) == 0
        sids.append(sid.value)
    assert L.ttice_server_stats(srv, ctypes.byref(c)) == 0
    assert c.waiting_streams == 1 and c.reserved_bytes == 2 * one, (c.waiting_streams, c.reserved_bytes, one)
    h = vp()
    assert L.ttice_server_stream_state(srv, sids[2], ctypes.byref(h)) == -4  # not admitted (ESTATE)
    data = list(synth.smooth_separable_stream(6, dims, 3, 1e-3, 2, 77, dtype=np.float64))
    keep, tickets = [], []
    for Y in data:
        Y = np.ascontiguousarray(Y)
        keep.append(Y)
        t = i64()
        assert L.ttice_server_submit(srv, sids[2], Y.ctypes.data, Y.shape[0], 1, None, ctypes.byref(t)) == 0
        tickets.append(t.value)
    done = i32()
    assert L.ttice_server_poll(srv, tickets[0], ctypes.byref(done), None, None) == 0 and done.value == 0
    assert L.ttice_server_stats(srv, ctypes.byref(c)) == 0
    assert c.pending == len(data)
    assert L.ttice_server_remove_stream(srv, sids[0]) == 0  # frees one stream's budget: the third is admitted
    status = i32()
    for t in tickets:
        assert L.ttice_server_wait(srv, t, ctypes.byref(status), None) == 0 and status.value == 0
    assert L.ttice_server_stats(srv, ctypes.byref(c)) == 0
    assert c.waiting_streams == 0 and c.reserved_bytes == 2 * one and c.pending == 0
    assert L.ttice_server_stream_state(srv, sids[2], ctypes.byref(h)) == 0
    served = EmuTTICE.borrowed(L, h, dims)
    alone_srv, (asid,) = _server_run([(dims, eps, 0)], [data], 1, 1 << 40)
    for Y in keep:
        t = i64()
        assert L.ttice_server_submit(alone_srv, asid, Y.ctypes.data, Y.shape[0], 1, None, ctypes.byref(t)) == 0
        assert L.ttice_server_wait(alone_srv, t.value, ctypes.byref(status), None) == 0 and status.value == 0
    ha = vp()
    assert L.ttice_server_stream_state(alone_srv, asid, ctypes.byref(ha)) == 0
    alone = EmuTTICE.borrowed(L, ha, dims)
    assert served.ranks() == alone.ranks()
    for i in range(len(dims) + 1):
        assert np.array_equal(served.core(i), alone.core(i)), i
    L.ttice_server_destroy(alone_srv)
    # a waiting stream with nothing queued can be removed
    assert L.ttice_server_add_stream(srv, 3, arr, eps, 0, 0, 4, 64, ctypes.byref(sid)) == 0
    assert L.ttice_server_stats(srv, ctypes.byref(c)) == 0 and c.waiting_streams == 1
    assert L.ttice_server_remove_stream(srv, sid.value) == 0
    assert L.ttice_server_stats(srv, ctypes.byref(c)) == 0 and c.waiting_streams == 0
    L.ttice_server_destroy(srv)


CASES = {k[5:]: v for k, v in globals().items() if k.startswith("case_")}

if __name__ == "__main__":
    L = load(sys.argv[1])
    names = sys.argv[2:] or list(CASES)
    for name in names:
        print("emu case", name, flush=True)
        CASES[name]()
    print("emu cases ok", flush=True)
