"""Plain FP64 CPU oracle for TT-ICE and TT-ICE* (TEST INFRASTRUCTURE ONLY).

This module is the correctness reference of the repository.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path (the HIP library and its Python binding) never does.
It shares no code with the GPU path.

It follows the paper (Aksoy, Gorsich, Veerapaneni, Gorodetsky, "An
Incremental Tensor Train Decomposition Algorithm", arXiv 2211.12487) step by
step in NumPy float64, with LAPACK's SVD (``numpy.linalg.svd``) as the only
library primitive besides matrix products:

* Sec. 2.1: unfolding, contraction (eq:tensorcontraction), TT-cores
  (eq:tt_core_reshape), delta-truncated SVD with the Eckart-Young tail
  (eq:deltasvd) and TT-SVD with delta = eps*||Y||/sqrt(d-1)  -> ``tt_svd``.
* Sec. 3.1, Algorithm 1 (TT-ICE): residual of the first unfolding
  (eq:first_resid), truncated SVD of the residual (eq:svdfirst), core
  expansion (eq:coreexpansion), zero padding of the next core (eq:ukpad),
  projection onto the updated core (eq:project_further), next residual
  (eq:ithresidual) and the last-core update (eq:lastcore)  -> ``TTICE.update``
  with ``algo="plain"``.
* Corollary 1: per-core tolerance eps_des*||Y^{k+1}||_F/sqrt(d).
* Sec. 3.3, Algorithm 2 (TT-ICE*): per-observation relative error with the
  existing cores (eq:relerror), skip rule, subselection (eq:subselectheuristic),
  relaxed tolerance (eq:epsilonmodification), occupancy (eq:coreoccupancy),
  re-projection of the whole batch and append  -> ``algo="star"``.
* Eq. eq:last_core_latent: extraction of stored tensors -> ``reconstruct``.
* Sec. 4.1: compression ratio (eq:compressionratio) and relative
  reconstruction error (eq:MRRE).

Readings taken where the paper is silent or ambiguous:

* The TT-ranks start at zero; the first update on empty cores is then a
  TT-SVD of the first increment at eps/sqrt(d).
* Rank choice: the smallest r whose discarded energy sum_{j>r} sigma_j^2 is
  <= eps_i^2 (non-strict); r = 0 is allowed, and r never exceeds the number
  of directions still free, r_{i-1} n_i - r_i.
* Unfoldings and reshapes are C-ordered; each increment is held frame-major
  as Z[b] (rows x cols), which only permutes the columns of the unfolding
  and leaves its left singular vectors and singular values unchanged.
* Eq. eq:ithresidual is read with the padded core of the *next* level, as in
  Algorithm 1's loop.
* New directions are re-orthogonalised against the existing core (two
  classical Gram-Schmidt passes) and among themselves (QR), and each new
  column gets the sign that makes its largest-magnitude entry positive.
  In exact arithmetic none of this changes the result.
* TT-ICE*: the relative error of an all-zero observation is 0; the last
  core is zero-padded (as in Algorithm 1) before the re-projected columns
  are appended; the exact relaxed tolerance is used.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "truncation_rank",
    "TTICE",
    "tt_svd",
    "tt_full",
    "compression_ratio",
    "relative_error",
]


# ---------------------------------------------------------------------------
# Truncated SVD (Sec. 2.1, eq:deltasvd)
# ---------------------------------------------------------------------------

def tail_energies(s: np.ndarray) -> np.ndarray:
    """tail[r] = sum_{j >= r} s_j^2 for r = 0..len(s) (tail[len(s)] = 0).

    By Eckart-Young-Mirsky this is the squared Frobenius error of the best
    rank-r approximation (eq:deltasvd)."""
    s2 = np.asarray(s, dtype=np.float64) ** 2
    tail = np.zeros(len(s2) + 1)
    for r in range(len(s2) - 1, -1, -1):
        tail[r] = tail[r + 1] + s2[r]
    return tail


def truncation_rank(s: np.ndarray, tol2: float) -> int:
    """Smallest r whose discarded energy sum_{j>=r} s_j^2 does not exceed tol2."""
    tail = tail_energies(s)
    for r in range(len(tail)):
        if tail[r] <= tol2:
            return r
    return len(s)


def truncated_svd(A: np.ndarray, tol: float):
    """SVD(A, tol) of Algorithm 1: leading left singular vectors whose
    truncation error ||E||_F is at most ``tol``.  Returns (U_r, s, r, tail_r)."""
    if A.size == 0:
        return np.zeros((A.shape[0], 0)), np.zeros(0), 0, 0.0
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    r = truncation_rank(s, tol * tol)
    return U[:, :r], s, r, float(tail_energies(s)[r])


# ---------------------------------------------------------------------------
# TT format helpers (Sec. 2.1)
# ---------------------------------------------------------------------------

def tt_full(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Contract 3-way cores G_i (r_{i-1}, n_i, r_i) along their shared rank
    modes (eq:tensorcontraction); the outer ranks must be 1 (or the last
    core's trailing mode is kept as an extra mode)."""
    out = cores[0]
    for G in cores[1:]:
        out = np.tensordot(out, G, axes=([-1], [0]))
    # drop the leading r_0 = 1 mode, and the trailing r_d mode when it is 1
    out = out.reshape(out.shape[1:])
    if out.shape[-1] == 1:
        out = out.reshape(out.shape[:-1])
    return out


def tt_svd(X: np.ndarray, eps: float):
    """TT-SVD of a D-way tensor (Sec. 2.1, eqs. ttcoresstep1-3): sequential
    truncated SVDs of the unfoldings with delta = eps*||X||_F/sqrt(D-1),
    carrying Sigma V forward.  Returns (cores, ranks) with cores[i] of shape
    (r_i, n_{i+1}, r_{i+1}) and ranks = [1, r_1, ..., r_{D-1}, 1]."""
    X = np.asarray(X, dtype=np.float64)
    dims = X.shape
    D = len(dims)
    delta = eps * np.linalg.norm(X) / math.sqrt(D - 1)
    ranks = [1]
    cores = []
    C = X.reshape(dims[0], -1)
    for k in range(D - 1):
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        r = truncation_rank(s, delta * delta)
        cores.append(U[:, :r].reshape(ranks[-1], dims[k], r))
        ranks.append(r)
        C = (s[:r, None] * Vt[:r]).reshape(r * dims[k + 1], -1)
    cores.append(C.reshape(ranks[-1], dims[-1], 1))
    ranks.append(1)
    return cores, ranks


def compression_ratio(dims: Sequence[int], n_total: int, ranks: Sequence[int]) -> float:
    """CR (eq:compressionratio) of the (d+1)-way accumulation with mode sizes
    n_1..n_d, n_total and TT-ranks r_0=1, r_1..r_d, r_{d+1}=1."""
    n = list(dims) + [n_total]
    num = float(np.prod(np.array(n, dtype=np.float64)))
    den = sum(ranks[i] * n[i] * ranks[i + 1] for i in range(len(n)))
    return num / den if den > 0 else float("inf")


def relative_error(X: np.ndarray, Xhat: np.ndarray) -> float:
    """RRE (eq:MRRE): ||X - Xhat||_F / ||X||_F."""
    nx = np.linalg.norm(X)
    return float(np.linalg.norm(X - Xhat) / nx) if nx > 0 else float(np.linalg.norm(Xhat))


# ---------------------------------------------------------------------------
# TT-ICE / TT-ICE*
# ---------------------------------------------------------------------------

def _orthonormal_new_directions(U: np.ndarray, UR: np.ndarray) -> np.ndarray:
    """Re-orthogonalise the new directions against U (two CGS passes), then
    among themselves (QR), with the sign convention: the largest-magnitude
    entry of each new column is positive (ties: lowest row index)."""
    if UR.shape[1] == 0:
        return UR
    W = UR.copy()
    for _ in range(2):
        if U.shape[1]:
            W = W - U @ (U.T @ W)
    Q, Rq = np.linalg.qr(W)
    # keep the orientation of the SVD's vectors: diag(Rq) > 0
    sgn = np.sign(np.diag(Rq))
    sgn[sgn == 0] = 1.0
    Q = Q * sgn
    for j in range(Q.shape[1]):
        k = int(np.argmax(np.abs(Q[:, j])))
        if Q[k, j] < 0:
            Q[:, j] = -Q[:, j]
    return Q


class TTICE:
    """Incremental TT accumulation maintained by TT-ICE (Algorithm 1) or
    TT-ICE* (Algorithm 2).

    State: the unfolded cores U_i of shape (r_{i-1} n_i, r_i), i = 1..d, with
    r_0 = 1, initially all ranks 0, and the last core G of shape
    (r_d, N_total) whose columns are the latent coefficients of the stored
    tensors (Sec. 3.1, eq:lastcore)."""

    def __init__(self, dims: Sequence[int], eps: float, algo: str = "plain",
                 tau: float = 1.0, skip_rule: str = "mean"):
        self.dims = tuple(int(n) for n in dims)
        self.d = len(self.dims)
        if self.d < 1 or any(n < 1 for n in self.dims):
            raise ValueError("bad dims")
        if not (0.0 < eps < 1.0):
            raise ValueError("eps must lie in (0, 1)")
        if algo not in ("plain", "star"):
            raise ValueError("algo must be 'plain' or 'star'")
        if skip_rule not in ("mean", "batch", "none"):
            raise ValueError("skip_rule must be 'mean', 'batch' or 'none'")
        self.eps = float(eps)
        self.algo = algo
        self.tau = float(tau)
        self.skip_rule = skip_rule
        self.ranks = [1] + [0] * self.d          # r_0 .. r_d
        self.U: List[np.ndarray] = []
        for i, n in enumerate(self.dims):
            rows = (1 if i == 0 else 0) * n
            self.U.append(np.zeros((rows, 0)))
        self.G = np.zeros((0, 0))                 # (r_d, N_total)
        self.history: List[dict] = []

    # -- helpers -----------------------------------------------------------
    @property
    def n_total(self) -> int:
        return self.G.shape[1]

    def cols(self, i: int) -> int:
        """Columns per tensor of the level-i unfolding (0-based i): n_{i+2}..n_d."""
        return int(np.prod(self.dims[i + 1:], dtype=np.int64)) if i + 1 < self.d else 1

    def _pad_next(self, i: int, r_old: int, r_new_dirs: int) -> None:
        """eq:ukpad: reshape U_{i+1} to (r_i, n_{i+1} r_{i+1}), stack r_R zero
        rows, reshape back; for the last level, pad the last core's rows."""
        if r_new_dirs == 0:
            return
        if i + 1 < self.d:
            Un = self.U[i + 1]
            n_next = self.dims[i + 1]
            r_next = Un.shape[1]
            M = Un.reshape(r_old, n_next * r_next)
            M = np.vstack([M, np.zeros((r_new_dirs, n_next * r_next))])
            self.U[i + 1] = M.reshape((r_old + r_new_dirs) * n_next, r_next)
        else:
            self.G = np.vstack([self.G, np.zeros((r_new_dirs, self.G.shape[1]))])

    def project(self, Y: np.ndarray):
        """Push tensors through the current cores without updating them.

        Returns (coefficients (N, r_d), Ytilde (N, n_1..n_d)) where Ytilde is
        the approximation of Y with the existing cores, i.e. the last-core
        columns a stored copy of Y would get, reconstructed (Sec. 3.3)."""
        Y = self._as_batch(Y)
        N = Y.shape[0]
        Z = Y.reshape(N, self.dims[0], self.cols(0))
        for i in range(self.d):
            U = self.U[i]
            C = np.einsum("rk,brc->bkc", U, Z)
            if i + 1 < self.d:
                Z = C.reshape(N, self.ranks[i + 1] * self.dims[i + 1], self.cols(i + 1))
            else:
                Z = C
        coef = Z.reshape(N, self.ranks[self.d])
        return coef, self._expand(coef.T)

    def _expand(self, cols: np.ndarray) -> np.ndarray:
        """Ŷ = G_1 x ... x G_d x cols (eq:last_core_latent) for a (r_d, m) block."""
        X = cols                                   # (r_d, m) = level-d data, cols_d = 1
        m = cols.shape[1]
        for i in range(self.d - 1, -1, -1):
            U = self.U[i]                          # (r_{i-1} n_i, r_i)
            # X: (r_i, m * tail) with tail = n_{i+1}..n_d arranged per tensor
            tail = self.cols(i)                                # n_{i+1}..n_d (1-based)
            Xb = X.reshape(self.ranks[i + 1], m, tail)         # (r_i, m, tail)
            Yb = np.einsum("pk,kmt->mpt", U, Xb)               # (m, r_{i-1} n_i, tail)
            # regroup: rows r_{i-1} n_i -> (r_{i-1}, n_i * tail)
            Yb = Yb.reshape(m, self.ranks[i], self.dims[i] * tail)
            X = np.transpose(Yb, (1, 0, 2)).reshape(self.ranks[i], m * self.dims[i] * tail)
        return X.reshape((m,) + self.dims)

    def reconstruct(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        """Stored tensors first..first+count-1 (eq:last_core_latent)."""
        if count is None:
            count = self.n_total - first
        if first < 0 or count < 0 or first + count > self.n_total:
            raise IndexError("range outside the stored tensors")
        return self._expand(self.G[:, first:first + count])

    @staticmethod
    def _as_batch(Y):
        return np.asarray(Y, dtype=np.float64)

    # -- Algorithm 1 core loop ----------------------------------------------
    def _core_loop(self, Z: np.ndarray, tol: float, info: dict,
                   use_occupancy: bool) -> np.ndarray:
        """Levels i = 1..d of Algorithm 1 on frame-major data Z (N, n_1, cols)
        with the SVD tolerance ``tol`` for every core.  Updates the cores in
        place and returns U_d^T Z_d, the (N, r_d) last-core coefficients."""
        N = Z.shape[0]
        for i in range(self.d):
            U = self.U[i]                          # padded core, (rows, r_i)
            rows, r_i = U.shape
            assert Z.shape[1] == rows
            occupancy = r_i / rows if rows else 1.0
            if use_occupancy and occupancy >= self.tau:
                # eq:coreoccupancy / Algorithm 2: leave the core as it is
                info["rho2"].append(float("nan"))
                info["rR"].append(0)
                info["tail2"].append(0.0)
                info["margin"].append(float("inf"))
                info["occupancy_skip"].append(True)
            else:
                info["occupancy_skip"].append(False)
                C = np.einsum("rk,brc->bkc", U, Z)                  # U^T Z
                R = Z - np.einsum("rk,bkc->brc", U, C)              # eq:first_resid / eq:ithresidual
                rho2 = float(np.sum(R * R))
                info["rho2"].append(rho2)
                rR, tail2, margin = 0, rho2, float("inf")
                if rho2 > tol * tol:
                    Rcat = np.transpose(R, (1, 0, 2)).reshape(rows, N * self.cols(i))   # [R(1) ... R(N)]
                    UR, s, rR, tail2 = truncated_svd(Rcat, tol)
                    tails = tail_energies(s)
                    rR = min(rR, rows - r_i)
                    tail2 = float(tails[rR])
                    UR = UR[:, :rR]
                    t2 = tol * tol
                    m_hi = abs(tails[rR] - t2) / t2
                    m_lo = abs(tails[rR - 1] - t2) / t2 if rR >= 1 else float("inf")
                    margin = min(m_hi, m_lo)
                    UR = _orthonormal_new_directions(U, UR)
                    self.U[i] = np.hstack([U, UR])                  # eq:coreexpansion
                    r_old = r_i
                    self.ranks[i + 1] = r_i + rR
                    self._pad_next(i, r_old, rR)                    # eq:ukpad
                info["rR"].append(int(rR))
                info["tail2"].append(float(tail2))
                info["margin"].append(float(margin))
            # eq:project_further: project onto the *updated* core, reshape
            Unew = self.U[i]
            C = np.einsum("rk,brc->bkc", Unew, Z)
            if i + 1 < self.d:
                Z = C.reshape(N, self.ranks[i + 1] * self.dims[i + 1], self.cols(i + 1))
            else:
                Z = C
        return Z.reshape(N, self.ranks[self.d])

    def _append_columns(self, coef: np.ndarray) -> None:
        """eq:lastcore: append the new latent columns to the last core."""
        r_d = self.ranks[self.d]
        if self.G.shape[0] != r_d:
            raise AssertionError("last core rows out of sync with r_d")
        self.G = np.hstack([self.G, coef.T.reshape(r_d, coef.shape[0])])

    def _new_info(self, N: int, normY2: float) -> dict:
        return dict(N=N, normY2=normY2, rho2=[], rR=[], tail2=[], margin=[],
                    occupancy_skip=[], skipped=False, used=N, eps_core=0.0,
                    eps_upd=self.eps)

    # -- public update ---------------------------------------------------------
    def update(self, Y: np.ndarray) -> dict:
        """Incorporate a batch Y of shape (N, n_1, ..., n_d) (or a single
        tensor of shape (n_1, ..., n_d)).  Returns a per-update info dict."""
        Y = self._as_batch(Y)
        if Y.shape == self.dims:
            Y = Y[None]
        if Y.shape[1:] != self.dims:
            raise ValueError("batch shape does not match dims")
        if not np.all(np.isfinite(Y)):
            raise ValueError("non-finite batch")
        N = Y.shape[0]
        normY2 = float(np.sum(Y * Y))
        info = self._new_info(N, normY2)
        if N == 0:
            info["ranks"] = list(self.ranks) + [1]
            return info
        if self.algo == "plain":
            tol = self.eps * math.sqrt(normY2) / math.sqrt(self.d)       # Corollary 1
            info["eps_core"] = tol
            coef = self._core_loop(Y.reshape(N, self.dims[0], self.cols(0)), tol, info, False)
            self._append_columns(coef)
        else:
            self._update_star(Y, info)
        info["ranks"] = list(self.ranks) + [1]
        # Theorem 1's proof is a chain of Pythagorean equalities, so for
        # Algorithm 1 the squared error of the increment is the discarded energy.
        info["achieved2"] = float(np.sum(info["tail2"])) if self.algo == "plain" else None
        self.history.append(info)
        return info

    def _update_star(self, Y: np.ndarray, info: dict) -> None:
        """Algorithm 2 (TT-ICE*)."""
        N = Y.shape[0]
        eps = self.eps
        # eq:relerror with the existing cores
        _, Ytil = self.project(Y)
        err2 = np.array([float(np.sum((Y[b] - Ytil[b]) ** 2)) for b in range(N)])
        nrm2 = np.array([float(np.sum(Y[b] ** 2)) for b in range(N)])
        rel = np.where(nrm2 > 0, np.sqrt(err2 / np.where(nrm2 > 0, nrm2, 1.0)), 0.0)
        info["rel_err_old"] = rel.tolist()
        if self.skip_rule == "mean":
            skip = float(np.mean(rel)) <= eps
        elif self.skip_rule == "batch":   # eq:batchrelativeerror
            tot = float(np.sum(nrm2))
            skip = (math.sqrt(float(np.sum(err2)) / tot) if tot > 0 else 0.0) <= eps
        else:   # "none": the Subselect variant of Sec. 5 never skips
            skip = False
        # with no tensor above eps there is nothing to update with
        skip = skip or not bool(np.any(rel > eps))
        if skip:
            info["skipped"] = True
            info["used"] = 0
            coef, _ = self.project(Y)                       # eq:appendupdate
            info["rR"] = [0] * self.d
            info["frame_err2"] = [float(x) for x in err2]
            self._append_columns(coef)
            return
        sel = rel > eps                                      # eq:subselectheuristic
        D = Y[sel]
        info["used"] = int(D.shape[0])
        normD2 = float(np.sum(D * D))
        normY2 = float(np.sum(nrm2))
        num = eps * eps * normY2 - float(np.sum(err2[~sel]))  # eq:epsilonmodification
        eps_upd = math.sqrt(max(num, 0.0) / normD2)
        info["eps_upd"] = eps_upd
        tol = eps_upd * math.sqrt(normD2) / math.sqrt(self.d)
        info["eps_core"] = tol
        self._core_loop(D.reshape(D.shape[0], self.dims[0], self.cols(0)), tol, info, True)
        coef, _ = self.project(Y)                            # re-project the whole batch
        self._append_columns(coef)

    # -- diagnostics --------------------------------------------------------
    def tt_cores(self) -> List[np.ndarray]:
        """3-way cores G_1..G_d (eq:tt_core_reshape) plus the last core as
        G_{d+1} of shape (r_d, N_total, 1)."""
        out = []
        for i in range(self.d):
            out.append(self.U[i].reshape(self.ranks[i], self.dims[i], self.ranks[i + 1]))
        out.append(self.G.reshape(self.ranks[self.d], self.n_total, 1))
        return out

    def orthogonality_error(self) -> float:
        """max_i ||U_i^T U_i - I||_max (Sec. 3.1: the cores stay orthonormal)."""
        e = 0.0
        for U in self.U:
            if U.shape[1]:
                e = max(e, float(np.max(np.abs(U.T @ U - np.eye(U.shape[1])))))
        return e
