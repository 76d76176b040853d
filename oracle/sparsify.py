"""Explicit Technique-B sparsification of a river endgame's payoff matrix
(oracle; test infrastructure only).

Proposition 1 writes the payoff matrix, in hand-major layout (row
h1 * S1 + sigma1, column h2 * S2 + sigma2), as

    A = C (x) F + (L1 W L2) (x) S,

with lambda_i = mu_i / sqrt(beta), L_i = diag(lambda_i), W the showdown
outcome gamma (0 on pairs that share a card), Hx the 0/1 matrix of such
pairs, C = lambda1 lambda2^T - L1 Hx L2, F[s1, s2] the sum of Player 1's fold
payoffs at the sequence pair and S[s1, s2] the sum of its showdown stakes.

Technique B (Section 4) ranks Player 1's hands by strength and writes
W = D^{-1} Y, where D is lower bidiagonal (1 on the diagonal, -1 below it)
and Y = D W holds the differences of consecutive rows, which are sparse.
Its proposition then gives A = Ahat + U M^{-1} V^T with

    Ahat = -(L1 Hx L2) (x) F,
    U = [L1 (x) I | lambda1 (x) I],      M = blockdiag(D (x) I, I),
    V = [(L2 Y^T) (x) S^T | lambda2 (x) F^T].

The printed proposition has mu where the rank-one fold term needs lambda: with
mu the product would lack the 1/beta of the deal probability.  lambda is used
here (the same reading as for C).

The Postprocessing subsection removes columns of V that are identically zero:
with M unit lower triangular, a zero column j makes y_j = -sum_i M[j, i] y_i,
so y_j is substituted into the other rows of M and into U's columns, and
column j leaves U, M and V.

Only river endgames (one final board) are handled.  Sizes are numbers of
stored nonzeros, the paper's size metric (Table 1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import skeleton as sk
from .payoff import Game


def sequence_matrices(game: Game):
    """F (fold payoffs) and S (showdown stakes) over sequence pairs."""
    S1, S2 = game.S
    F = np.zeros((S1, S2))
    S = np.zeros((S1, S2))
    for t in game.sf.terminals:
        if t.board >= 0 or t.runout:
            raise ValueError("Technique B is built here for river endgames only")
        if t.kind == sk.SHOWDOWN:
            S[t.seq1, t.seq2] += t.c1
        else:
            F[t.seq1, t.seq2] += t.u1
    return F, S


def strength_order(game: Game):
    """Player 1's hands by increasing strength (ties keep list order)."""
    return np.argsort(game.desc.strength[0][0].astype(np.int64), kind="stable")


def factors(game: Game):
    """(Ahat, U, M, V, order) in hand-major layout with Player 1's hands in
    `order` (strength order); Player 2's hands keep their list order."""
    hm = game.hm
    if hm.rivers:
        raise ValueError("Technique B is built here for river endgames only")
    S1, S2 = game.S
    N1, N2 = game.N
    order = strength_order(game)
    lam1 = hm.mu[0][order] / np.sqrt(hm.beta)
    lam2 = hm.mu[1] / np.sqrt(hm.beta)
    Hx = hm.share[order].astype(np.float64)
    W = hm.gamma(-1)[order]
    F, S = sequence_matrices(game)
    D = sp.eye(N1, format="csr") - sp.eye(N1, k=-1, format="csr")
    Y = sp.csr_matrix(D @ W)
    L1, L2 = sp.diags(lam1), sp.diags(lam2)
    I1 = sp.eye(S1, format="csr")
    Ahat = -sp.kron(sp.csr_matrix(L1 @ Hx @ L2), sp.csr_matrix(F), format="csr")
    U = sp.hstack([sp.kron(L1, I1), sp.kron(sp.csr_matrix(lam1[:, None]), I1)], format="csc")
    M = sp.block_diag([sp.kron(D, I1), sp.eye(S1)], format="csr")
    V = sp.hstack([sp.kron(sp.csr_matrix(L2 @ Y.T), sp.csr_matrix(S.T)),
                   sp.kron(sp.csr_matrix(lam2[:, None]), sp.csr_matrix(F.T))], format="csc")
    return [m.tocsr() if i in (0, 2) else m for i, m in enumerate((Ahat, U, M, V))] + [order]


def _clean(m):
    m = m.copy()
    m.eliminate_zeros()
    return m


def postprocess(U, M, V):
    """Drop the identically zero columns of V, substituting their unknowns
    (Postprocessing subsection).  M must be unit lower triangular."""
    V = _clean(sp.csc_matrix(V))
    U = _clean(sp.csc_matrix(U))
    M = _clean(sp.csr_matrix(M))
    n = M.shape[0]
    ucol = [dict(zip(U.indices[U.indptr[j]:U.indptr[j + 1]].tolist(),
                     U.data[U.indptr[j]:U.indptr[j + 1]].tolist())) for j in range(n)]
    mrow = []
    mcol = [set() for _ in range(n)]
    for k in range(n):
        cols = M.indices[M.indptr[k]:M.indptr[k + 1]]
        vals = M.data[M.indptr[k]:M.indptr[k + 1]]
        row = {}
        for i, v in zip(cols.tolist(), vals.tolist()):
            if i == k:
                if v != 1.0:
                    raise ValueError("M must have a unit diagonal")
            elif i > k:
                raise ValueError("M must be lower triangular")
            else:
                row[i] = v
                mcol[i].add(k)
        mrow.append(row)
    zero = np.diff(V.indptr) == 0
    for j in np.flatnonzero(zero).tolist():
        a = mrow[j]                      # y_j = -sum_i a[i] y_i
        for i, ai in a.items():
            for r, u in ucol[j].items():
                ucol[i][r] = ucol[i].get(r, 0.0) - ai * u
            mcol[i].discard(j)
        for k in mcol[j]:
            mkj = mrow[k].pop(j)
            for i, ai in a.items():
                mrow[k][i] = mrow[k].get(i, 0.0) - mkj * ai
                mcol[i].add(k)
        ucol[j], mrow[j], mcol[j] = {}, {}, set()
    keep = np.flatnonzero(~zero)
    pos = -np.ones(n, dtype=np.int64)
    pos[keep] = np.arange(len(keep))
    ur, uc, uv, mr, mc, mv = [], [], [], [], [], []
    for new, j in enumerate(keep.tolist()):
        for r, u in ucol[j].items():
            ur.append(r), uc.append(new), uv.append(u)
        mr.append(new), mc.append(new), mv.append(1.0)
        for i, v in mrow[j].items():
            mr.append(new), mc.append(int(pos[i])), mv.append(v)
    m = len(keep)
    U2 = _clean(sp.csc_matrix((uv, (ur, uc)), shape=(U.shape[0], m)))
    M2 = _clean(sp.csr_matrix((mv, (mr, mc)), shape=(m, m)))
    V2 = V[:, keep]
    return U2, M2, V2


def size(*mats) -> int:
    """Stored nonzeros (explicit zeros not counted)."""
    return int(sum(_clean(sp.csr_matrix(m)).nnz for m in mats))


def payoff_nnz(game: Game) -> int:
    """Nonzeros of A without forming it: fold and showdown terminals sit on
    different sequence pairs, so each pair contributes the nonzeros of its
    hand factor (C for folds, L1 W L2 for showdowns)."""
    hm = game.hm
    F, S = sequence_matrices(game)
    lam1 = hm.mu[0] / np.sqrt(hm.beta)
    lam2 = hm.mu[1] / np.sqrt(hm.beta)
    C = np.where(hm.share, 0.0, np.outer(lam1, lam2))
    Wl = hm.gamma(-1) * np.outer(lam1, lam2)
    both = (F != 0) & (S != 0)
    if both.any():
        raise ValueError("a sequence pair holds both fold and showdown payoffs")
    return int((F != 0).sum()) * int((C != 0).sum()) + int((S != 0).sum()) * int((Wl != 0).sum())


def dense_hand_major(game: Game, order=None):
    """The oracle's dense A moved to hand-major layout, Player 1's hands in
    `order`."""
    S1, S2 = game.S
    N1, N2 = game.N
    A = game.dense_A().reshape(S1, N1, S2, N2).transpose(1, 0, 3, 2)
    if order is not None:
        A = A[order]
    return A.reshape(N1 * S1, N2 * S2)


def product(Ahat, U, M, V):
    """Ahat + U M^{-1} V^T as a dense matrix (small games)."""
    from scipy.sparse.linalg import spsolve_triangular
    Z = spsolve_triangular(sp.csr_matrix(M), V.T.toarray(), lower=True, unit_diagonal=True)
    return Ahat.toarray() + U @ Z
