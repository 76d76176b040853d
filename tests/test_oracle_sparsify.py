"""Explicit Technique-B factors (Section 4 and its Postprocessing subsection)
checked against the payoff matrix the oracle sums from terminals, and the
sparsity the technique is built on."""
import dataclasses

import numpy as np
import pytest

from paper_2112_03804_amd import instances as I
from oracle import payoff, sparsify

RIVERS = [
    ("kuhn", I.kuhn),
    ("tiny", I.tiny_config),
    ("small_river", lambda: I.small_river(0)),
    ("small_river_pruned", lambda: I.small_river(5, deck_size=11, n_keep=(20, 13))),
    ("small_river_3", lambda: I.small_river(3)),
]


def _disjoint(d):
    """The same game with each player's hands drawn from its own half of the
    deck, so no hand pair shares a card."""
    cards = sorted(set(int(c) for p in range(2) for c in d.hands[p].ravel()))
    half = set(cards[: len(cards) // 2])
    keep = [np.array([all((int(c) in half) == (p == 0) for c in h) for h in d.hands[p]]) for p in range(2)]
    return dataclasses.replace(
        d.copy(),
        hands=[d.hands[p][keep[p]] for p in range(2)],
        strength=[d.strength[p][:, keep[p]] for p in range(2)],
        range_=[d.range_[p][keep[p]] for p in range(2)],
    )


@pytest.mark.parametrize("name,fn", RIVERS)
def test_factors_reproduce_payoff_matrix(name, fn):
    g = payoff.Game(fn())
    Ahat, U, M, V, order = sparsify.factors(g)
    A = sparsify.dense_hand_major(g, order)
    scale = np.abs(A).max()
    assert np.abs(sparsify.product(Ahat, U, M, V) - A).max() <= 1e-12 * scale
    # a wrong hand order breaks it: the factors are tied to strength order
    if g.N[0] > 2:
        A_list = sparsify.dense_hand_major(g)
        if not np.array_equal(order, np.arange(g.N[0])):
            assert np.abs(sparsify.product(Ahat, U, M, V) - A_list).max() > 1e-6 * scale


@pytest.mark.parametrize("name,fn", RIVERS)
def test_postprocessing_keeps_the_product_and_drops_zero_columns(name, fn):
    g = payoff.Game(fn())
    Ahat, U, M, V, order = sparsify.factors(g)
    U2, M2, V2 = sparsify.postprocess(U, M, V)
    A = sparsify.dense_hand_major(g, order)
    assert np.abs(sparsify.product(Ahat, U2, M2, V2) - A).max() <= 1e-12 * np.abs(A).max()
    assert (np.diff(V2.tocsc().indptr) > 0).all()
    Md = M2.toarray()
    assert np.array_equal(np.diag(Md), np.ones(M2.shape[0])) and not np.triu(Md, 1).any()
    # rows of M keep at most two nonzeros (a substitution moves, never adds)
    assert (np.diff(M2.tocsr().indptr) <= 2).all()
    assert sparsify.size(Ahat, U2, M2, V2) <= sparsify.size(Ahat, U, M, V)


DISJOINT = [
    ("small_river", lambda: I.small_river(0)),
    ("small_river_3", lambda: I.small_river(3)),
    ("river_52", lambda: I.river_config(seed=3, n_keep=(160, 200), bet_fracs=(0.5, 1.0), max_raises=1,
                                        stack=100.0)),
]


@pytest.mark.parametrize("name,fn", DISJOINT)
def test_strength_order_makes_row_differences_sparse(name, fn):
    """Without shared cards each column of W runs -1, 0, +1 down the rows in
    strength order, so each column of Y = D W changes value at most twice
    after its first entry: nnz(Y) <= 3 N2, and Ahat vanishes."""
    g = payoff.Game(_disjoint(fn()))
    assert min(g.N) > 1 and not g.hm.share.any()
    Ahat, U, M, V, order = sparsify.factors(g)
    assert sparsify.size(Ahat) == 0
    F, S = sparsify.sequence_matrices(g)
    nS = int((S != 0).sum())
    N1, S1 = g.N[0], g.S[0]
    nY = sparsify.size(V[:, : N1 * S1]) // nS
    assert nY <= 3 * g.N[1]
    A = sparsify.dense_hand_major(g, order)
    assert np.abs(sparsify.product(Ahat, U, M, V) - A).max() <= 1e-12 * np.abs(A).max()


def test_payoff_nnz_counts_the_dense_matrix():
    for _, fn in RIVERS:
        g = payoff.Game(fn())
        assert sparsify.payoff_nnz(g) == int((g.dense_A() != 0).sum())


def test_sparsification_is_smaller_on_a_mid_size_river():
    """Table 1's size metric on a seeded river endgame of 300 x 517 hands."""
    d = I.river_config(seed=7, n_keep=(300, 517), bet_fracs=(0.33, 1.5), max_raises=2, stack=250.0)
    g = payoff.Game(d)
    Ahat, U, M, V, _ = sparsify.factors(g)
    U2, M2, V2 = sparsify.postprocess(U, M, V)
    nA = sparsify.payoff_nnz(g)
    before = sparsify.size(Ahat, U, M, V)
    after = sparsify.size(Ahat, U2, M2, V2)
    print(f"nnz(A) {nA}, Technique B {before}, postprocessed {after} ({nA / after:.1f}x smaller)")
    assert after <= before < nA


@pytest.mark.parametrize("seed", range(6))
def test_postprocessing_on_random_triangular_systems(seed):
    """Substitution with general coefficients and runs of consecutive zero
    columns of V: U M^-1 V^T is unchanged (dense solve on both sides)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    n, r, c = 12, 7, 5
    M = np.eye(n)
    for j in range(1, n):
        for i in rng.choice(j, size=min(j, 2), replace=False):
            M[j, i] = rng.normal()
    U = rng.normal(size=(r, n)) * (rng.random((r, n)) < 0.6)
    V = rng.normal(size=(c, n))
    zero = rng.random(n) < 0.45
    zero[[3, 4, 5]] = True                     # a run of three
    V[:, zero] = 0.0
    ref = U @ np.linalg.solve(M, V.T)
    U2, M2, V2 = sparsify.postprocess(sp.csc_matrix(U), sp.csr_matrix(M), sp.csc_matrix(V))
    assert M2.shape[0] == n - zero.sum()
    got = U2.toarray() @ np.linalg.solve(M2.toarray(), V2.toarray().T)
    assert np.abs(got - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
