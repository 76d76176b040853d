"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the values
printed in the paper (Fig. 1 table, the Appendix B worked example), a
published closed form (Kuhn poker's value -1/18), identities the paper states
(Prop. 1, eq. cf, the Technique-B factorization), the game value reached
from both players' LPs (zero-sum symmetry), expected payoffs obtained by
playing out every deal on the tree (independent of A), brute-force best
responses over pure strategies, and properties that hold for any game
(gap >= 0, symmetric games have value 0, chance sums to one).
"""
import itertools
import os

import numpy as np
import pytest

from paper_2112_03804_amd import instances as I
from oracle import payoff, play, skeleton as sk, solver


# ---------------------------------------------------------------------------
# Fig. 1 skeleton and its pot-contribution table (Section 3, Appendix B)
# ---------------------------------------------------------------------------

def _fig1_tree():
    return sk.build_tree(1875.0, (18125.0, 18125.0), [0.75], 1, True)


def test_fig1_pot_contribution_table(golden_dir):
    kinds = {"fold1": sk.FOLD1, "fold2": sk.FOLD2, "sd": sk.SHOWDOWN}
    rows = []
    with open(os.path.join(golden_dir, "fig1_pot_contributions.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            lab, path, kind, c1, c2 = line.split()
            rows.append((tuple(path.split(",")), kinds[kind], float(c1), float(c2)))
    leaves = sk.leaf_paths(_fig1_tree())
    assert len(rows) == 21 and len(leaves) == 21
    for path, kind, c1, c2 in rows:
        assert path in leaves, path
        k, a, b = leaves[path]
        assert k == kind, path
        # the figure rounds to one decimal
        assert abs(a - c1) <= 0.05 + 1e-12 and abs(b - c2) <= 0.05 + 1e-12, (path, a, b)


def test_fig1_sequence_counts():
    sf = sk.sequence_form(_fig1_tree())
    assert sf.n_seq == [16, 16]                       # sequences numbered 1..16 in Fig. 1
    assert [len(x) for x in sf.infosets] == [6, 6]
    assert len(sf.terminals) == 21


def test_fig1_state_D_worked_example(golden_dir):
    with open(os.path.join(golden_dir, "fig1_state_D.txt")) as f:
        vals = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")][0]
    root = _fig1_tree()
    d = root.children[root.labels.index(vals[0])]
    assert d.c == (float(vals[1]), float(vals[2]))
    assert d.s == (float(vals[3]), float(vals[4]))


def test_bet_base_is_pot_after_matching():
    # raise at D: match 4687.5, then 3/4 of 9375 -> 11718.75 (T in Fig. 1);
    # the other reading (3/4 of the pot before matching) would give 9609.375
    root = _fig1_tree()
    d = root.children[root.labels.index("bet")]
    k = d.children[d.labels.index("raise")]
    assert k.c[1] == 11718.75


# ---------------------------------------------------------------------------
# Game values
# ---------------------------------------------------------------------------

def test_kuhn_value_is_minus_one_eighteenth():
    g = payoff.Game(I.kuhn())
    v1, _ = solver.lp_value(g, player=0)
    v2, _ = solver.lp_value(g, player=1)
    assert abs(v1 - (-1.0 / 18.0)) < 1e-9
    assert abs(v2 - (1.0 / 18.0)) < 1e-9


@pytest.mark.parametrize("desc_fn", [
    I.tiny_config,
    lambda: I.small_river(0, deck_size=9, n_board=1, cards_per_hand=1, max_raises=1),
    lambda: I.small_river(3, deck_size=8, n_board=2, bet_fracs=(0.5,), max_raises=1),
])
def test_zero_sum_symmetry_of_lp_values(desc_fn):
    g = payoff.Game(desc_fn())
    v1, _ = solver.lp_value(g, player=0)
    v2, _ = solver.lp_value(g, player=1)
    assert abs(v1 + v2) < 1e-8


def test_symmetric_no_betting_game_has_value_zero():
    d = I.small_river(1, deck_size=10, n_board=2, bet_fracs=(), allow_allin=False,
                      zero_frac=0.0)
    d.range_[1] = d.range_[0].copy()
    g = payoff.Game(d)
    assert g.S == [1, 1]                                   # check, check
    v, _ = solver.lp_value(g)
    assert abs(v) < 1e-12
    x = np.ones((1, g.N[0]))
    assert abs(solver.value(g, x, x)) < 1e-12


# ---------------------------------------------------------------------------
# A against independent computations
# ---------------------------------------------------------------------------

GAMES = [
    ("kuhn", I.kuhn),
    ("tiny", I.tiny_config),
    ("river2card", lambda: I.small_river(0)),
    ("river_pruned", lambda: I.small_river(5, deck_size=11, n_keep=(20, 13))),
    ("turn1card", lambda: I.small_turn_river(0)),
    ("turn2card", lambda: I.small_turn_river(1, deck_size=9, n_board=3, cards_per_hand=2,
                                             bet_fracs=(0.5,), max_raises=0, stack=8.0)),
]


@pytest.mark.parametrize("name,desc_fn", GAMES)
def test_deal_enumeration_equals_xAy(name, desc_fn):
    desc = desc_fn()
    g = payoff.Game(desc)
    rng = np.random.default_rng(11)
    tp = [solver.Treeplex(g, p) for p in range(2)]
    for _ in range(2):
        b = [tp[p].behaviour_from_regret(rng.random((g.S[p], g.N[p])) * (rng.random((g.S[p], g.N[p])) < 0.8))
             for p in range(2)]
        x = [tp[p].realization(b[p]) for p in range(2)]
        ev = play.expected_payoff(desc, b[0], b[1])
        A = g.dense_A()
        assert abs(ev - x[0].ravel() @ A @ x[1].ravel()) < 1e-10 * max(1.0, desc.contrib)
        # the matrix-free forms evaluate the same sum
        assert np.allclose(g.matvec_A(x[1]).ravel(), A @ x[1].ravel(), atol=1e-13, rtol=0)
        assert np.allclose(g.matvec_AT(x[0]).ravel(), A.T @ x[0].ravel(), atol=1e-13, rtol=0)


def _hand_major(A, S1, N1, S2, N2):
    """Reorder rows/cols from (sigma, h) to (h, sigma) (the Kronecker order)."""
    r = np.arange(S1 * N1).reshape(S1, N1).T.ravel()
    c = np.arange(S2 * N2).reshape(S2, N2).T.ravel()
    return A[np.ix_(r, c)]


def _fold_showdown_matrices(g):
    S1, S2 = g.S
    F = np.zeros((S1, S2))
    Sm = np.zeros((S1, S2))
    for t in g.sf.terminals:
        if t.kind == sk.SHOWDOWN:
            Sm[t.seq1, t.seq2] += t.c1
        else:
            F[t.seq1, t.seq2] += t.u1
    return F, Sm


@pytest.mark.parametrize("seed,cph", [(0, 2), (2, 2), (4, 1)])
def test_prop1_kronecker_identity(seed, cph):
    """Prop. 1: A = C (x) F + (L1 W L2) (x) S with lambda_i = mu_i / sqrt(beta)
    and C = lambda1 lambda2^T - L1 H^x L2 (the printed mu1 mu2^T only agrees
    when beta = 1)."""
    d = I.small_river(seed, deck_size=10 if cph == 2 else 9, n_board=2, cards_per_hand=cph)
    g = payoff.Game(d)
    S1, S2 = g.S
    N1, N2 = g.N
    F, Sm = _fold_showdown_matrices(g)
    mu1, mu2 = g.hm.mu
    beta = g.hm.beta
    lam1, lam2 = mu1 / np.sqrt(beta), mu2 / np.sqrt(beta)
    Hx = np.zeros((N1, N2))
    W = np.zeros((N1, N2))
    for i in range(N1):
        for j in range(N2):
            a, b = set(d.hands[0][i].tolist()), set(d.hands[1][j].tolist())
            if a & b:
                Hx[i, j] = 1.0
            else:
                W[i, j] = np.sign(int(d.strength[0][0][i]) - int(d.strength[1][0][j]))
    C = np.outer(lam1, lam2) - np.diag(lam1) @ Hx @ np.diag(lam2)
    K = np.kron(C, F) + np.kron(np.diag(lam1) @ W @ np.diag(lam2), Sm)
    A = _hand_major(g.dense_A(), S1, N1, S2, N2)
    assert np.allclose(A, K, atol=1e-14, rtol=0)
    # eq. (cf): C (x) F = -(L1 H L2) (x) F + (lam1 (x) I)(lam2 (x) F^T)^T
    cf = -np.kron(np.diag(lam1) @ Hx @ np.diag(lam2), F) + \
        np.kron(lam1[:, None], np.eye(S1)) @ np.kron(lam2[:, None], F.T).T
    assert np.allclose(np.kron(C, F), cf, atol=1e-14, rtol=0)
    # Technique B: with hands in ascending strength order, Y = D W is sparse and
    # (L1 W L2) (x) S = (L1 (x) I)(D (x) I)^-1 ((L2 Y^T) (x) S^T)^T
    o1 = np.argsort(d.strength[0][0], kind="stable")
    o2 = np.argsort(d.strength[1][0], kind="stable")
    Ws = W[np.ix_(o1, o2)]
    L1s, L2s = np.diag(lam1[o1]), np.diag(lam2[o2])
    D = np.eye(N1) - np.eye(N1, k=-1)
    Y = D @ Ws
    lhs = np.kron(L1s @ Ws @ L2s, Sm)
    rhs = np.kron(L1s, np.eye(S1)) @ np.linalg.inv(np.kron(D, np.eye(S1))) @ \
        np.kron(L2s @ Y.T, Sm.T).T
    assert np.allclose(lhs, rhs, atol=1e-12, rtol=0)


def test_river_chance_sums_to_one():
    d = I.small_turn_river(2, deck_size=9, n_board=3, cards_per_hand=2)
    hm = payoff.HandModel(d)
    tot = sum(hm.river_prob(r) for r in range(len(hm.rivers)))
    assert np.allclose(tot[~hm.share], 1.0)


# ---------------------------------------------------------------------------
# Best response, gap and RM+
# ---------------------------------------------------------------------------

def _pure_plans(tp):
    """All pure sequence-form plans of a 1-hand-at-a-time treeplex (per hand)."""
    choices = [range(n) for (_, _, n) in tp.inf]
    for pick in itertools.product(*choices):
        b = np.zeros(tp.S)
        for (par, f, n), a in zip(tp.inf, pick):
            b[f + a] = 1.0
        x = np.zeros(tp.S)
        for (par, f, n) in tp.inf:
            x[f:f + n] = b[f:f + n] * (1.0 if par < 0 else x[par])
        yield x


def test_best_response_equals_brute_force_over_pure_strategies():
    g = payoff.Game(I.kuhn())
    rng = np.random.default_rng(5)
    tp = [solver.Treeplex(g, p) for p in range(2)]
    y = tp[1].realization(tp[1].behaviour_from_regret(rng.random((g.S[1], g.N[1]))))
    x = tp[0].realization(tp[0].behaviour_from_regret(rng.random((g.S[0], g.N[0]))))
    gap, br1, br2 = solver.saddle_gap(g, x, y)
    gy = g.matvec_A(y)           # per-hand payoffs are separable across hands
    best1 = sum(max(float(xp @ gy[:, h]) for xp in _pure_plans(tp[0])) for h in range(g.N[0]))
    gx = g.matvec_AT(x)
    best2 = sum(min(float(yp @ gx[:, h]) for yp in _pure_plans(tp[1])) for h in range(g.N[1]))
    assert abs(br1 - best1) < 1e-12 and abs(br2 - best2) < 1e-12
    assert gap >= 0
    v = solver.value(g, x, y)
    assert br2 - 1e-12 <= v <= br1 + 1e-12


def test_gap_vanishes_at_lp_equilibrium():
    g = payoff.Game(I.tiny_config())
    v1, x = solver.lp_value(g, player=0)
    v2, y = solver.lp_value(g, player=1)
    gap, br1, br2 = solver.saddle_gap(g, x, y)
    assert gap < 1e-8
    assert abs(br1 - v1) < 1e-8 and abs(br2 + v2) < 1e-8


def test_rmplus_single_update_closed_form():
    """One infoset, two actions, zero regrets, values (1, 3): the uniform
    strategy is worth 2, regrets become (0, 1), next strategy plays action 2."""
    g = payoff.Game(I.kuhn())
    tp = solver.Treeplex(g, 0)
    root = tp.inf[tp.roots[0]]
    f, n = root[1], root[2]
    gvec = np.zeros((g.S[0], 1))
    gvec[f, 0], gvec[f + 1, 0] = 1.0, 3.0
    tp1 = solver.Treeplex(g, 0)
    tp1.N = 1
    R = tp1.rmplus_update(np.zeros((g.S[0], 1)), gvec)
    assert R[f, 0] == 0.0 and R[f + 1, 0] == 1.0
    b = tp1.behaviour_from_regret(R)
    assert b[f, 0] == 0.0 and b[f + 1, 0] == 1.0


@pytest.mark.parametrize("desc_fn,target", [(I.kuhn, 1e-5), (I.tiny_config, 1e-5)])
def test_rmplus_reaches_lp_value(desc_fn, target):
    g = payoff.Game(desc_fn())
    v, _ = solver.lp_value(g)
    s = solver.RMPlus(g)
    gap = np.inf
    for it in range(20000):
        s.step()
        if it % 50 == 49:
            gap, br1, br2 = s.gap()
            assert gap >= -1e-12
            assert br2 - 1e-9 <= v <= br1 + 1e-9
            if gap < target * g.pot:
                break
    assert gap < target * g.pot


def test_gap_nonnegative_for_random_strategies():
    d = I.small_turn_river(3)
    g = payoff.Game(d)
    rng = np.random.default_rng(2)
    tp = [solver.Treeplex(g, p) for p in range(2)]
    for _ in range(3):
        x = tp[0].realization(tp[0].behaviour_from_regret(rng.random((g.S[0], g.N[0]))))
        y = tp[1].realization(tp[1].behaviour_from_regret(rng.random((g.S[1], g.N[1]))))
        gap, br1, br2 = solver.saddle_gap(g, x, y)
        assert gap >= 0
        v = solver.value(g, x, y)
        assert br2 - 1e-12 <= v <= br1 + 1e-12


def test_single_entries_match_matrix_free_product():
    d = I.small_turn_river(4, deck_size=9, n_board=3, cards_per_hand=2, stack=6.0)
    g = payoff.Game(d)
    rng = np.random.default_rng(3)
    y = rng.random((g.S[1], g.N[1]))
    x = rng.random((g.S[0], g.N[0]))
    Ay, ATx = g.matvec_A(y), g.matvec_AT(x)
    for _ in range(20):
        s, h = rng.integers(g.S[0]), rng.integers(g.N[0])
        assert abs(g.entry_A(y, s, h) - Ay[s, h]) < 1e-12
        s, h = rng.integers(g.S[1]), rng.integers(g.N[1])
        assert abs(g.entry_AT(x, s, h) - ATx[s, h]) < 1e-12


def test_dcfr_reaches_lp_value_and_beats_rmplus_on_tiny():
    """Discounted CFR (alpha 1.5, beta 0, gamma 2) converges to the LP value."""
    g = payoff.Game(I.tiny_config())
    v, _ = solver.lp_value(g)
    s = solver.RMPlus(g, kind="dcfr")
    for _ in range(2000):
        s.step()
    gap, br1, br2 = s.gap()
    assert gap >= -1e-12 and br2 - 1e-9 <= v <= br1 + 1e-9
    assert gap < 1e-4 * g.pot


def test_dcfr_single_update_closed_form():
    """Regrets (2, -2) at t = 1 discount to (1, -1) (factors 1/2 each), then
    the instantaneous regrets of values (1, 3) under strategy (1, 0) add
    (0, 2): (1, 1)."""
    g = payoff.Game(I.kuhn())
    tp = solver.Treeplex(g, 0)
    tp.N = 1
    f = tp.inf[tp.roots[0]][1]
    gvec = np.zeros((g.S[0], 1))
    gvec[f, 0], gvec[f + 1, 0] = 1.0, 3.0
    R = np.zeros((g.S[0], 1))
    R[f, 0], R[f + 1, 0] = 2.0, -2.0
    Rn = tp.dcfr_update(R, gvec, 1.0, 1.5, 0.0)
    assert Rn[f, 0] == 1.0 and Rn[f + 1, 0] == 1.0


# ---------------------------------------------------------------------------
# Tolerance scales: |A| |y|, row and column sums of |A|
# ---------------------------------------------------------------------------

ABS_GAMES = [
    ("tiny", I.tiny_config),
    ("river_pruned", lambda: I.small_river(5, deck_size=11, n_keep=(20, 13))),
    ("turn2card", lambda: I.small_turn_river(1, deck_size=9, n_board=3, cards_per_hand=2,
                                             bet_fracs=(0.5,), max_raises=0, stack=8.0)),
]


@pytest.mark.parametrize("name,desc_fn", ABS_GAMES)
def test_abs_scales_equal_dense_abs_products(name, desc_fn):
    """Every parity tolerance is scaled by |A| |v| or a row / column sum of
    |A|.  The matrix-free forms must equal the same products taken on the
    dense A (which deal enumeration pins); an inflated scale would loosen
    every bound silently."""
    g = payoff.Game(desc_fn())
    A = np.abs(g.dense_A())
    S1, S2 = g.S
    N1, N2 = g.N
    rng = np.random.default_rng(7)
    y = rng.standard_normal((S2, N2))
    x = rng.standard_normal((S1, N1))
    ref_y = (A @ np.abs(y).ravel()).reshape(S1, N1)
    ref_x = (A.T @ np.abs(x).ravel()).reshape(S2, N2)
    tol = 1e-13 * max(1.0, float(A.max()))
    assert np.allclose(payoff.abs_matvec_A(g, y), ref_y, atol=tol, rtol=1e-13)
    assert np.allclose(payoff.abs_matvec_AT(g, x), ref_x, atol=tol, rtol=1e-13)
    assert np.allclose(g.abs_row_sums().ravel(), A.sum(axis=1), atol=tol, rtol=1e-13)
    assert np.allclose(g.abs_col_sums().ravel(), A.sum(axis=0), atol=tol, rtol=1e-13)
    for _ in range(12):
        s, h = int(rng.integers(S1)), int(rng.integers(N1))
        assert abs(payoff.abs_entry_A(g, y, s, h) - ref_y[s, h]) <= tol + 1e-13 * ref_y[s, h]
        s, h = int(rng.integers(S2)), int(rng.integers(N2))
        assert abs(payoff.abs_entry_AT(g, x, s, h) - ref_x[s, h]) <= tol + 1e-13 * ref_x[s, h]


def test_kuhn_abs_row_and_column_sums_by_hand():
    """Kuhn poker (antes 1, a bet of 1, no raise): each card has two
    compatible opponent cards of deal probability 1/6.  Row sums of |A| per
    Player 1 sequence: check -> showdown for 1 (2/6); bet -> fold for 1 plus
    showdown for 2 (2/6 + 4/6 = 1); check-bet-fold -> 1 (1/3); check-bet-call
    -> 2 (2/3).  Column sums per Player 2 sequence: after a check, check (1/3)
    and bet (1/3 + 2/3); after a bet, fold (1/3) and call (2/3)."""
    g = payoff.Game(I.kuhn())
    rows = g.abs_row_sums()
    cols = g.abs_col_sums()
    tp1 = solver.Treeplex(g, 0)
    root = tp1.inf[tp1.roots[0]]
    lab1 = {}
    for i, I1 in enumerate(g.sf.infosets[0]):
        for a, lab in enumerate(I1.labels):
            lab1[I1.first_seq + a] = ("root" if I1.parent_seq < 0 else "after", lab)
    want1 = {("root", "check"): 1 / 3, ("root", "bet"): 1.0, ("after", "fold"): 1 / 3,
             ("after", "call"): 2 / 3}
    assert root[2] == 2
    for s, key in lab1.items():
        assert np.allclose(rows[s], want1[key], atol=1e-15), key
    want2 = {"check": 1 / 3, "bet": 1.0, "fold": 1 / 3, "call": 2 / 3}
    for I2 in g.sf.infosets[1]:
        for a, lab in enumerate(I2.labels):
            assert np.allclose(cols[I2.first_seq + a], want2[lab], atol=1e-15), lab
    assert abs(rows.max() - 1.0) < 1e-15 and abs(cols.max() - 1.0) < 1e-15


# ---------------------------------------------------------------------------
# A two-round skeleton (turn, chance node, river) derived by hand
# ---------------------------------------------------------------------------

def _walk_leaves(node, path, out):
    """(path, kind, c1, c2, runout) of every leaf, depth first; a chance node
    adds "/" to the path and continues into its river round."""
    if node.kind == "leaf":
        out.append((",".join(path), node.term_kind, node.runout, node.c[0], node.c[1]))
        return
    if node.kind == "chance":
        assert len(node.children) == 1
        _walk_leaves(node.children[0], path + ["/"], out)
        return
    for lab, ch in zip(node.labels, node.children):
        _walk_leaves(ch, path + [lab], out)


def test_two_round_skeleton_matches_hand_derivation(golden_dir):
    kinds = {"fold1": (sk.FOLD1, False), "fold2": (sk.FOLD2, False), "sd": (sk.SHOWDOWN, False),
             "ro": (sk.SHOWDOWN, True)}
    want = []
    with open(os.path.join(golden_dir, "two_round_leaves.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            path, kind, c1, c2 = line.split()
            k, ro = kinds[kind]
            want.append((path, k, ro, float(c1), float(c2)))
    root = sk.build_tree(1.0, (4.0, 4.0), [0.5], 0, True, two_rounds=True)
    got = []
    _walk_leaves(root, [], got)
    assert len(got) == len(want) == 49
    for g_, w_ in zip(got, want):
        assert g_ == w_, (g_, w_)
    # the sequence form expands each chance node once per river card: the 10
    # turn leaves stay, the 3 river rounds of 13 leaves repeat per card
    sf = sk.sequence_form(root, n_rivers=2)
    assert len(sf.terminals) == 10 + 3 * 13 * 2
    first = [t for t in sf.terminals if t.board < 0]
    assert len(first) == 10
    assert sum(t.runout for t in first) == 4 and not any(t.runout for t in sf.terminals if t.board >= 0)
    for r in range(2):
        assert sum(t.board == r for t in sf.terminals) == 39
    # the river rounds under different cards share sizes but not sequences
    r0 = sorted((t.seq1, t.seq2) for t in sf.terminals if t.board == 0)
    r1 = sorted((t.seq1, t.seq2) for t in sf.terminals if t.board == 1)
    assert not set(r0) & set(r1)


def test_tiny_game_value_is_minus_one_thirteenth():
    """The 13-card game (antes 1, one pot-sized bet, at most one raise, no
    all-in): both players' LPs give Player 1 the value -1/13."""
    g = payoff.Game(I.tiny_config())
    v1, _ = solver.lp_value(g, player=0)
    v2, _ = solver.lp_value(g, player=1)
    assert abs(v1 - (-1.0 / 13.0)) < 1e-9
    assert abs(v2 - (1.0 / 13.0)) < 1e-9
