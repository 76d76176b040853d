"""Pins of the hand evaluator, the suit isomorphism and the asymmetric betting
menu (the inputs of the paper's experimental setup in Section 5 and its
appendix on Libratus' betting abstraction).

* Five-card values: the exact category counts over all C(52, 5) hands and the
  7,462 distinct values (the standard enumeration of poker hands).
* Seven-card values: the best-of-21 evaluator against a direct evaluator of
  seven cards written independently below, on random deals.
* Suit isomorphism: 169 classes of the 1,326 starting hands; on boards, the
  class count equals Burnside's orbit count over the board's suit symmetries,
  and hands of one class have one value.
* Betting menu: a skeleton derived by hand, a menu that repeats one list
  reproduces Fig. 1, and menu games pass the payoff-matrix pins (deal
  enumeration, zero-sum LP values) and the RM+ convergence to the LP value.
"""
import os
from collections import Counter
from itertools import combinations

import numpy as np
import pytest

from paper_2112_03804_amd import handeval as H
from paper_2112_03804_amd import instances as I
from oracle import payoff, play, skeleton as sk, solver


# ---------------------------------------------------------------------------
# hand values
# ---------------------------------------------------------------------------

def test_five_card_category_counts_and_distinct_values():
    allc = np.array(list(combinations(range(52), 5)), dtype=np.int8)
    vals = np.concatenate([H.rank5(allc[i:i + 400000]) for i in range(0, len(allc), 400000)])
    cats = H.category(vals)
    want = [1302540, 1098240, 123552, 54912, 10200, 5108, 3744, 624, 40]
    assert len(allc) == 2598960
    assert np.bincount(cats, minlength=9).tolist() == want
    distinct = [len(np.unique(vals[cats == c])) for c in range(9)]
    assert distinct == [1277, 2860, 858, 858, 10, 1277, 156, 156, 10]
    assert len(np.unique(vals)) == 7462


def _card(s):
    r = "23456789TJQKA".index(s[0])
    return 4 * r + "cdhs".index(s[1])


def _v(*cards):
    return int(H.rank5(np.array([[_card(c) for c in cards]]))[0])


def test_five_card_orderings_by_hand():
    royal = _v("As", "Ks", "Qs", "Js", "Ts")
    sf_k = _v("Ks", "Qs", "Js", "Ts", "9s")
    steel_wheel = _v("5d", "4d", "3d", "2d", "Ad")
    quads = _v("Ah", "Ad", "Ac", "As", "2c")
    full = _v("Kh", "Kd", "Kc", "2s", "2c")
    flush = _v("Ah", "Jh", "9h", "5h", "3h")
    broadway = _v("Ah", "Kd", "Qc", "Js", "Tc")
    six_high = _v("6h", "5d", "4c", "3s", "2c")
    wheel = _v("5h", "4d", "3c", "2s", "Ac")
    trips = _v("7h", "7d", "7c", "Ks", "2c")
    two_pair = _v("Jh", "Jd", "4c", "4s", "9c")
    pair = _v("Th", "Td", "Ac", "8s", "3c")
    high = _v("Ah", "Qd", "9c", "6s", "3c")
    order = [royal, sf_k, steel_wheel, quads, full, flush, broadway, six_high, wheel, trips, two_pair, pair,
             high]
    assert all(a > b for a, b in zip(order, order[1:]))
    # suits never matter outside flushes; kickers decide within a category
    assert _v("Ah", "Kd", "Qc", "Js", "9c") == _v("Ac", "Kh", "Qd", "Jh", "9s")
    assert _v("Jh", "Jd", "4c", "4s", "9c") > _v("Jh", "Jd", "4c", "4s", "8c")
    assert _v("Jh", "Jd", "4c", "4s", "2c") > _v("Th", "Td", "9c", "9s", "Ac")


def _direct7(cards):
    """Value of seven cards found directly (best flush, straight, multiples
    and kickers of the seven), encoded as the evaluator's values."""
    ranks = [c >> 2 for c in cards]
    suits = [c & 3 for c in cards]

    def enc(cat, digits):
        if cat in (4, 8):
            return cat * 13 ** 5 + digits[0]
        return cat * 13 ** 5 + sum(d * 13 ** (4 - i) for i, d in enumerate(digits))

    def top_straight(rs):
        rs = set(rs)
        for top in range(12, 3, -1):
            if all(top - i in rs for i in range(5)):
                return top
        if {12, 0, 1, 2, 3} <= rs:
            return 3
        return None

    flush = None
    for s in range(4):
        rs = [r for r, t in zip(ranks, suits) if t == s]
        if len(rs) >= 5:
            t = top_straight(rs)
            if t is not None:
                return enc(8, [t])
            flush = sorted(rs, reverse=True)[:5]
    cnt = Counter(ranks)
    quads = sorted((r for r in cnt if cnt[r] == 4), reverse=True)
    trips = sorted((r for r in cnt if cnt[r] == 3), reverse=True)
    pairs = sorted((r for r in cnt if cnt[r] == 2), reverse=True)
    if quads:
        q = quads[0]
        return enc(7, [q] * 4 + [max(r for r in ranks if r != q)])
    if trips and (len(trips) > 1 or pairs):
        t = trips[0]
        return enc(6, [t] * 3 + [max(trips[1:] + pairs)] * 2)
    if flush:
        return enc(5, flush)
    t = top_straight(ranks)
    if t is not None:
        return enc(4, [t])
    if trips:
        t = trips[0]
        return enc(3, [t] * 3 + sorted((r for r in ranks if r != t), reverse=True)[:2])
    if len(pairs) >= 2:
        a, b = pairs[:2]
        return enc(2, [a, a, b, b, max(r for r in ranks if r not in (a, b))])
    if pairs:
        p = pairs[0]
        return enc(1, [p, p] + sorted((r for r in ranks if r != p), reverse=True)[:3])
    return enc(0, sorted(ranks, reverse=True)[:5])


def test_seven_card_values_match_a_direct_evaluator():
    rng = np.random.default_rng(5)
    seen = Counter()
    for _ in range(200):
        deal = rng.choice(52, size=5 + 2 * 23, replace=False)
        board, holes = deal[:5], deal[5:].reshape(-1, 2)
        got = H.rank7(holes, board)
        for h, v in zip(holes, got):
            want = _direct7(list(h) + list(board))
            assert v == want, (h, board, v, want)
            seen[int(v) // 13 ** 5] += 1
    # the random deals reach every category but the rarest
    assert all(seen[c] > 0 for c in range(8)), seen
    # made categories on purpose: straight flush, wheel, and a board that plays
    board = [_card(c) for c in ("9s", "Ts", "Js", "2d", "3c")]
    assert int(H.rank7(np.array([[_card("Qs"), _card("Ks")]]), board)[0]) == _direct7(
        [_card("Qs"), _card("Ks")] + board) == 8 * 13 ** 5 + 11
    board = [_card(c) for c in ("Ah", "Kh", "Qh", "Jh", "Th")]
    v = H.rank7(np.array([[_card("2c"), _card("3d")], [_card("4c"), _card("5d")]]), board)
    assert v[0] == v[1] == 8 * 13 ** 5 + 12


def test_strength_levels_are_dense_and_ordered():
    rng = np.random.default_rng(2)
    d = I.river_config(seed=9, strengths="eval")
    universe = np.concatenate(d.hands[:1])
    lev = H.strength_levels(universe, d.board)
    v = H.rank7(universe, d.board)
    assert lev.min() == 0 and set(np.unique(lev)) == set(range(lev.max() + 1))
    for i, j in rng.integers(0, len(v), size=(2000, 2)):
        assert (lev[i] > lev[j]) == (v[i] > v[j]) and (lev[i] == lev[j]) == (v[i] == v[j])
    assert np.array_equal(d.strength[0][0], lev)


# ---------------------------------------------------------------------------
# suit isomorphism
# ---------------------------------------------------------------------------

def test_starting_hands_fall_in_169_classes():
    hands = np.array(list(combinations(range(52), 2)))
    cls = H.suit_classes(hands)
    assert len(hands) == 1326 and cls.max() + 1 == 169
    # 13 pairs of 6 combos, 78 suited of 4, 78 offsuit of 12
    sizes = sorted(Counter(cls.tolist()).values())
    assert Counter(sizes) == {4: 78, 6: 13, 12: 78}


def _burnside(hands, board):
    syms = H.board_suit_symmetries(board)
    fixed = 0
    for pi in syms:
        for a, b in hands:
            ia, ib = 4 * (a >> 2) + pi[a & 3], 4 * (b >> 2) + pi[b & 3]
            fixed += {ia, ib} == {int(a), int(b)}
    assert fixed % len(syms) == 0
    return fixed // len(syms)


@pytest.mark.parametrize("board", [
    ("2c", "7d", "9h", "Js", "Ks"),      # two spades: swapping hearts and diamonds is no symmetry
    ("2s", "5s", "9s", "Js", "Ks"),      # monotone: the three other suits permute freely
    ("4c", "4d", "4h", "4s", "Ah"),      # quads: suits of 4 permute with the ace's suit fixed
    ("8c", "8d", "Ts", "Th", "3c"),
])
def test_board_classes_count_orbits(board):
    b = [_card(c) for c in board]
    hands = np.array([h for h in combinations(range(52), 2) if not set(h) & set(b)])
    cls = H.suit_classes(hands, b)
    assert cls.max() + 1 == _burnside(hands, b)
    v = H.rank7(hands, b)
    for c in range(cls.max() + 1):
        assert len(set(v[cls == c].tolist())) == 1


# ---------------------------------------------------------------------------
# asymmetric betting menu
# ---------------------------------------------------------------------------

MENU_GOLDEN = (((0.5,), (), (1.0,), (), ()), ((), (1.0,), (0.5,), (), ()))


def test_menu_skeleton_matches_hand_derivation(golden_dir):
    kinds = {"fold1": sk.FOLD1, "fold2": sk.FOLD2, "sd": sk.SHOWDOWN}
    want = {}
    with open(os.path.join(golden_dir, "menu_skeleton_leaves.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            path, kind, c1, c2 = line.split()
            want[tuple(path.split(","))] = (kinds[kind], float(c1), float(c2))
    root = sk.build_tree(1.0, (4.0, 4.0), [], 64, True, menu=MENU_GOLDEN)
    got = sk.leaf_paths(root)
    assert len(want) == 17 and got == want
    sf = sk.sequence_form(root)
    assert sf.n_seq == [13, 13] and [len(x) for x in sf.infosets] == [5, 5]


def test_menu_repeating_one_list_reproduces_fig1():
    plain = sk.build_tree(1875.0, (18125.0, 18125.0), [0.75], 1, True)
    menu = tuple(tuple((0.75,) for _ in range(5)) for _ in range(2))
    same = sk.build_tree(1875.0, (18125.0, 18125.0), [], 1, True, menu=menu)
    assert sk.leaf_paths(same) == sk.leaf_paths(plain)
    assert len(sk.leaf_paths(plain)) == 21


def test_libratus_menu_sizes():
    d = I.libratus_river(stack=1000.0)
    root = sk.build_tree(d.contrib, d.stack, list(d.bet_fracs), d.max_raises, d.allow_allin, menu=d.bet_menu)
    # the AI opens with 0.25 .. 8 x pot (8 x reaches past the stack: all-in)
    assert root.labels == ["check"] + ["bet"] * 6 + ["allin"]
    assert [ch.c[0] for ch in root.children] == [50, 75, 100, 150, 250, 450, 850, 1050]
    # the opponent answers a check with 0.5 / 0.75 / 1 x pot, raises a bet by 0.7 / 1.1
    assert [ch.c[1] for ch in root.children[0].children] == [50, 100, 125, 150, 1050]
    assert [ch.c[1] for ch in root.children[1].children] == [50, 75, 180, 240, 1050]
    # the AI re-raises a raise by 0.4 / 0.7 / 2
    assert [ch.c[0] for ch in root.children[1].children[2].children] == [75, 180, 324, 432, 900, 1050]
    swapped = I.libratus_river(stack=1000.0, ai=1)
    assert swapped.bet_menu == (d.bet_menu[1], d.bet_menu[0])


def _menu_small(seed=0, **kw):
    d = I.small_river(seed, **kw)
    d.bet_menu = (((0.5, 1.0), (), (1.0,), (0.5,), ()), ((), (0.75,), (0.5, 2.0), (), (1.0,)))
    d.max_raises = 64
    return d


MENU_GAMES = [
    ("menu_river", lambda: _menu_small(0, deck_size=9, n_board=2)),
    ("menu_river_1card", lambda: _menu_small(3, deck_size=8, n_board=1, cards_per_hand=1, stack=40.0)),
]


@pytest.mark.parametrize("name,desc_fn", MENU_GAMES)
def test_menu_games_pass_the_payoff_pins(name, desc_fn):
    desc = desc_fn()
    g = payoff.Game(desc)
    acts = [sorted(inf.n_actions for inf in g.sf.infosets[p]) for p in range(2)]
    assert acts[0] != acts[1]                      # the two players bet differently
    rng = np.random.default_rng(4)
    tp = [solver.Treeplex(g, p) for p in range(2)]
    b = [tp[p].behaviour_from_regret(rng.random((g.S[p], g.N[p]))) for p in range(2)]
    x = [tp[p].realization(b[p]) for p in range(2)]
    A = g.dense_A()
    ev = play.expected_payoff(desc, b[0], b[1])
    assert abs(ev - x[0].ravel() @ A @ x[1].ravel()) < 1e-10 * max(1.0, desc.contrib)
    v1, _ = solver.lp_value(g, player=0)
    v2, _ = solver.lp_value(g, player=1)
    assert abs(v1 + v2) < 1e-8
    # RM+ closes the gap around the LP value
    s = solver.RMPlus(g)
    gap = np.inf
    for it in range(4000):
        s.step()
        if it % 50 == 49:
            gap, br1, br2 = s.gap()
            assert br2 - 1e-9 <= v1 <= br1 + 1e-9
            if gap < 1e-3 * g.pot:
                break
    assert gap < 1e-3 * g.pot


def test_isomorphic_hands_have_equal_oracle_values():
    """With ranges drawn per class on a monotone board, the oracle's A y of a
    class-constant y is class-constant: the classes are symmetries of the
    whole game, not only of the strengths."""
    board = [4 * r + 3 for r in (0, 3, 7, 9, 11)]
    d = I.river_config(seed=2, board=board, strengths="eval", iso_ranges=True, bet_fracs=(0.5, 1.0),
                       max_raises=2)
    cls = H.suit_classes(d.hands[0], d.board)
    o = payoff.Game(d)
    rng = np.random.default_rng(3)
    y = rng.random((o.S[1], cls.max() + 1))[:, cls]
    Ay = o.matvec_A(y)
    norm = o.abs_row_sums().max()
    for c in range(cls.max() + 1):
        v = Ay[:, cls == c]
        assert np.abs(v - v[:, :1]).max() <= 1e-12 * norm
    # a board without suit symmetries leaves every hand its own class
    d2 = I.river_config(seed=1, strengths="eval")
    assert len(H.board_suit_symmetries(d2.board)) == 1
    assert H.suit_classes(d2.hands[0], d2.board).max() + 1 == len(d2.hands[0])
