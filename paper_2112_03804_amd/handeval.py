"""Texas hold'em hand values and suit isomorphism (input generation only).

The paper's endgames are river (and turn) situations of no-limit hold'em,
whose hand strengths come from the game's hand ranking, with hands that are
equal up to a permutation of suits collapsed (Section 5, experimental setup).
This module computes those inputs for synthetic boards: it holds none of the
method's arithmetic (no payoffs, no betting tree, no deal distribution), so
the CPU oracle and the GPU library can both consume its strengths.

Cards are ``0 .. 51`` with card = 4 * rank + suit, rank 0 = deuce ..
12 = ace.  A hand value is an integer; a larger value wins, equal values
tie.  Five-card values are

    category * 13**5 + (ranks ordered by multiplicity, then rank, descending),

read as base-13 digits, with categories 0 high card, 1 pair, 2 two pair,
3 three of a kind, 4 straight, 5 flush, 6 full house, 7 four of a kind,
8 straight flush; a straight is valued by its top card alone (the wheel
A-2-3-4-5 tops at five).  A seven-card value is the best of its 21
five-card subsets.
"""
from __future__ import annotations

from itertools import combinations, permutations
from typing import Sequence

import numpy as np

__all__ = ["CATEGORIES", "rank5", "rank7", "category", "strength_levels", "suit_classes",
           "board_suit_symmetries"]

CATEGORIES = ("high card", "pair", "two pair", "three of a kind", "straight", "flush",
              "full house", "four of a kind", "straight flush")
_B5 = 13 ** 5
_POW = np.array([13 ** 4, 13 ** 3, 13 ** 2, 13, 1], dtype=np.int64)
_SUBSETS7 = np.array(list(combinations(range(7), 5)), dtype=np.int64)   # 21 x 5


def rank5(cards: np.ndarray) -> np.ndarray:
    """Values of five-card hands: ``cards`` int array [..., 5] -> int64 [...]."""
    c = np.asarray(cards, dtype=np.int64)
    shape = c.shape[:-1]
    c = c.reshape(-1, 5)
    r, s = c >> 2, c & 3
    n = len(c)
    cnt = np.zeros((n, 13), dtype=np.int64)
    for k in range(5):
        cnt[np.arange(n), r[:, k]] += 1
    # each card's key: multiplicity first, then rank; the five cards in
    # descending key order give the tiebreak digits
    key = cnt[np.arange(n)[:, None], r] * 16 + r
    order = np.argsort(-key, axis=1, kind="stable")
    digits = np.take_along_axis(r, order, axis=1)
    tiebreak = digits @ _POW
    mult = np.sort(cnt, axis=1)[:, ::-1]
    top, second = mult[:, 0], mult[:, 1]
    flush = (s == s[:, :1]).all(axis=1)
    distinct = top == 1
    rs = np.sort(r, axis=1)
    plain_straight = distinct & (rs[:, 4] - rs[:, 0] == 4)
    wheel = distinct & (rs[:, 4] == 12) & (rs[:, 3] == 3)
    straight = plain_straight | wheel
    high = np.where(wheel, 3, rs[:, 4])
    cat = np.zeros(n, dtype=np.int64)
    cat[(top == 2) & (second == 1)] = 1
    cat[(top == 2) & (second == 2)] = 2
    cat[(top == 3) & (second == 1)] = 3
    cat[straight] = 4
    cat[flush] = 5
    cat[(top == 3) & (second == 2)] = 6
    cat[top == 4] = 7
    cat[straight & flush] = 8
    val = cat * _B5 + np.where(straight, high, tiebreak)
    return val.reshape(shape)


def rank7(hole: np.ndarray, board: Sequence[int]) -> np.ndarray:
    """Best five-card value of each hand's hole cards with a five-card board:
    ``hole`` int array [n, 2] -> int64 [n]."""
    h = np.asarray(hole, dtype=np.int64).reshape(-1, 2)
    b = np.asarray(board, dtype=np.int64).reshape(-1)
    if len(b) != 5:
        raise ValueError("a seven-card value needs a five-card board")
    seven = np.concatenate([h, np.broadcast_to(b, (len(h), 5))], axis=1)   # n x 7
    return rank5(seven[:, _SUBSETS7]).max(axis=1)


def category(values: np.ndarray) -> np.ndarray:
    """Category index (see CATEGORIES) of hand values."""
    return np.asarray(values, dtype=np.int64) // _B5


def strength_levels(hole: np.ndarray, board: Sequence[int]) -> np.ndarray:
    """Dense strength levels of hands on a final board: 0 for the weakest
    value present, equal values equal levels (int32 [n])."""
    v = rank7(hole, board)
    _, lev = np.unique(v, return_inverse=True)
    return lev.astype(np.int32).reshape(-1)


def board_suit_symmetries(board: Sequence[int]) -> list:
    """The permutations of the four suits that map the board onto itself
    (as a set of cards); each is a tuple pi with suit s -> pi[s]."""
    b = sorted(int(x) for x in board)
    out = []
    for pi in permutations(range(4)):
        if sorted(4 * (c >> 2) + pi[c & 3] for c in b) == b:
            out.append(pi)
    return out


def suit_classes(hands: np.ndarray, board: Sequence[int] = ()) -> np.ndarray:
    """Isomorphism class of each hand: hands that one suit permutation
    fixing the board maps onto each other share a class (the smallest
    sorted image of the hand under those permutations names it).  Returns
    int64 [n] class ids, numbered in order of first appearance."""
    h = np.asarray(hands, dtype=np.int64)
    syms = board_suit_symmetries(board)
    canon = None
    for pi in syms:
        p = np.asarray(pi, dtype=np.int64)
        img = np.sort(4 * (h >> 2) + p[h & 3], axis=1)
        k = img[:, 0] * 64 + (img[:, 1] if h.shape[1] > 1 else 0)
        canon = k if canon is None else np.minimum(canon, k)
    _, first, inv = np.unique(canon, return_index=True, return_inverse=True)
    # renumber by first appearance
    order = np.argsort(first, kind="stable")
    rename = np.empty_like(order)
    rename[order] = np.arange(len(order))
    return rename[inv].reshape(-1)
