"""Expected payoff by playing out every deal on the game tree (oracle; test
infrastructure only).

Independent of the payoff matrix: it walks the betting skeleton of
``skeleton.build_tree`` once per deal (h1, h2) with each player's behavioural
strategy for that hand, and weighs the leaf payoff by the deal probability
(Section 3: mu1 mu2 on hand pairs that share no card, normalized) and, for a
turn + river endgame, by the river card's probability (uniform over the cards
left).  Showdowns compare the two strengths on the final board directly.

Behavioural strategies are given per sequence: b[p][sigma, h] is the
probability of the action ending sigma at its decision node for hand h.  The
walk numbers decision nodes in the same depth-first order the sequence form
documents (all actions of a node get consecutive ids, children in action
order, river cards in list order).
"""
from __future__ import annotations

import numpy as np

from . import skeleton as sk


def expected_payoff(desc, b1, b2):
    root = sk.build_tree(desc.contrib, desc.stack, list(desc.bet_fracs), int(desc.max_raises),
                         bool(desc.allow_allin), two_rounds=len(desc.river_cards) > 0,
                         menu=getattr(desc, "bet_menu", None))
    hands = [np.asarray(h, dtype=np.int64) for h in desc.hands]
    mu = [np.asarray(r, dtype=np.float64) for r in desc.range_]
    rivers = [int(r) for r in desc.river_cards]
    left = desc.deck_size - len(desc.board) - 2 * desc.cards_per_hand
    strat = [b1, b2]

    # number each decision node's actions exactly once, in depth-first preorder
    ids = {}
    counter = [0, 0]

    def number(n, board):
        if n.kind == 'leaf':
            return
        if n.kind == 'chance':
            for r in range(len(rivers)):
                number(n.children[0], r)
            return
        p = 0 if n.kind == 'p0' else 1
        ids[(id(n), board)] = counter[p]
        counter[p] += len(n.children)
        for ch in n.children:
            number(ch, board)
    number(root, -1)

    def outcome(h1, h2, board):
        b = 0 if board < 0 else board
        s1 = int(desc.strength[0][b][h1])
        s2 = int(desc.strength[1][b][h2])
        return float(np.sign(s1 - s2))

    def walk(n, h1, h2, board):
        if n.kind == 'leaf':
            if n.term_kind == sk.FOLD1:
                return -n.c[0]
            if n.term_kind == sk.FOLD2:
                return n.c[1]
            if n.runout:
                cards = set(hands[0][h1].tolist()) | set(hands[1][h2].tolist())
                acc = 0.0
                for r, card in enumerate(rivers):
                    if card not in cards:
                        acc += outcome(h1, h2, r) / left
                return acc * n.c[0]
            return n.c[0] * outcome(h1, h2, board)
        if n.kind == 'chance':
            cards = set(hands[0][h1].tolist()) | set(hands[1][h2].tolist())
            acc = 0.0
            for r, card in enumerate(rivers):
                if card not in cards:
                    acc += walk(n.children[0], h1, h2, r) / left
            return acc
        p = 0 if n.kind == 'p0' else 1
        first = ids[(id(n), board)]
        h = h1 if p == 0 else h2
        acc = 0.0
        for a, ch in enumerate(n.children):
            pr = strat[p][first + a, h]
            if pr != 0.0:
                acc += pr * walk(ch, h1, h2, board)
        return acc

    total, norm = 0.0, 0.0
    for h1 in range(len(hands[0])):
        for h2 in range(len(hands[1])):
            if set(hands[0][h1].tolist()) & set(hands[1][h2].tolist()):
                continue
            w = mu[0][h1] * mu[1][h2]
            norm += w
            if w != 0.0:
                total += w * walk(root, h1, h2, -1)
    return total / norm
