"""Betting skeleton and sequence form (oracle; test infrastructure only).

Rules followed (paper, Appendix A "Betting rounds", and the caption of Fig. 1):

* A player whose pot contribution is not below the opponent's may check or
  bet; a player facing a larger contribution may fold, call, or raise.
* A bet or raise first matches the opponent's contribution and then adds a
  fraction of the cumulative pot *after matching* (Fig. 1 caption; the
  worked example of state D in Appendix B: 3/4 x (1875 x 2) = 2812.5).
* Nobody may put in more than the opponent can still match; putting in that
  maximum is the all-in.  A bet or raise that reaches it is the all-in.
* The round ends when a player folds, a player calls, or both check.
* ``max_raises`` counts raises after the opening bet of a round (Fig. 1:
  after a bet and one raise only fold / call / all-in remain).  The all-in is
  offered whenever it exceeds a call, also past the raise cap (Fig. 1, nodes
  K and O).
* Action order inside a decision node: fold, check/call, bets and raises by
  ascending size, all-in.
* Bet sizes are one list for every decision, or a menu per player and
  situation, as in the asymmetric abstraction of the paper's appendix on the
  betting abstraction (the two players draw on different lists, and each
  player's list depends on whether it opens the round, answers a check, or
  faces a bet, one raise, or more raises).

Payoffs are Player 1's (Section 3): a fold costs the folder its contribution,
a showdown moves the (equal) contribution of the loser to the winner.

A turn + river endgame (Section 3, last paragraph) is a betting round whose
non-fold ends lead to a chance node that reveals the river card, followed by
a river betting round; if a player is all-in at the end of the turn round the
cards are simply run out to a showdown.

Sequence form: every decision node of the skeleton is one infoset of the
acting player (betting is public; the private hand is the Kronecker factor).
Sequences are numbered per player in depth-first preorder: when a decision
node is first visited all its actions receive consecutive ids, then the
children are visited in action order; a chance node visits its river cards
in the order given.  The empty sequence is not numbered (parent id -1).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

EPS = 1e-9

FOLD1, FOLD2, SHOWDOWN = 0, 1, 2   # terminal kinds (who folded / showdown)


@dataclasses.dataclass
class Terminal:
    seq1: int           # Player 1's last sequence (-1 = empty)
    seq2: int           # Player 2's last sequence (-1 = empty)
    kind: int           # FOLD1, FOLD2 or SHOWDOWN
    c1: float           # pot contributions at the leaf
    c2: float
    board: int          # -1: first-round (turn or river endgame); r >= 0: river card index
    runout: bool        # showdown reached all-in before the river card: averaged over rivers

    @property
    def u1(self) -> float:
        """Player 1's payoff at a fold leaf, or the stake at a showdown."""
        if self.kind == FOLD1:
            return -self.c1
        if self.kind == FOLD2:
            return self.c2
        return self.c1


@dataclasses.dataclass
class Infoset:
    player: int         # 0 or 1
    parent_seq: int     # -1 = empty sequence
    first_seq: int
    n_actions: int
    labels: List[str]
    board: int          # -1 first round, r >= 0 river card index


@dataclasses.dataclass
class Node:
    kind: str                          # 'p0', 'p1', 'leaf', 'chance'
    c: tuple                           # contributions (c1, c2)
    s: tuple                           # stacks behind (s1, s2)
    labels: List[str] = dataclasses.field(default_factory=list)
    children: List["Node"] = dataclasses.field(default_factory=list)
    term_kind: int = -1
    runout: bool = False
    name: str = ""


def _snap(x: float) -> float:
    return 0.0 if abs(x) < EPS else x


# situations of a betting menu
OPEN, AFTER_CHECK, FACING_BET, FACING_RAISE, FACING_RERAISE = range(5)


def situation(facing, raises, checked):
    """Situation of a decision for the betting menu: opening the round,
    answering a check, facing a bet, one raise, or two and more raises."""
    if not facing:
        return AFTER_CHECK if checked else OPEN
    return FACING_BET + min(raises, 2)


def _round(c, s, fracs, max_raises, allow_allin, last_round, menu=None):
    """Build one betting round starting with Player 1 to act, contributions c
    and stacks s.  Round ends become 'leaf' (showdown) when last_round, else
    'chance' (next round) unless a player is all-in (then a run-out leaf).
    menu[p][k]: player p's bet fractions in situation k (None: fracs)."""

    def end_of_round(c, s):
        if last_round:
            return Node('leaf', c, s, term_kind=SHOWDOWN)
        if s[0] <= EPS or s[1] <= EPS:
            return Node('leaf', c, s, term_kind=SHOWDOWN, runout=True)
        return Node('chance', c, s)

    def node(p, c, s, facing, raises, checked):
        o = 1 - p
        ci, cj = c[p], c[o]
        allin_to = min(ci + s[p], cj + s[o])      # no more than the opponent can match
        labels, kids = [], []

        def put(target):
            nc = list(c)
            ns = list(s)
            nc[p] = target
            ns[p] = _snap(s[p] - (target - ci))
            return tuple(nc), tuple(ns)

        if facing:
            labels.append('fold')
            kids.append(Node('leaf', c, s, term_kind=(FOLD1 if p == 0 else FOLD2)))
            nc, ns = put(cj)
            labels.append('call')
            kids.append(end_of_round(nc, ns))
        else:
            labels.append('check')
            if checked:
                kids.append(end_of_round(c, s))
            else:
                kids.append(node(o, c, s, False, raises, True))
        # bets / raises ascending, then all-in
        can_grow = allin_to > cj + EPS
        targets = []
        sizes = fracs if menu is None else sorted(menu[p][situation(facing, raises, checked)])
        if can_grow and (not facing or raises < max_raises):
            for f in sizes:
                t = cj + f * 2.0 * cj
                if t >= allin_to - EPS:
                    t = allin_to
                if targets and abs(targets[-1] - t) <= EPS:
                    continue
                targets.append(t)
        if can_grow and allow_allin and (not targets or abs(targets[-1] - allin_to) > EPS):
            targets.append(allin_to)
        for t in targets:
            is_allin = abs(t - allin_to) <= EPS
            nc, ns = put(allin_to if is_allin else t)
            labels.append('allin' if is_allin else ('raise' if facing else 'bet'))
            kids.append(node(o, nc, ns, True, raises + (1 if facing else 0), False))
        return Node('p%d' % p, c, s, labels=labels, children=kids)

    return node(0, tuple(c), tuple(s), False, 0, False)


def build_tree(contrib, stacks, fracs, max_raises, allow_allin, two_rounds=False, menu=None):
    """Skeleton of a river endgame (two_rounds=False) or of a turn + river
    endgame, whose chance nodes get river-round children later (the river
    round depends only on the contributions and stacks at the chance node).
    menu: per-player, per-situation bet fractions replacing fracs."""
    root = _round((contrib, contrib), tuple(stacks), list(fracs), max_raises,
                  allow_allin, last_round=not two_rounds, menu=menu)
    if two_rounds:
        def attach(n):
            if n.kind == 'chance':
                n.children = [_round(n.c, n.s, list(fracs), max_raises, allow_allin,
                                     last_round=True, menu=menu)]
                return
            for ch in n.children:
                attach(ch)
        attach(root)
    return root


@dataclasses.dataclass
class SequenceForm:
    n_seq: List[int]
    infosets: List[List[Infoset]]
    seq_infoset: List[List[int]]       # infoset owning each sequence
    terminals: List[Terminal]
    n_boards: int                      # rivers (0 for a river endgame)

    def root_infosets(self, p):
        return [i for i, I in enumerate(self.infosets[p]) if I.parent_seq < 0]


def sequence_form(root: Node, n_rivers: int = 0) -> SequenceForm:
    """Number sequences and infosets in depth-first preorder; collect terminals.
    A chance node expands into one river subtree per river card index."""
    n_seq = [0, 0]
    infosets: List[List[Infoset]] = [[], []]
    seq_inf: List[List[int]] = [[], []]
    terms: List[Terminal] = []

    def visit(n: Node, last, board):
        if n.kind == 'leaf':
            terms.append(Terminal(last[0], last[1], n.term_kind, n.c[0], n.c[1],
                                  board, n.runout))
            return
        if n.kind == 'chance':
            sub = n.children[0]
            for r in range(n_rivers):
                visit(sub, last, r)
            return
        p = 0 if n.kind == 'p0' else 1
        first = n_seq[p]
        iid = len(infosets[p])
        infosets[p].append(Infoset(p, last[p], first, len(n.children), list(n.labels), board))
        n_seq[p] += len(n.children)
        seq_inf[p].extend([iid] * len(n.children))
        for a, ch in enumerate(n.children):
            nl = list(last)
            nl[p] = first + a
            visit(ch, tuple(nl), board)

    visit(root, (-1, -1), -1)
    return SequenceForm(n_seq, infosets, seq_inf, terms, n_rivers)


def leaf_contributions(root: Node):
    """(c1, c2) of every leaf in depth-first order (for the Fig. 1 table)."""
    out = []

    def visit(n):
        if n.kind == 'leaf':
            out.append((n.term_kind, n.c[0], n.c[1]))
        for ch in n.children:
            visit(ch)
    visit(root)
    return out


def from_desc(desc) -> SequenceForm:
    """Sequence form of a GameDesc-like instance."""
    two = len(desc.river_cards) > 0
    root = build_tree(desc.contrib, desc.stack, list(desc.bet_fracs), int(desc.max_raises),
                      bool(desc.allow_allin), two_rounds=two, menu=getattr(desc, "bet_menu", None))
    return sequence_form(root, len(desc.river_cards))


def leaf_paths(root: Node):
    """{action path: (kind, c1, c2)} for every leaf of a one-round skeleton."""
    out = {}

    def visit(n, path):
        if n.kind == 'leaf':
            out[tuple(path)] = (n.term_kind, n.c[0], n.c[1])
            return
        for lab, ch in zip(n.labels, n.children):
            visit(ch, path + [lab])
    visit(root, [])
    return out
