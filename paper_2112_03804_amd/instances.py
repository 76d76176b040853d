"""Seeded synthetic endgame instances.

This module only draws *inputs*: decks, boards, private-hand lists, per-board
hand strengths, belief distributions (ranges), pot/stack sizes and betting
abstractions.  It holds none of the method's arithmetic (no deal
distribution, no payoffs, no betting tree) so that the CPU oracle and the GPU
library can both consume the very same instance without sharing any
algorithmic code.

An instance describes a river endgame (Section 3 of the paper: board B,
stacks (s1, s2), initial pot contribution c, beliefs mu_1, mu_2) or a
turn-plus-river endgame (a betting round on a 4-card board, then a chance
node revealing one more public card, then a river betting round).  The real
endgames of the paper's experiments are not available; the generators below
stand in for them with the shapes described in the accompanying design notes.

Card ids are ``0 .. deck_size-1``.  For the 52-card deck, card = 4*rank + suit.
A two-card hand is stored as ``(lo, hi)`` with ``lo < hi``; hand lists are in
lexicographic (lo, hi) order unless stated otherwise.
"""
from __future__ import annotations

import dataclasses
from itertools import combinations
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "GameDesc",
    "tiny_config",
    "kuhn",
    "river_config",
    "turn_river_config",
    "batched_configs",
    "small_river",
    "small_turn_river",
    "libratus_menu",
    "libratus_river",
    "config",
    "to_dict",
    "from_dict",
    "save_json",
    "load_json",
]


@dataclasses.dataclass
class GameDesc:
    """Plain-array description of one endgame instance.

    Attributes mirror the C descriptor of the library one-to-one.

    deck_size, cards_per_hand : deck size and private cards per hand (1 or 2).
    board           : uint8[n_board] public cards already dealt.
    river_cards     : uint8[n_river] cards the chance node may reveal after the
                      first betting round (empty for a river endgame).
    hands[p]        : uint8[n_hands[p], cards_per_hand] player p's hand list.
    strength[p]     : int32[n_boards, n_hands[p]] hand strength on each final
                      board (n_boards = max(1, n_river)); higher wins, equal
                      ties.  Entries for hands that collide with a river card
                      are ignored.
    range_[p]       : float64[n_hands[p]] belief weights (any positive scale).
    contrib         : pot contribution of each player before the endgame.
    stack           : (s1, s2) chips behind.
    bet_fracs       : bet/raise sizes as fractions of the pot after matching.
    max_raises      : raises allowed after the opening bet of a round.
    allow_allin     : whether an all-in action is offered.
    bet_menu        : None, or per player five tuples of fractions that
                      replace bet_fracs by situation: opening the round,
                      answering a check, facing a bet, facing one raise,
                      facing two or more raises (an asymmetric abstraction).
    """

    deck_size: int
    cards_per_hand: int
    board: np.ndarray
    river_cards: np.ndarray
    hands: List[np.ndarray]
    strength: List[np.ndarray]
    range_: List[np.ndarray]
    contrib: float
    stack: tuple
    bet_fracs: np.ndarray
    max_raises: int
    allow_allin: bool
    name: str = ""
    bet_menu: Optional[tuple] = None

    @property
    def n_hands(self):
        return (len(self.hands[0]), len(self.hands[1]))

    @property
    def n_river(self):
        return len(self.river_cards)

    @property
    def pot(self):
        return 2.0 * self.contrib

    def copy(self) -> "GameDesc":
        return dataclasses.replace(
            self,
            board=self.board.copy(),
            river_cards=self.river_cards.copy(),
            hands=[h.copy() for h in self.hands],
            strength=[s.copy() for s in self.strength],
            range_=[r.copy() for r in self.range_],
            bet_fracs=self.bet_fracs.copy(),
        )


# --------------------------------------------------------------------------
# helpers (input drawing only)
# --------------------------------------------------------------------------

def _all_hands(deck_size: int, cards_per_hand: int, dead: Sequence[int]) -> np.ndarray:
    live = [c for c in range(deck_size) if c not in set(int(d) for d in dead)]
    if cards_per_hand == 1:
        return np.array([[c] for c in live], dtype=np.uint8).reshape(-1, 1)
    return np.array(list(combinations(live, 2)), dtype=np.uint8).reshape(-1, 2)


def _hand_keys(hands: np.ndarray, deck_size: int) -> np.ndarray:
    """Integer key of each hand (for looking hands up across lists)."""
    h = hands.astype(np.int64)
    if h.shape[1] == 1:
        return h[:, 0]
    return h[:, 0] * deck_size + h[:, 1]


def _strength_with_ties(n: int, rng: np.random.Generator, tie_p: float) -> np.ndarray:
    """A random total order over n items in which each item (in order) joins
    its predecessor's tie group with probability tie_p.  Returns int32 levels."""
    order = rng.permutation(n)
    joins = rng.random(n) < tie_p
    joins[0] = False
    level = np.cumsum(~joins) - 1
    s = np.empty(n, dtype=np.int32)
    s[order] = level.astype(np.int32)
    return s


def _dirichlet_range(n: int, rng: np.random.Generator, zero_frac: float) -> np.ndarray:
    w = rng.dirichlet(np.ones(n))
    if zero_frac > 0:
        k = int(round(zero_frac * n))
        w[rng.choice(n, size=k, replace=False)] = 0.0
    return w.astype(np.float64)


def _board_strengths(universe: np.ndarray, board: np.ndarray, deck_size: int, rng: np.random.Generator,
                     tie_p: float, strengths: str) -> np.ndarray:
    """Strength levels of the hands in universe on a final board: a seeded
    random order with ties ("random") or the hold'em hand ranking ("eval",
    52-card deck and two-card hands only)."""
    if strengths == "random":
        return _strength_with_ties(len(universe), rng, tie_p)
    if strengths == "eval":
        if deck_size != 52 or universe.shape[1] != 2 or len(board) != 5:
            raise ValueError("hand-ranking strengths need a 52-card deck, two-card hands and a 5-card board")
        from . import handeval
        return handeval.strength_levels(universe, board)
    raise ValueError(f"unknown strengths {strengths!r}")


def _lookup(universe_keys: np.ndarray, keys: np.ndarray) -> np.ndarray:
    pos = {int(k): i for i, k in enumerate(universe_keys)}
    return np.array([pos[int(k)] for k in keys], dtype=np.int64)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def tiny_config(seed: int = 0) -> GameDesc:
    """13-card deck, no board, one private card each, strength = card rank,
    antes of 1, one pot-sized bet, at most one raise, no all-in, deep stacks,
    uniform deals."""
    del seed
    hands = np.arange(13, dtype=np.uint8).reshape(-1, 1)
    s = np.arange(13, dtype=np.int32).reshape(1, -1)
    return GameDesc(
        deck_size=13, cards_per_hand=1,
        board=np.zeros(0, np.uint8), river_cards=np.zeros(0, np.uint8),
        hands=[hands.copy(), hands.copy()], strength=[s.copy(), s.copy()],
        range_=[np.ones(13), np.ones(13)],
        contrib=1.0, stack=(1e6, 1e6), bet_fracs=np.array([1.0]),
        max_raises=1, allow_allin=False, name="tiny13")


def kuhn() -> GameDesc:
    """Kuhn's simplified poker: 3 cards, ante 1, a single bet of half the pot,
    no raise, uniform deals."""
    hands = np.arange(3, dtype=np.uint8).reshape(-1, 1)
    s = np.arange(3, dtype=np.int32).reshape(1, -1)
    return GameDesc(
        deck_size=3, cards_per_hand=1,
        board=np.zeros(0, np.uint8), river_cards=np.zeros(0, np.uint8),
        hands=[hands.copy(), hands.copy()], strength=[s.copy(), s.copy()],
        range_=[np.ones(3), np.ones(3)],
        contrib=1.0, stack=(1e6, 1e6), bet_fracs=np.array([0.5]),
        max_raises=0, allow_allin=False, name="kuhn")


def river_config(seed: int = 1, deck_size: int = 52, bet_fracs=(0.5, 1.0, 2.0),
                 max_raises: int = 3, pot: float = 100.0, stack: float = 400.0,
                 zero_frac: float = 0.30, tie_p: float = 0.05,
                 n_keep: Optional[Sequence[int]] = None,
                 name: str = "river", strengths: str = "random",
                 bet_menu: Optional[tuple] = None, board: Optional[Sequence[int]] = None,
                 iso_ranges: bool = False) -> GameDesc:
    """River endgame: 5 board cards (seeded, or the given board), two-card
    hands, seeded strengths (random order with ~tie_p tie groups, or the
    hand ranking with strengths="eval"), Dirichlet(1) ranges with a
    zero_frac share zeroed (drawn per suit-isomorphism class of the board
    with iso_ranges, so that hands a suit symmetry of the board maps onto
    each other weigh the same).  With n_keep=(n1, n2) each player's list is
    pruned to a random subset of that size (ranges then strictly
    positive)."""
    rng = np.random.default_rng([seed, 1])
    if board is None:
        board = np.sort(rng.choice(deck_size, size=5, replace=False)).astype(np.uint8)
    else:
        board = np.sort(np.asarray(board, dtype=np.uint8))
    universe = _all_hands(deck_size, 2, board)
    s_univ = _board_strengths(universe, board, deck_size, rng, tie_p, strengths)
    hands, strength, ranges = [], [], []
    for p in range(2):
        if n_keep is None and iso_ranges:
            from . import handeval
            idx = np.arange(len(universe))
            cls = handeval.suit_classes(universe, board)
            r = _dirichlet_range(int(cls.max()) + 1, rng, zero_frac)[cls]
        elif n_keep is None:
            idx = np.arange(len(universe))
            r = _dirichlet_range(len(idx), rng, zero_frac)
        else:
            idx = np.sort(rng.choice(len(universe), size=int(n_keep[p]), replace=False))
            r = _dirichlet_range(len(idx), rng, 0.0)
        hands.append(universe[idx].copy())
        strength.append(s_univ[idx].reshape(1, -1).astype(np.int32))
        ranges.append(r)
    return GameDesc(
        deck_size=deck_size, cards_per_hand=2, board=board,
        river_cards=np.zeros(0, np.uint8), hands=hands, strength=strength,
        range_=ranges, contrib=pot / 2.0, stack=(float(stack), float(stack)),
        bet_fracs=np.array(sorted(bet_fracs), dtype=np.float64),
        max_raises=max_raises, allow_allin=True, name=name, bet_menu=bet_menu)


def turn_river_config(seed: int = 2, deck_size: int = 52,
                      bet_fracs=(0.33, 0.75, 1.5), max_raises: int = 3,
                      pot: float = 100.0, stack: float = 400.0,
                      zero_frac: float = 0.30, tie_p: float = 0.05,
                      n_board: int = 4, cards_per_hand: int = 2,
                      name: str = "turn_river", strengths: str = "random") -> GameDesc:
    """Turn-plus-river endgame: n_board (4) fixed cards, a betting round, then a
    chance node revealing one card uniformly from those not on the board or in
    either hand, then a river betting round.  Every possible river board gets
    its own seeded strength order (or, with strengths="eval", the hand
    ranking on that board)."""
    rng = np.random.default_rng([seed, 2])
    board = np.sort(rng.choice(deck_size, size=n_board, replace=False)).astype(np.uint8)
    live = np.array([c for c in range(deck_size) if c not in set(board.tolist())], np.uint8)
    rivers = live
    universe = _all_hands(deck_size, cards_per_hand, board)
    n = len(universe)
    s = np.zeros((len(rivers), n), dtype=np.int32)
    for bi, r in enumerate(rivers):
        alive = ~(universe == r).any(axis=1)
        if strengths == "random":
            sa = _strength_with_ties(int(alive.sum()), rng, tie_p)
        else:
            sa = _board_strengths(universe[alive], np.sort(np.append(board, r)), deck_size, rng, tie_p,
                                  strengths)
        s[bi, alive] = sa
        s[bi, ~alive] = -1
    ranges = [_dirichlet_range(n, rng, zero_frac) for _ in range(2)]
    return GameDesc(
        deck_size=deck_size, cards_per_hand=cards_per_hand, board=board,
        river_cards=rivers.astype(np.uint8), hands=[universe.copy(), universe.copy()],
        strength=[s.copy(), s.copy()], range_=ranges,
        contrib=pot / 2.0, stack=(float(stack), float(stack)),
        bet_fracs=np.array(sorted(bet_fracs), dtype=np.float64),
        max_raises=max_raises, allow_allin=True, name=name)


_BATCH_FRACS = (0.33, 0.5, 0.75, 1.0, 1.5, 2.0)


def batched_configs(n_instances: int = 512, seed: int = 3, n_lo: int = 200,
                    n_hi: int = 1081) -> List[GameDesc]:
    """Many river endgames of uneven size: per-player hand counts uniform on
    [n_lo, n_hi] after pruning, 1-3 bet sizes from a fixed menu, raise caps in
    {2,3,4}, pots uniform on [20,400], stack/pot uniform on [1,10]."""
    out = []
    for i in range(n_instances):
        rng = np.random.default_rng([seed, 3, i])
        n1, n2 = rng.integers(n_lo, n_hi + 1, size=2)
        k = int(rng.integers(1, 4))
        fr = np.sort(rng.choice(_BATCH_FRACS, size=k, replace=False))
        mr = int(rng.integers(2, 5))
        pot = float(rng.uniform(20, 400))
        spr = float(rng.uniform(1, 10))
        g = river_config(seed=int(rng.integers(0, 2**31 - 1)), bet_fracs=tuple(fr),
                         max_raises=mr, pot=pot, stack=spr * pot,
                         n_keep=(int(n1), int(n2)), name=f"batch{i}")
        out.append(g)
    return out


def small_river(seed: int = 0, deck_size: int = 12, n_board: int = 2,
                bet_fracs=(0.5, 1.0), max_raises: int = 2, pot: float = 10.0,
                stack: float = 30.0, zero_frac: float = 0.2, tie_p: float = 0.2,
                n_keep: Optional[Sequence[int]] = None, cards_per_hand: int = 2,
                allow_allin: bool = True) -> GameDesc:
    """A small-deck river endgame for brute-force checks (few hands)."""
    rng = np.random.default_rng([seed, 4])
    board = np.sort(rng.choice(deck_size, size=n_board, replace=False)).astype(np.uint8)
    universe = _all_hands(deck_size, cards_per_hand, board)
    s_univ = _strength_with_ties(len(universe), rng, tie_p)
    hands, strength, ranges = [], [], []
    for p in range(2):
        if n_keep is None:
            idx = np.arange(len(universe))
            r = _dirichlet_range(len(idx), rng, zero_frac)
        else:
            idx = np.sort(rng.choice(len(universe), size=int(n_keep[p]), replace=False))
            r = _dirichlet_range(len(idx), rng, 0.0)
        hands.append(universe[idx].copy())
        strength.append(s_univ[idx].reshape(1, -1).astype(np.int32))
        ranges.append(r)
    return GameDesc(
        deck_size=deck_size, cards_per_hand=cards_per_hand, board=board,
        river_cards=np.zeros(0, np.uint8), hands=hands, strength=strength,
        range_=ranges, contrib=pot / 2.0, stack=(float(stack), float(stack)),
        bet_fracs=np.array(sorted(bet_fracs), np.float64), max_raises=max_raises,
        allow_allin=allow_allin, name=f"small_river{seed}")


def small_turn_river(seed: int = 0, deck_size: int = 10, n_board: int = 2,
                     bet_fracs=(1.0,),
                     max_raises: int = 1, pot: float = 10.0, stack: float = 25.0,
                     cards_per_hand: int = 1, tie_p: float = 0.2,
                     zero_frac: float = 0.0) -> GameDesc:
    """A small-deck turn-plus-river endgame for brute-force checks."""
    return turn_river_config(seed=seed, deck_size=deck_size, bet_fracs=bet_fracs,
                             max_raises=max_raises, pot=pot, stack=stack,
                             zero_frac=zero_frac, tie_p=tie_p, n_board=n_board,
                             cards_per_hand=cards_per_hand,
                             name=f"small_turn{seed}")


def libratus_menu(ai: int = 0) -> tuple:
    """The asymmetric river abstraction of the paper's appendix on the
    betting abstraction, as a bet_menu: the AI (player ``ai``) opens with
    0.25 / 0.5 / 1 / 2 / 4 / 8 x pot and answers a check with the same sizes,
    raises a bet by 0.4 / 0.7 / 1.1 / 2, a single raise by 0.4 / 0.7 / 2 and
    later raises by 0.7; the opponent opens with 0.35 / 0.65 / 1, answers a
    check with 0.5 / 0.75 / 1, raises a bet by 0.7 / 1.1 and any raise by 0.7.
    All-in is offered everywhere; there is no raise cap."""
    ai_sizes = ((0.25, 0.5, 1.0, 2.0, 4.0, 8.0), (0.25, 0.5, 1.0, 2.0, 4.0, 8.0),
                (0.4, 0.7, 1.1, 2.0), (0.4, 0.7, 2.0), (0.7,))
    opp_sizes = ((0.35, 0.65, 1.0), (0.5, 0.75, 1.0), (0.7, 1.1), (0.7,), (0.7,))
    return (ai_sizes, opp_sizes) if ai == 0 else (opp_sizes, ai_sizes)


# raise cap standing in for "no cap": the all-in ends every raise war long before
LIBRATUS_MAX_RAISES = 64


def libratus_river(seed: int = 1, ai: int = 0, pot: float = 100.0, stack: float = 400.0,
                   zero_frac: float = 0.30, n_keep: Optional[Sequence[int]] = None,
                   name: str = "libratus_river") -> GameDesc:
    """A river endgame with hand-ranking strengths and the asymmetric
    betting abstraction of libratus_menu (otherwise as river_config)."""
    return river_config(seed=seed, bet_fracs=(1.0,), max_raises=LIBRATUS_MAX_RAISES, pot=pot, stack=stack,
                        zero_frac=zero_frac, n_keep=n_keep, name=name, strengths="eval",
                        bet_menu=libratus_menu(ai))


def config(k: int, seed: Optional[int] = None):
    """The five named workloads: 0 tiny, 1 river, 2 turn+river, 3 batched
    (list of 512), 4 = same instances as 3 (the warm start differs only in how
    they are solved)."""
    if k == 0:
        return tiny_config()
    if k == 1:
        return river_config(seed=1 if seed is None else seed)
    if k == 2:
        return turn_river_config(seed=2 if seed is None else seed)
    if k in (3, 4):
        return batched_configs(512, seed=3 if seed is None else seed)
    raise ValueError(f"unknown workload {k}")


# --------------------------------------------------------------------------
# JSON instance specs
# --------------------------------------------------------------------------

SPEC_FORMAT = "pmx-instances"
SPEC_VERSION = 1


def to_dict(d: GameDesc) -> dict:
    """A JSON-ready dictionary of one instance (exact: floats keep every bit
    through Python's JSON round trip)."""
    return {
        "name": d.name,
        "deck_size": int(d.deck_size), "cards_per_hand": int(d.cards_per_hand),
        "board": [int(c) for c in d.board], "river_cards": [int(c) for c in d.river_cards],
        "hands": [np.asarray(h, dtype=np.int64).tolist() for h in d.hands],
        "strength": [np.asarray(st, dtype=np.int64).tolist() for st in d.strength],
        "range": [[float(v) for v in r] for r in d.range_],
        "contrib": float(d.contrib), "stack": [float(d.stack[0]), float(d.stack[1])],
        "bet_fracs": [float(f) for f in d.bet_fracs], "max_raises": int(d.max_raises),
        "allow_allin": bool(d.allow_allin),
        "bet_menu": None if d.bet_menu is None else [[[float(f) for f in lst] for lst in pl] for pl in d.bet_menu],
    }


def from_dict(o: dict) -> GameDesc:
    """The instance of a dictionary written by to_dict (or by hand, with the
    same keys; "name" and "bet_menu" may be left out)."""
    cph = int(o["cards_per_hand"])
    menu = o.get("bet_menu")
    return GameDesc(
        deck_size=int(o["deck_size"]), cards_per_hand=cph,
        board=np.array(o["board"], dtype=np.uint8).reshape(-1),
        river_cards=np.array(o["river_cards"], dtype=np.uint8).reshape(-1),
        hands=[np.array(h, dtype=np.uint8).reshape(-1, cph) for h in o["hands"]],
        strength=[np.array(st, dtype=np.int32).reshape(max(1, len(o["river_cards"])), -1) for st in o["strength"]],
        range_=[np.array(r, dtype=np.float64) for r in o["range"]],
        contrib=float(o["contrib"]), stack=(float(o["stack"][0]), float(o["stack"][1])),
        bet_fracs=np.array(o["bet_fracs"], dtype=np.float64), max_raises=int(o["max_raises"]),
        allow_allin=bool(o["allow_allin"]), name=str(o.get("name", "")),
        bet_menu=None if menu is None else tuple(tuple(tuple(float(f) for f in lst) for lst in pl) for pl in menu))


def save_json(path: str, descs) -> None:
    """Write one instance or a list of them as a JSON spec."""
    import json
    lst = [descs] if isinstance(descs, GameDesc) else list(descs)
    with open(path, "w") as f:
        json.dump({"format": SPEC_FORMAT, "version": SPEC_VERSION, "instances": [to_dict(d) for d in lst]}, f)


def load_json(path: str) -> List[GameDesc]:
    """The instances of a JSON spec written by save_json."""
    import json
    with open(path) as f:
        o = json.load(f)
    if o.get("format") != SPEC_FORMAT or o.get("version") != SPEC_VERSION:
        raise ValueError(f"{path}: not a {SPEC_FORMAT} version {SPEC_VERSION} file")
    return [from_dict(x) for x in o["instances"]]
