"""Payoff matrix from its definition (oracle; test infrastructure only).

Section 2 of the paper: Player 1's payoff matrix has rows indexed by
Player 1's sequences and columns by Player 2's; each terminal z adds, at
(sigma1(z), sigma2(z)), its payoff u times the probability c of the chance
events on the way to z.  In a poker endgame the chance events are the deal of
private hands (Section 3: pi(h1, h2) = mu1(h1) mu2(h2) / beta on compatible
pairs, 0 otherwise) and, in a turn + river endgame, the river card (drawn
uniformly from the cards not on the board and not in either hand).  The
showdown outcome gamma(h1, h2) is +1 / -1 / 0 for win / loss / tie-or-
incompatible (Section 3).

So the matrix, in sequence-major layout (row sigma1*N1 + h1, column
sigma2*N2 + h2), is  A = sum_z  e_{sigma1(z)} e_{sigma2(z)}^T (x) Q_z  with

    Q_z[h1, h2] = pi(h1, h2) * P(board of z | h1, h2) * u1(z; h1, h2),

u1 = -c1 (Player 1 folded), +c2 (Player 2 folded), c * gamma (showdown).  A
showdown reached all-in before the river averages gamma over the river card.

Everything is FP64.  No sorting, prefix sums or inclusion-exclusion: the
oracle evaluates this sum over (terminal, hand pair) directly.
"""
from __future__ import annotations

import numpy as np

from . import skeleton as sk


class HandModel:
    """Deal distribution, chance and showdown outcomes of one instance."""

    def __init__(self, desc):
        self.desc = desc
        self.hands = [np.asarray(h, dtype=np.int64) for h in desc.hands]
        self.mu = [np.asarray(r, dtype=np.float64) for r in desc.range_]
        self.N = [len(h) for h in self.hands]
        board = set(int(c) for c in desc.board)
        for h in self.hands:
            for row in h:
                if board & set(int(c) for c in row):
                    raise ValueError("hand collides with the board")
        # H^x: incompatible pairs (share a card); hands never touch the board
        self.share = np.zeros((self.N[0], self.N[1]), dtype=bool)
        for a in range(self.hands[0].shape[1]):
            for b in range(self.hands[1].shape[1]):
                self.share |= self.hands[0][:, a, None] == self.hands[1][None, :, b]
        prod = np.outer(self.mu[0], self.mu[1])
        self.beta = float(prod[~self.share].sum())
        if not self.beta > 0:
            raise ValueError("beta must be positive")
        self.pi = np.where(self.share, 0.0, prod / self.beta)
        self.rivers = [int(r) for r in desc.river_cards]
        self.remaining = desc.deck_size - len(desc.board) - 2 * desc.cards_per_hand

    # --- chance over the river card -------------------------------------
    def has_card(self, p, card):
        return (self.hands[p] == card).any(axis=1)

    def river_prob(self, r_idx):
        """P(river card = rivers[r_idx] | h1, h2): uniform over the cards left."""
        r = self.rivers[r_idx]
        ok = np.outer(~self.has_card(0, r), ~self.has_card(1, r))
        return np.where(ok, 1.0 / self.remaining, 0.0)

    # --- showdown outcome -------------------------------------------------
    def gamma(self, board):
        """gamma on final board `board` (-1: the only board of a river endgame)."""
        b = 0 if board < 0 else board
        s1 = self.desc.strength[0][b].astype(np.int64)
        s2 = self.desc.strength[1][b].astype(np.int64)
        g = np.sign(s1[:, None] - s2[None, :]).astype(np.float64)
        g[self.share] = 0.0
        if board >= 0:
            r = self.rivers[board]
            g[self.has_card(0, r), :] = 0.0
            g[:, self.has_card(1, r)] = 0.0
        return g

    # --- per-terminal hand matrices --------------------------------------
    def q_matrix(self, t: sk.Terminal):
        """Q_z = pi * P(board) * u1 for terminal t."""
        if t.kind != sk.SHOWDOWN:
            m = self.pi * t.u1
            if t.board >= 0:
                m = m * self.river_prob(t.board)
            return m
        if t.runout:
            acc = np.zeros_like(self.pi)
            for r in range(len(self.rivers)):
                acc += self.river_prob(r) * self.gamma(r)
            return self.pi * acc * t.c1
        m = self.pi * self.gamma(t.board) * t.c1
        if t.board >= 0:
            m = m * self.river_prob(t.board)
        return m

    def q_row(self, t: sk.Terminal, h1: int):
        """Row h1 of Q_z (for one output entry of A y)."""
        return self._q_line(t, h1, axis=0)

    def q_col(self, t: sk.Terminal, h2: int):
        """Column h2 of Q_z (for one output entry of A^T x)."""
        return self._q_line(t, h2, axis=1)

    def _q_line(self, t, k, axis):
        def take(m):
            return m[k, :] if axis == 0 else m[:, k]
        pi = take(self.pi)
        if t.kind != sk.SHOWDOWN:
            v = pi * t.u1
            if t.board >= 0:
                v = v * self._river_line(t.board, k, axis)
            return v
        if t.runout:
            acc = np.zeros_like(pi)
            for r in range(len(self.rivers)):
                acc += self._river_line(r, k, axis) * self._gamma_line(r, k, axis)
            return pi * acc * t.c1
        v = pi * self._gamma_line(t.board, k, axis) * t.c1
        if t.board >= 0:
            v = v * self._river_line(t.board, k, axis)
        return v

    def _river_line(self, r_idx, k, axis):
        r = self.rivers[r_idx]
        own = 0 if axis == 0 else 1
        other = 1 - own
        if self.has_card(own, r)[k]:
            return np.zeros(self.N[other])
        return np.where(self.has_card(other, r), 0.0, 1.0 / self.remaining)

    def _gamma_line(self, board, k, axis):
        b = 0 if board < 0 else board
        own = 0 if axis == 0 else 1
        other = 1 - own
        s_own = int(self.desc.strength[own][b][k])
        s_oth = self.desc.strength[other][b].astype(np.int64)
        g = np.sign(s_own - s_oth).astype(np.float64)
        if own == 1:
            g = -g                        # gamma is from Player 1's side
        share = self.share[k, :] if axis == 0 else self.share[:, k]
        g[share] = 0.0
        if board >= 0:
            r = self.rivers[board]
            if self.has_card(own, r)[k]:
                g[:] = 0.0
            g[self.has_card(other, r)] = 0.0
        return g


class Game:
    """An instance with its sequence form and hand model."""

    def __init__(self, desc):
        self.desc = desc
        self.sf = sk.from_desc(desc)
        self.hm = HandModel(desc)
        self.S = self.sf.n_seq
        self.N = self.hm.N
        for t in self.sf.terminals:
            if t.seq1 < 0 or t.seq2 < 0:
                raise ValueError("terminal reached without both players acting")

    @property
    def pot(self):
        return 2.0 * self.desc.contrib

    # ------------------------------------------------------------------
    def dense_A(self):
        """A as a dense (S1*N1) x (S2*N2) FP64 matrix, sequence-major."""
        S1, S2 = self.S
        N1, N2 = self.N
        A = np.zeros((S1 * N1, S2 * N2))
        for t in self.sf.terminals:
            A[t.seq1 * N1:(t.seq1 + 1) * N1, t.seq2 * N2:(t.seq2 + 1) * N2] += self.hm.q_matrix(t)
        return A

    def _by_board(self):
        order = sorted(range(len(self.sf.terminals)),
                       key=lambda i: (self.sf.terminals[i].board, self.sf.terminals[i].runout,
                                      self.sf.terminals[i].kind == sk.SHOWDOWN))
        return [self.sf.terminals[i] for i in order]

    def _groups(self):
        """Terminals grouped by their hand matrix up to the payoff factor:
        (board, run-out, showdown or fold) -> (base Q with u1 = 1, terminals).
        Bases are built one group at a time (a turn + river game has 100 of
        them, 10 MB each)."""
        groups = {}
        for t in self._by_board():
            groups.setdefault((t.board, t.runout, t.kind == sk.SHOWDOWN), []).append(t)
        for key, ts in groups.items():
            t0 = ts[0]
            base = self.hm.q_matrix(sk.Terminal(0, 0, t0.kind if t0.kind == sk.SHOWDOWN else sk.FOLD2,
                                                1.0, 1.0, t0.board, t0.runout))
            yield base, ts

    @staticmethod
    def _coef(t):
        return t.c1 if t.kind == sk.SHOWDOWN else t.u1

    def matvec_A(self, y):
        """A y for y of shape (S2, N2): sum over terminals of Q_z y[sigma2(z)].
        Terminals sharing a base matrix are taken together: one product of
        the base with their stacked input rows, each scaled by its payoff."""
        y = np.asarray(y, dtype=np.float64)
        out = np.zeros((self.S[0], self.N[0]))
        for base, ts in self._groups():
            s1 = np.array([t.seq1 for t in ts])
            s2 = np.array([t.seq2 for t in ts])
            coef = np.array([self._coef(t) for t in ts])
            np.add.at(out, s1, coef[:, None] * (y[s2] @ base.T))
        return out

    def matvec_AT(self, x):
        """A^T x for x of shape (S1, N1)."""
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros((self.S[1], self.N[1]))
        for base, ts in self._groups():
            s1 = np.array([t.seq1 for t in ts])
            s2 = np.array([t.seq2 for t in ts])
            coef = np.array([self._coef(t) for t in ts])
            np.add.at(out, s2, coef[:, None] * (x[s1] @ base))
        return out

    def entry_A(self, y, s1, h1):
        """One entry (A y)[s1, h1], summed directly over terminals and hands."""
        acc = 0.0
        for t in self.sf.terminals:
            if t.seq1 == s1:
                acc += float(self.hm.q_row(t, h1) @ y[t.seq2])
        return acc

    def entry_AT(self, x, s2, h2):
        """One entry (A^T x)[s2, h2]."""
        acc = 0.0
        for t in self.sf.terminals:
            if t.seq2 == s2:
                acc += float(self.hm.q_col(t, h2) @ x[t.seq1])
        return acc

    def abs_row_sums(self):
        """Row sums of |A| (their max is the infinity norm), matrix-free:
        |Q_z| = |u1(z)| |base| within a group of terminals."""
        acc = np.zeros((self.S[0], self.N[0]))
        for base, ts in self._groups():
            rs = np.abs(base).sum(axis=1)
            for t in ts:
                acc[t.seq1] += abs(self._coef(t)) * rs
        return acc

    def abs_col_sums(self):
        acc = np.zeros((self.S[1], self.N[1]))
        for base, ts in self._groups():
            cs = np.abs(base).sum(axis=0)
            for t in ts:
                acc[t.seq2] += abs(self._coef(t)) * cs
        return acc


def abs_entry_A(game: Game, y, s1, h1):
    """(|A| |y|)[s1, h1]: the scale of one output entry (tolerances)."""
    acc = 0.0
    for t in game.sf.terminals:
        if t.seq1 == s1:
            acc += float(np.abs(game.hm.q_row(t, h1)) @ np.abs(y[t.seq2]))
    return acc


def abs_entry_AT(game: Game, x, s2, h2):
    acc = 0.0
    for t in game.sf.terminals:
        if t.seq2 == s2:
            acc += float(np.abs(game.hm.q_col(t, h2)) @ np.abs(x[t.seq1]))
    return acc


def abs_matvec_A(game: Game, y):
    """|A| |y| for every entry (matrix-free)."""
    ay = np.abs(np.asarray(y, dtype=np.float64))
    out = np.zeros((game.S[0], game.N[0]))
    for base, ts in game._groups():
        s1 = np.array([t.seq1 for t in ts])
        s2 = np.array([t.seq2 for t in ts])
        coef = np.abs(np.array([game._coef(t) for t in ts]))
        np.add.at(out, s1, coef[:, None] * (ay[s2] @ np.abs(base).T))
    return out


def abs_matvec_AT(game: Game, x):
    ax = np.abs(np.asarray(x, dtype=np.float64))
    out = np.zeros((game.S[1], game.N[1]))
    for base, ts in game._groups():
        s1 = np.array([t.seq1 for t in ts])
        s2 = np.array([t.seq2 for t in ts])
        coef = np.abs(np.array([game._coef(t) for t in ts]))
        np.add.at(out, s2, coef[:, None] * (ax[s1] @ np.abs(base)))
    return out
