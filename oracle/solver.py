"""Regret matching+, best response, saddle gap and the sequence-form LP
(oracle; test infrastructure only).  Everything in FP64.

Vectors are sequence-major and hand-contiguous: v[sigma, h] for a player's
non-empty sequences sigma and hands h (the empty sequence, shared by every
hand, is implicit with value 1).

* Gradients (Section 2, application 3): Player 1 maximizes x^T A y and
  receives g1 = A y; Player 2 minimizes and receives g2 = -A^T x.
* Regret matching+ on the treeplex of each player, per hand (the paper's GPU
  solver updates all hands in parallel; its DCFR parameters are unstated, so
  the plain RM+ rule is used): counterfactual values are accumulated
  bottom-up,  q(I,a) = g[Ia] + sum of V(J) over infosets J below Ia,
  V(I) = sum_a b(a|I) q(I,a);  regrets R(I,a) <- max(0, R + q - V); the next
  behavioural strategy is R / sum R (uniform when the sum is 0); the
  realization plan is rebuilt top-down x[Ia] = x[parent(I)] b(a|I).
  Updates alternate (Player 1 with y_t, then Player 2 with x_{t+1}); the
  averages weight the iterate of step t by t.
* Exploitability (Section 5, first-order methods): the saddle gap
  max_x x^T A ybar - min_y xbar^T A y, each side by a bottom-up max / min over
  the treeplex; half of it, over the initial pot, is the paper's measure.
* The sequence-form LP on the left of eq. (lp) gives the exact game value.
"""
from __future__ import annotations

import numpy as np

from .payoff import Game


class Treeplex:
    """One player's infosets, in depth-first preorder (parents first)."""

    def __init__(self, game: Game, p: int):
        self.p = p
        self.S = game.S[p]
        self.N = game.N[p]
        self.inf = [(I.parent_seq, I.first_seq, I.n_actions) for I in game.sf.infosets[p]]
        self.roots = [i for i, (par, _, _) in enumerate(self.inf) if par < 0]

    def behaviour_from_regret(self, R):
        """b(a|I) = R+ / sum R+ (uniform where the sum is 0); shape (S, N)."""
        b = np.zeros_like(R)
        for par, f, n in self.inf:
            r = np.maximum(R[f:f + n], 0.0)
            s = r.sum(axis=0)
            pos = s > 0
            b[f:f + n] = np.where(pos[None, :], r / np.where(pos, s, 1.0)[None, :], 1.0 / n)
        return b

    def realization(self, b):
        """Sequence-form plan of a behavioural strategy b (top-down)."""
        x = np.zeros_like(b)
        for par, f, n in self.inf:
            reach = 1.0 if par < 0 else x[par]
            x[f:f + n] = b[f:f + n] * reach
        return x

    def rmplus_update(self, R, g):
        """One RM+ regret update from gradient g; returns new regrets."""
        b = self.behaviour_from_regret(R)
        q = np.array(g, dtype=np.float64, copy=True)
        R = R.copy()
        for par, f, n in reversed(self.inf):
            V = (b[f:f + n] * q[f:f + n]).sum(axis=0)
            R[f:f + n] = np.maximum(R[f:f + n] + q[f:f + n] - V[None, :], 0.0)
            if par >= 0:
                q[par] += V
        return R

    def dcfr_update(self, R, g, t, alpha, beta):
        """Discounted CFR regret update at iteration t: positive regrets are
        scaled by t^a/(t^a+1), the others by t^b/(t^b+1), then the
        instantaneous regret q - V is added (no floor)."""
        b = self.behaviour_from_regret(R)
        q = np.array(g, dtype=np.float64, copy=True)
        R = R.copy()
        dp = t ** alpha / (t ** alpha + 1.0)
        dn = t ** beta / (t ** beta + 1.0)
        for par, f, n in reversed(self.inf):
            V = (b[f:f + n] * q[f:f + n]).sum(axis=0)
            r = R[f:f + n]
            R[f:f + n] = r * np.where(r > 0, dp, dn) + q[f:f + n] - V[None, :]
            if par >= 0:
                q[par] += V
        return R

    def best_value(self, g, maximize=True):
        """Per-hand best-response value: sum over root infosets of the
        bottom-up max (or min) of g plus the values below."""
        q = np.array(g, dtype=np.float64, copy=True)
        rootv = np.zeros(self.N)
        for i in reversed(range(len(self.inf))):
            par, f, n = self.inf[i]
            blk = q[f:f + n]
            V = blk.max(axis=0) if maximize else blk.min(axis=0)
            if par >= 0:
                q[par] += V
            else:
                rootv += V
        return rootv

    def uniform(self):
        return self.realization(self.behaviour_from_regret(np.zeros((self.S, self.N))))


class RMPlus:
    """Plain FP64 alternating RM+ with linear averaging; with kind="dcfr",
    Discounted CFR (the solver of the paper's GPU experiments): discounted
    regrets (alpha, beta) and averages weighted t^gamma."""

    def __init__(self, game: Game, matvec_A=None, matvec_AT=None, kind="rm+", alpha=1.5, beta=0.0,
                 gamma=2):
        self.kind, self.alpha, self.beta, self.gamma = kind, alpha, beta, gamma
        self.g = game
        self.tp = [Treeplex(game, 0), Treeplex(game, 1)]
        self.A = matvec_A or game.matvec_A
        self.AT = matvec_AT or game.matvec_AT
        self.R = [np.zeros((game.S[p], game.N[p])) for p in range(2)]
        self.x = [self.tp[p].uniform() for p in range(2)]
        self.sum = [np.zeros_like(self.x[p]) for p in range(2)]
        self.wsum = 0.0
        self.t = 0

    def _update(self, p, g):
        if self.kind == "dcfr":
            return self.tp[p].dcfr_update(self.R[p], g, float(self.t), self.alpha, self.beta)
        return self.tp[p].rmplus_update(self.R[p], g)

    def step(self):
        self.t += 1
        t = float(self.t)
        w = t ** self.gamma if self.kind == "dcfr" else t
        for p in range(2):
            self.sum[p] += w * self.x[p]
        self.wsum += w
        g1 = self.A(self.x[1])
        self.R[0] = self._update(0, g1)
        self.x[0] = self.tp[0].realization(self.tp[0].behaviour_from_regret(self.R[0]))
        g2 = -self.AT(self.x[0])
        self.R[1] = self._update(1, g2)
        self.x[1] = self.tp[1].realization(self.tp[1].behaviour_from_regret(self.R[1]))

    def average(self, p):
        return self.sum[p] / self.wsum if self.wsum > 0 else self.x[p].copy()

    def gap(self):
        return saddle_gap(self.g, self.average(0), self.average(1), self.A, self.AT)


def saddle_gap(game: Game, x, y, A=None, AT=None):
    """(gap, br1, br2) with br1 = max_x' x'^T A y, br2 = min_y' x^T A y'."""
    A = A or game.matvec_A
    AT = AT or game.matvec_AT
    tp1, tp2 = Treeplex(game, 0), Treeplex(game, 1)
    br1 = float(tp1.best_value(A(y), maximize=True).sum())
    br2 = float(tp2.best_value(AT(x), maximize=False).sum())
    return br1 - br2, br1, br2


def value(game: Game, x, y):
    return float((x * game.matvec_A(y)).sum())


# ----------------------------------------------------------------------
# Sequence-form LP (left-hand side of eq. lp)
# ----------------------------------------------------------------------

def _constraints(game: Game, p: int):
    """F, f of one player over [empty] + (sigma, h) variables."""
    S, N = game.S[p], game.N[p]
    infs = game.sf.infosets[p]
    nvar = 1 + S * N
    rows = [np.eye(1, nvar, 0).ravel()]        # x_empty = 1
    for I in infs:
        for h in range(N):
            r = np.zeros(nvar)
            for a in range(I.n_actions):
                r[1 + (I.first_seq + a) * N + h] = 1.0
            r[0 if I.parent_seq < 0 else 1 + I.parent_seq * N + h] -= 1.0
            rows.append(r)
    F = np.array(rows)
    f = np.zeros(len(rows))
    f[0] = 1.0
    return F, f


def lp_value(game: Game, A_dense=None, player: int = 0):
    """Game value for `player` (0: Player 1 maximizing x^T A y; 1: Player 2
    maximizing -x^T A y) from the sequence-form LP, solved with HiGHS:
        max f_o^T v  s.t.  B^T x - F_o^T v >= 0,  F x = f,  x >= 0."""
    from scipy.optimize import linprog
    from scipy.sparse import csr_matrix
    A = game.dense_A() if A_dense is None else A_dense
    S1, S2 = game.S
    N1, N2 = game.N
    Ae = np.zeros((1 + S1 * N1, 1 + S2 * N2))
    Ae[1:, 1:] = A
    if player == 0:
        B = Ae
        F, f = _constraints(game, 0)
        Fo, fo = _constraints(game, 1)
    else:
        B = -Ae.T
        F, f = _constraints(game, 1)
        Fo, fo = _constraints(game, 0)
    nx, nv = B.shape[0], Fo.shape[0]
    c = np.concatenate([np.zeros(nx), -fo])
    A_ub = np.hstack([-B.T, Fo.T])
    b_ub = np.zeros(B.shape[1])
    A_eq = np.hstack([F, np.zeros((F.shape[0], nv))])
    bounds = [(0, None)] * nx + [(None, None)] * nv
    res = linprog(c, A_ub=csr_matrix(A_ub), b_ub=b_ub, A_eq=csr_matrix(A_eq), b_eq=f,
                  bounds=bounds, method="highs",
                  options={"primal_feasibility_tolerance": 1e-10,
                           "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        raise RuntimeError(res.message)
    x = res.x[:nx]
    strat = x[1:].reshape(game.S[player], game.N[player])
    return -res.fun, strat
