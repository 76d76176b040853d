"""Sequence-form LP on the sparsified payoff matrix (eq. lp, right side).

Player 1's equilibrium LP

    max f2^T v   s.t.  A^T x - F2^T v >= 0,  F1 x = f1,  x >= 0

is rewritten with Technique B's factors A = Ahat + U M^-1 V^T (the
library's own, ``Game.tb_build`` / ``Game.tb_matrix``) by naming
w = M^-T U^T x:

    max f2^T v   s.t.  Ahat^T x - F2^T v + V w >= 0,
                       F1 x = f1,  U^T x - M^T w = 0,  x >= 0, v, w free,

whose constraint matrix holds the factors' nonzeros instead of A's (Table 2's
application).  F_i, f_i are the sequence-form constraints built from
``game_layout``: x[empty] = 1 and, for every infoset I and hand h, the
actions of I sum to the parent sequence.  Solved with HiGHS on the CPU (small
games: the LP is not part of the data-parallel path).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _constraints(game, p: int):
    """F (rows: [empty] + (infoset, hand)) over the variables [empty] +
    player p's vector elements, and f."""
    L = game.layouts[0][p]
    lay = game.layout(0, p)
    E = L["n_seq"] * L["stride"]
    N, st = L["n_hands"], L["stride"]
    rows, cols, vals = [0], [0], [1.0]
    r = 1
    for I in range(len(lay["infoset_first"])):
        f, n, par = lay["infoset_first"][I], lay["infoset_nact"][I], lay["infoset_parent"][I]
        for h in range(N):
            for a in range(n):
                rows.append(r), cols.append(1 + (f + a) * st + h), vals.append(1.0)
            rows.append(r), cols.append(0 if par < 0 else 1 + par * st + h), vals.append(-1.0)
            r += 1
    F = sp.csr_matrix((vals, (rows, cols)), shape=(r, 1 + E))
    fvec = np.zeros(r)
    fvec[0] = 1.0
    return F, fvec


def lp_value_sparsified(game):
    """Player 1's game value (chips) and equilibrium strategy (sequence form,
    [n_seq][n_hands]) from the LP over the sparsified matrix.  `game` is a
    pmx.Game of one river endgame (host-only games work)."""
    from scipy.optimize import linprog
    game.tb_build()

    def csr(which):
        ptr, idx, val, shape = game.tb_matrix(which)
        return sp.csr_matrix((val, idx, ptr), shape=shape)

    Ahat, U, M, V = csr(0), csr(1), csr(2), csr(3)
    L0, L1 = game.layouts[0]
    E0 = L0["n_seq"] * L0["stride"]
    E1 = L1["n_seq"] * L1["stride"]
    m = M.shape[0]
    F1, f1 = _constraints(game, 0)
    F2, f2 = _constraints(game, 1)
    nx, nv = 1 + E0, F2.shape[0]
    # variables [x (empty + E0) | v | w]; constraint 1 over [empty] + E1
    Ahat_e = sp.vstack([sp.csr_matrix((1, E1)), Ahat]).tocsr()      # rows [empty] + E0
    Ahat_e = sp.hstack([sp.csr_matrix((1 + E0, 1)), Ahat_e]).tocsr()  # columns [empty] + E1
    V_e = sp.vstack([sp.csr_matrix((1, m)), V]).tocsr()              # rows [empty] + E1
    c1 = sp.hstack([Ahat_e.T, -F2.T, V_e]).tocsr()                    # >= 0
    U_e = sp.vstack([sp.csr_matrix((1, m)), U]).tocsr()              # rows [empty] + E0
    eq = sp.vstack([sp.hstack([F1, sp.csr_matrix((F1.shape[0], nv + m))]),
                    sp.hstack([U_e.T, sp.csr_matrix((m, nv)), -M.T])]).tocsr()
    beq = np.concatenate([f1, np.zeros(m)])
    cost = np.concatenate([np.zeros(nx), -f2, np.zeros(m)])
    # padding elements (hands past the list, stride) are fixed at 0
    xb = [(0.0, None)] + [(0.0, None if (e % L0["stride"]) < L0["n_hands"] else 0.0) for e in range(E0)]
    bounds = xb + [(None, None)] * (nv + m)
    res = linprog(cost, A_ub=-c1, b_ub=np.zeros(c1.shape[0]), A_eq=eq, b_eq=beq, bounds=bounds,
                  method="highs", options={"primal_feasibility_tolerance": 1e-10,
                                           "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        raise RuntimeError(res.message)
    x = res.x[1:nx].reshape(L0["n_seq"], L0["stride"])[:, :L0["n_hands"]]
    return -res.fun, x
