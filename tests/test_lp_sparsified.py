"""The sequence-form LP over the library's sparsified matrix (eq. lp, right
side; paper_2112_03804_amd/lp.py with the C++ Technique-B factors) has the
game value of the oracle's LP over the dense matrix (eq. lp, left side) to
1e-9, and its strategy is an equilibrium strategy of the dense game (its
worst-case value equals the game value).  CPU only."""
import numpy as np
import pytest

from oracle import payoff, solver
from paper_2112_03804_amd import instances as I
from paper_2112_03804_amd import lp
from paper_2112_03804_amd import pmx

CASES = [
    ("kuhn", I.kuhn),
    ("tiny", I.tiny_config),
    ("small_river", lambda: I.small_river(0)),
    ("small_river_pruned", lambda: I.small_river(5, deck_size=11, n_keep=(20, 13))),
    ("small_river_deep", lambda: I.small_river(3, deck_size=10, bet_fracs=(0.5, 1.0), max_raises=2)),
]


@pytest.mark.parametrize("name,fn", CASES)
def test_sparsified_lp_value_equals_the_dense_lp(name, fn):
    d = fn()
    o = payoff.Game(d)
    v_dense, _ = solver.lp_value(o)
    g = pmx.Game(d, device=False)
    v_sp, x = lp.lp_value_sparsified(g)
    g.close()
    assert abs(v_sp - v_dense) <= 1e-9 * max(1.0, abs(v_dense)), (v_sp, v_dense)
    # the LP's strategy guarantees the value against every reply
    tp = solver.Treeplex(o, 1)
    worst = tp.best_value(-o.matvec_AT(x), maximize=True).sum()
    assert abs(-worst - v_dense) <= 1e-7 * max(1.0, abs(v_dense)), (-worst, v_dense)
