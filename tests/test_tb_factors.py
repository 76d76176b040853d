"""Technique B's explicit factors built by the library (host_sparsify.cpp,
no oracle code) have the sizes of the oracle's factors (oracle/sparsify.py,
pinned by its own tests): nonzeros of A, of Ahat, U, M and V before and
after the Postprocessing subsection's removal of V's zero columns, and the
solve's dimension.  CPU only (host-side build)."""
import pytest

from oracle import payoff, sparsify
from paper_2112_03804_amd import instances as I
from paper_2112_03804_amd import pmx

CASES = [
    ("small_river", lambda: I.small_river(0)),
    ("small_river_pruned", lambda: I.small_river(5, deck_size=11, n_keep=(20, 13))),
    ("one_card_deck", lambda: I.tiny_config()),
    ("river_pruned_mid", lambda: I.river_config(seed=7, n_keep=(300, 517), bet_fracs=(0.33, 1.5),
                                                max_raises=2, stack=250.0)),
]


@pytest.mark.parametrize("name,fn", CASES)
def test_factor_sizes_match_the_oracle(name, fn):
    d = fn()
    g = pmx.Game(d, device=False)
    z = g.tb_build()
    o = payoff.Game(d)
    Ah, U, M, V, _ = sparsify.factors(o)
    U2, M2, V2 = sparsify.postprocess(U, M, V)
    ref = dict(nnz_A=sparsify.payoff_nnz(o), nnz_ahat=sparsify.size(Ah), nnz_u=sparsify.size(U),
               nnz_m=sparsify.size(M), nnz_v=sparsify.size(V), nnz_u_pp=sparsify.size(U2),
               nnz_m_pp=sparsify.size(M2), nnz_v_pp=sparsify.size(V2), m_dim=M.shape[0], m_dim_pp=M2.shape[0])
    assert {k: z[k] for k in ref} == ref
    assert z["chain_depth"] >= 1
    g.close()


def test_factors_refuse_batches_and_turn_games():
    for descs in ([I.small_river(0), I.small_river(1)], [I.small_turn_river(0)]):
        g = pmx.Game(descs, device=False)
        with pytest.raises(pmx.PmxError):
            g.tb_build()
        g.close()
