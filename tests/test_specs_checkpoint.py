"""JSON instance specs and solver checkpoint files (host side).

A spec round trip gives back every array bit for bit (and the library builds
the same game from it); a checkpoint is refused for a game of another shape
or a file of another format before any device work.  The device round trip
(save, load into a fresh game, identical next iterations) is a GPU test.
"""
import json

import numpy as np
import pytest

from paper_2112_03804_amd import checkpoint, instances as I, pmx


def _same(a, b):
    assert a.name == b.name and a.deck_size == b.deck_size and a.cards_per_hand == b.cards_per_hand
    for u, v in ((a.board, b.board), (a.river_cards, b.river_cards), (a.bet_fracs, b.bet_fracs)):
        assert u.dtype == v.dtype and np.array_equal(u, v)
    for p in range(2):
        for u, v in ((a.hands[p], b.hands[p]), (a.strength[p], b.strength[p]), (a.range_[p], b.range_[p])):
            assert u.shape == v.shape and np.array_equal(u, v)
    assert (a.contrib, tuple(a.stack), a.max_raises, bool(a.allow_allin)) == \
        (b.contrib, tuple(b.stack), b.max_raises, bool(b.allow_allin))
    assert a.bet_menu == b.bet_menu


@pytest.mark.parametrize("descs", [
    lambda: [I.config(1)],
    lambda: I.batched_configs(4),
    lambda: [I.libratus_river(seed=3, ai=1, stack=400.0, n_keep=(40, 60))],
    lambda: [I.small_turn_river(1, deck_size=9, n_board=3, cards_per_hand=2, bet_fracs=(0.5,), max_raises=0,
                                stack=8.0), I.tiny_config()],
])
def test_json_spec_round_trip(descs, tmp_path):
    ds = descs()
    path = str(tmp_path / "spec.json")
    I.save_json(path, ds)
    back = I.load_json(path)
    assert len(back) == len(ds)
    for a, b in zip(ds, back):
        _same(a.copy(), b)
    # the library builds the same game from the spec
    g1, g2 = pmx.Game(ds, device=False), pmx.Game(back, device=False)
    assert np.array_equal(checkpoint.game_shape(g1), checkpoint.game_shape(g2)) and g1.elems == g2.elems
    for L1, L2 in zip(g1.layouts, g2.layouts):
        for p in range(2):
            for k, v in L1[p].items():
                assert np.array_equal(np.asarray(v), np.asarray(L2[p][k])), (p, k)
    g1.close()
    g2.close()


def test_json_spec_rejects_other_files(tmp_path):
    path = str(tmp_path / "other.json")
    with open(path, "w") as f:
        json.dump({"format": "something-else", "instances": []}, f)
    with pytest.raises(ValueError):
        I.load_json(path)


def test_checkpoint_refuses_other_shapes_and_formats(tmp_path):
    d = I.small_river(0)
    g = pmx.Game(d, device=False)
    shape = checkpoint.game_shape(g)
    assert shape.shape == (1, 6) and shape[0, 1] == len(d.hands[0])
    meta = {"format": checkpoint.FORMAT, "version": checkpoint.VERSION, "params": {"kind": "rm+"}, "t": 3,
            "wsum": 6.0, "tuning": [4, 1]}
    arrays = {f"{k}{p}": np.zeros(g.elems[p], dt) for p in range(2)
              for k, dt in (("regret", np.float32), ("plan", np.float32), ("avg", np.float64))}
    good = str(tmp_path / "good.npz")
    np.savez(good, meta=np.array(json.dumps(meta)), shape=shape, weights=np.zeros(1), active=np.ones(1, np.int32),
             **arrays)
    data = checkpoint.read(good)
    checkpoint.check_shape(g, data)            # accepted
    other = pmx.Game(I.small_river(5, deck_size=11, n_keep=(20, 13)), device=False)
    with pytest.raises(ValueError):
        checkpoint.check_shape(other, data)
    with pytest.raises(ValueError):
        checkpoint.load(other, good)           # refused before any device call
    bad = str(tmp_path / "bad.npz")
    np.savez(bad, meta=np.array(json.dumps(dict(meta, version=99))), shape=shape, **arrays)
    with pytest.raises(ValueError):
        checkpoint.read(bad)
    short = dict(arrays, regret0=np.zeros(3, np.float32))
    bad2 = str(tmp_path / "bad2.npz")
    np.savez(bad2, meta=np.array(json.dumps(meta)), shape=shape, weights=np.zeros(1), active=np.ones(1, np.int32),
             **short)
    with pytest.raises(ValueError):
        checkpoint.check_shape(g, checkpoint.read(bad2))
    g.close()
    other.close()
