"""Solver checkpoint files on the GPU: saving a batch mid-solve (DCFR, one
instance retired) and loading the file into a fresh game of the same shape
continues with bit-identical iterates, weights and gaps."""
import numpy as np
import pytest

from paper_2112_03804_amd import checkpoint, instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_checkpoint_file_round_trip(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_03804_amd import pmx
    print("checkpoint round trip", flush=True)
    descs = [I.river_config(seed=60 + i, n_keep=(90 + 40 * i, 150 - 30 * i), bet_fracs=((0.5,), (0.33, 1.0))[i % 2],
                            max_raises=2) for i in range(3)]
    params = {"kind": "dcfr", "alpha": 1.5, "beta": 0.0, "gamma": 2}
    g = pmx.Game(descs)
    g.game_tune(4, 2)
    g.solver_set_params(**params)
    g.solver_step(40)
    active = np.array([1, 0, 1], np.int32)
    g.solver_set_active(active)
    g.solver_step(10)
    torch.cuda.synchronize()
    path = str(tmp_path / "ckpt.npz")
    checkpoint.save(g, path, params=params, active=active)
    g.solver_step(30)
    torch.cuda.synchronize()
    want = [g.solver_get_state(p) for p in range(2)]
    want_w = g.solver_get_weights()
    want_gap = g.saddle_gap()[0]

    g2 = pmx.Game(descs)
    meta = checkpoint.load(g2, path)
    assert meta["t"] == 50 and tuple(g2.game_get_tuning()) == (4, 2)
    g2.solver_step(30)
    torch.cuda.synchronize()
    for p in range(2):
        got = g2.solver_get_state(p)
        for k in ("regret", "plan", "avg_sum"):
            assert np.array_equal(got[k], want[p][k]), (p, k)
        assert got["t"] == want[p]["t"] == 80
    assert np.array_equal(g2.solver_get_weights(), want_w)
    # the retired instance took no weight after it retired
    assert want_w[1] < want_w[0]
    assert np.allclose(g2.saddle_gap()[0], want_gap, rtol=0, atol=1e-12 * max(2 * d.contrib for d in descs))
    g.close()
    g2.close()
