"""The allocation-free gap entry point (saddle_gap_of_static) against
saddle_gap_of, through the C ABI: the same kernels on the static device
scratch give the same FP64 gap and best responses (to 1e-9 * pot, and in
fact the same bits), on two calls in a row, the second on a smaller game,
and a game too large for the static scratch is refused with an error."""
import numpy as np
import pytest

from paper_2112_03804_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_03804_amd import pmx
    pmx.lib()
    return pmx


def _plans(g, seed):
    """Random sequence-form strategies: uniform-start iterates after a few
    solver steps, exported in FP64."""
    g.solver_step(seed)
    torch.cuda.synchronize()
    xs = [torch.from_numpy(np.ascontiguousarray(g.get_average_strategy(p))).cuda() for p in range(2)]
    return xs


def test_static_gap_matches_allocating_gap():
    pmx = _need_gpu()
    for name, desc, steps in (("river", I.config(1), 37),
                              ("small river", I.river_config(seed=11, n_keep=(150, 90), bet_fracs=(0.5,),
                                                             max_raises=1), 11)):
        print("static gap:", name, flush=True)
        g = pmx.Game(desc)
        x, y = _plans(g, steps)
        pot = 2 * desc.contrib
        gap, b1, b2 = g.saddle_gap_of(x, y)
        sgap, sb1, sb2 = g.saddle_gap_of_static(x, y)
        assert abs(sgap[0] - gap[0]) <= 1e-9 * pot and abs(sb1[0] - b1[0]) <= 1e-9 * pot
        assert abs(sb2[0] - b2[0]) <= 1e-9 * pot
        assert sgap[0] == gap[0] and sb1[0] == b1[0] and sb2[0] == b2[0]
        assert gap[0] >= 0
        g.close()


def test_static_gap_refuses_games_beyond_its_scratch():
    pmx = _need_gpu()
    descs = I.batched_configs(64)
    g = pmx.Game(descs)
    x = torch.zeros(g.elems[0], dtype=torch.float64, device="cuda")
    y = torch.zeros(g.elems[1], dtype=torch.float64, device="cuda")
    with pytest.raises(pmx.PmxError, match="scratch"):
        g.saddle_gap_of_static(x, y)
    g.close()
