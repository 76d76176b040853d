"""CPU checks of the host-built kernel plans (host logic, no GPU).

* `tests/cpp/rm_plan_check.cpp`: for each game and piece size, every
  sequence lies in exactly one regret-update piece within the size cap, and
  one RM+ update of one hand per instance played through the pieces in launch
  order (deep bottom-up passes, the fused pass with its subtree groups, deep
  top-down passes) equals a plain walk over the whole treeplex.
* `tests/cpp/mc_layout_check.cpp`: the chunk-aligned matvec layout (slots,
  query positions, chunk descriptors, row chunks per class) for 256- and
  512-thread workgroups, evaluated in FP64 the way the workgroup kernel walks
  it, gives the oracle's A y and A^T x.

Each helper is compiled with g++ together with the library's host builder.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2112_03804_amd import instances as I
from paper_2112_03804_amd import pmx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def helper(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("rmplan") / "librmplan.so")
    cmd = [gxx, "-O2", "-std=c++17", "-shared", "-fPIC",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2112_03804_amd", "csrc"),
           os.path.join(ROOT, "tests", "cpp", "rm_plan_check.cpp"),
           os.path.join(ROOT, "paper_2112_03804_amd", "csrc", "host_build.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    L = ctypes.CDLL(out)
    ip = ctypes.POINTER(ctypes.c_int)
    L.check_rm_plan.argtypes = [ctypes.POINTER(pmx.GameDescC), ctypes.c_int, ctypes.c_int, ctypes.c_char_p,
                                ctypes.c_int, ip, ip, ip]
    return L


def _run(L, descs, cap):
    packs = [pmx._DescPack(d) for d in descs]
    arr = (pmx.GameDescC * len(descs))(*[p.c for p in packs])
    msg = ctypes.create_string_buffer(256)
    nt, ng, md = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rc = L.check_rm_plan(arr, len(descs), cap, msg, 256, ctypes.byref(nt), ctypes.byref(ng), ctypes.byref(md))
    return rc, msg.value.decode(), nt.value, ng.value, md.value


CASES = [
    ("kuhn", lambda: [I.kuhn()]),
    ("tiny", lambda: [I.tiny_config()]),
    ("river", lambda: [I.config(1)]),
    ("turn_2card_deep", lambda: [I.small_turn_river(4, deck_size=10, n_board=3, cards_per_hand=2,
                                                    bet_fracs=(0.5, 1.0), max_raises=1, stack=30.0,
                                                    zero_frac=0.2)]),
    ("river_big_tree", lambda: [I.river_config(seed=21, n_keep=(150, 170), bet_fracs=(0.33, 0.75, 1.5),
                                               max_raises=4, stack=400.0)]),
    ("batch_64", lambda: I.batched_configs(64)),
]


@pytest.mark.parametrize("cap", [8, 13, 64])
@pytest.mark.parametrize("name,fn", CASES)
def test_pieces_reproduce_whole_tree_update(helper, name, fn, cap):
    rc, msg, n_tasks, n_grouped, depth = _run(helper, fn(), cap)
    assert rc == 0, msg
    assert n_tasks >= 2


def test_small_caps_give_several_levels_and_groups(helper):
    rc, msg, n_tasks, n_grouped, depth = _run(helper, [I.config(1)], 8)
    assert rc == 0 and depth >= 2, (msg, depth)
    rc, msg, n_tasks, n_grouped, depth = _run(helper, [I.config(1)], 64)
    assert rc == 0 and n_grouped == 2, (msg, n_grouped)   # both players' river trees are split
    rc, msg, *_ = _run(helper, [I.config(1)], 2)           # an infoset has more than 2 actions
    assert rc != 0 and "task_rows" in msg


def test_small_games_take_one_piece_per_treeplex(helper):
    """A game whose treeplexes each fit one piece of 192 rows (the river
    with Libratus' sizes: 166 rows, 56 infosets per player) is planned as one
    piece per player, which the replay still matches; a larger cap is refused
    where it does not apply (the batch)."""
    rc, msg, n_tasks, n_grouped, depth = _run(helper, [I.libratus_river(stack=1000.0)], 192)
    assert rc == 0, msg
    assert n_tasks == 2 and depth == 0, (n_tasks, depth)   # no deep pieces
    rc, msg, *_ = _run(helper, I.batched_configs(64), 192)
    assert rc != 0 and "task_rows" in msg


# ---------------------------------------------------------------------------
# chunk-aligned matvec layout
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def mc_helper(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("mclayout") / "libmclayout.so")
    cmd = [gxx, "-O2", "-std=c++17", "-shared", "-fPIC",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2112_03804_amd", "csrc"),
           os.path.join(ROOT, "tests", "cpp", "mc_layout_check.cpp"),
           os.path.join(ROOT, "paper_2112_03804_amd", "csrc", "host_build.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    L = ctypes.CDLL(out)
    dp = ctypes.POINTER(ctypes.c_double)
    L.mc_matvec.argtypes = [ctypes.POINTER(pmx.GameDescC), ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                            ctypes.c_int64, dp, ctypes.c_int64, ctypes.c_char_p, ctypes.c_int]
    return L


MC_CASES = [
    ("kuhn", lambda: [I.kuhn()]),
    ("tiny", lambda: [I.tiny_config()]),
    ("small_river_pruned", lambda: [I.small_river(5, deck_size=11, n_keep=(20, 13))]),
    ("turn_2card_deep", CASES[3][1]),
    ("river_pruned_mid", lambda: [I.river_config(seed=7, n_keep=(300, 517), bet_fracs=(0.33, 1.5),
                                                 max_raises=2, stack=250.0)]),
    ("uneven_batch", lambda: [I.river_config(seed=600 + i, n_keep=(60 + 90 * i, 400 - 70 * i),
                                             bet_fracs=((0.5,), (0.33, 1.0))[i % 2], max_raises=2)
                              for i in range(4)]),
    ("turn_1card", lambda: [I.small_turn_river(0)]),
]


@pytest.mark.parametrize("block", [256, 512])
@pytest.mark.parametrize("name,fn", MC_CASES)
def test_chunk_aligned_layout_reproduces_oracle_matvec(mc_helper, name, fn, block):
    """The chunk-aligned layout (slots, query positions, chunk descriptors,
    row chunks per class), evaluated in FP64 the way the workgroup kernel
    walks it, gives the oracle's A y and A^T x."""
    import numpy as np
    from oracle import payoff
    descs = fn()
    g = pmx.Game(descs, device=False)
    os_ = [payoff.Game(d) for d in descs]
    rng = np.random.default_rng(block)
    packs = [pmx._DescPack(d) for d in descs]
    arr = (pmx.GameDescC * len(descs))(*[p.c for p in packs])
    dp = ctypes.POINTER(ctypes.c_double)
    parts = 0
    for d in (0, 1):
        vin = [rng.standard_normal((o.S[1 - d], o.N[1 - d])) for o in os_]
        flat_in = np.ascontiguousarray(g.pack(1 - d, vin, np.float64))
        flat_out = np.zeros(g.elems[d])
        msg = ctypes.create_string_buffer(256)
        rc = mc_helper.mc_matvec(arr, len(descs), block, d, flat_in.ctypes.data_as(dp), flat_in.size,
                                 flat_out.ctypes.data_as(dp), flat_out.size, msg, 256)
        assert rc == 0, msg.value
        parts += int(msg.value.decode().split("parts=")[1])
        got = g.unpack(d, flat_out)
        for i, o in enumerate(os_):
            ref = o.matvec_A(vin[i]) if d == 0 else o.matvec_AT(vin[i])
            scale = (o.abs_row_sums() if d == 0 else o.abs_col_sums()).max() * np.abs(vin[i]).max()
            assert np.abs(got[i] - ref).max() <= 1e-12 * scale, (name, d, i)
    # turn games: the all-in run-outs span every river card, more contexts
    # than a chunk's rows, so they are cut into partial rows
    if name.startswith("turn"):
        assert parts > 0, name


# ---------------------------------------------------------------------------
# grouped matvec layout (kernel 4)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def grp_helper(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("grplayout") / "libgrplayout.so")
    cmd = [gxx, "-O2", "-std=c++17", "-shared", "-fPIC",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2112_03804_amd", "csrc"),
           os.path.join(ROOT, "tests", "cpp", "grp_layout_check.cpp"),
           os.path.join(ROOT, "paper_2112_03804_amd", "csrc", "host_build.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    L = ctypes.CDLL(out)
    dp = ctypes.POINTER(ctypes.c_double)
    L.grp_matvec.argtypes = [ctypes.POINTER(pmx.GameDescC), ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                             ctypes.c_int64, dp, ctypes.c_int64, ctypes.c_char_p, ctypes.c_int]
    return L


GRP_CASES = MC_CASES + [
    # enough rows (at least 1024 per direction) for the two-wide and the split kinds
    ("batch_24", lambda: I.batched_configs(24, seed=8)),
    ("turn_1card", lambda: [I.small_turn_river(0)]),
    ("river", lambda: [I.config(1)]),
    ("max_hands", lambda: [I.river_config(seed=5, deck_size=57, n_keep=(1280, 1280), bet_fracs=(0.5,),
                                          max_raises=1)]),
]


@pytest.mark.parametrize("gpc", [1, 8])
@pytest.mark.parametrize("name,fn", GRP_CASES)
def test_grouped_layout_reproduces_oracle_matvec(grp_helper, name, fn, gpc):
    """The grouped layout (components staged in strength order, entry
    gathers, prefix slots, query records, group coefficients and the carry
    flags of rows summed over several boards), evaluated in FP64 the way the
    grouped workgroup kernel walks it, gives the oracle's A y and A^T x."""
    import numpy as np
    from oracle import payoff
    descs = fn()
    g = pmx.Game(descs, device=False)
    os_ = [payoff.Game(d) for d in descs]
    rng = np.random.default_rng(gpc)
    packs = [pmx._DescPack(d) for d in descs]
    arr = (pmx.GameDescC * len(descs))(*[p.c for p in packs])
    dp = ctypes.POINTER(ctypes.c_double)
    for d in (0, 1):
        vin = [rng.standard_normal((o.S[1 - d], o.N[1 - d])) for o in os_]
        flat_in = np.ascontiguousarray(g.pack(1 - d, vin, np.float64))
        flat_out = np.zeros(g.elems[d])
        msg = ctypes.create_string_buffer(256)
        rc = grp_helper.grp_matvec(arr, len(descs), gpc, d, flat_in.ctypes.data_as(dp), flat_in.size,
                                   flat_out.ctypes.data_as(dp), flat_out.size, msg, 256)
        assert rc == 0, msg.value
        got = g.unpack(d, flat_out)
        for i, o in enumerate(os_):
            ref = o.matvec_A(vin[i]) if d == 0 else o.matvec_AT(vin[i])
            scale = (o.abs_row_sums() if d == 0 else o.abs_col_sums()).max() * np.abs(vin[i]).max()
            assert np.abs(got[i] - ref).max() <= 1e-12 * scale, (name, d, i)
