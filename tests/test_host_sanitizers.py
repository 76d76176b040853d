"""The host builder under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): tests/cpp/host_sanitize.cpp, built with g++ together with
host_build.cpp, runs every host-side plan builder on games from the seeded
generators (the one-card and two-card small games, turn + river games, the
river, pruned and uneven batches, the maximum hand count); any report of an
out-of-bounds access, a use after free, a leak or undefined behaviour fails
the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2112_03804_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write(descs, path):
    out = [str(len(descs))]
    for d in descs:
        board = list(d.board)
        rivers = list(d.river_cards)
        parts = [d.deck_size, d.cards_per_hand, len(board), *board, len(rivers), *rivers,
                 len(d.hands[0]), len(d.hands[1])]
        for p in range(2):
            parts += list(np.asarray(d.hands[p]).ravel())
        for p in range(2):
            parts += list(np.asarray(d.strength[p]).ravel())
        line = " ".join(str(int(v)) for v in parts)
        rng = " ".join(repr(float(v)) for p in range(2) for v in np.asarray(d.range_[p]))
        tail = [repr(float(d.contrib)), repr(float(d.stack[0])), repr(float(d.stack[1])), str(len(d.bet_fracs))]
        tail += [repr(float(f)) for f in d.bet_fracs] + [str(int(d.max_raises)), str(1 if d.allow_allin else 0)]
        menu = getattr(d, "bet_menu", None)
        if menu is None:
            tail.append("0")
        else:
            tail += ["1"] + [str(len(menu[p][k])) for p in range(2) for k in range(5)]
            tail += [repr(float(f)) for p in range(2) for k in range(5) for f in menu[p][k]]
        out.append(line + " " + rng + " " + " ".join(tail))
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("asan") / "host_sanitize")
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2112_03804_amd", "csrc"),
           os.path.join(ROOT, "tests", "cpp", "host_sanitize.cpp"),
           os.path.join(ROOT, "paper_2112_03804_amd", "csrc", "host_build.cpp"),
           os.path.join(ROOT, "paper_2112_03804_amd", "csrc", "host_sparsify.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("the sanitizer runtime is not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return exe


CASES = [
    ("kuhn_tiny", lambda: [I.kuhn(), I.tiny_config()]),
    ("small_rivers", lambda: [I.small_river(0), I.small_river(5, deck_size=11, n_keep=(20, 13))]),
    ("turn_games", lambda: [I.small_turn_river(0),
                            I.small_turn_river(4, deck_size=10, n_board=3, cards_per_hand=2,
                                               bet_fracs=(0.5, 1.0), max_raises=1, stack=30.0, zero_frac=0.2)]),
    ("river", lambda: [I.config(1)]),
    ("small_river_alone", lambda: [I.small_river(5, deck_size=11, n_keep=(20, 13))]),
    ("uneven_batch", lambda: I.batched_configs(16)),
    ("libratus_menu", lambda: [I.libratus_river(stack=1000.0, n_keep=(300, 250)),
                               I.libratus_river(seed=3, ai=1, stack=400.0, n_keep=(40, 60))]),
    ("ragged", lambda: [I.river_config(seed=41, n_keep=(2, 3), bet_fracs=(1.0,), max_raises=1),
                        I.river_config(seed=42, deck_size=57, n_keep=(1280, 1277), bet_fracs=(0.5,),
                                       max_raises=1)]),
]


@pytest.mark.parametrize("name,fn", CASES)
def test_host_builder_is_clean_under_sanitizers(sanitized, name, fn, tmp_path):
    path = str(tmp_path / "descs.txt")
    _write(fn(), path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sanitized, path], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (name, r.stdout[-500:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.startswith("ok"), r.stdout
