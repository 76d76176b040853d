"""Schedule autotuner for the structured matvec.

For a game it times every candidate schedule (``game_tune(kernel, rows)``:
kernel 2 / 3 = chunk-aligned scan layout with 256- / 512-thread workgroups,
rows = output rows per chunk; kernel 4 = grouped layout, rows = groups of
up to four input rows per chunk; each launched per hands-per-thread class)
on A y followed by A^T x (two single-direction launches, as the solver
makes them), or on whole solver iterations, with HIP events, keeps the
fastest, and remembers the choice in a JSON cache keyed by GPU architecture,
a size class of the game (instances, rows, largest hand count) and the
objective, so later games of the same class are tuned without timing.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Tuple

import numpy as np

DEFAULT_CANDIDATES = [(2, 1), (2, 4), (2, 8), (3, 1), (3, 4), (3, 8), (4, 1), (4, 2), (4, 4)]
CACHE_ENV = "PMX_TUNE_CACHE"


def _bucket(v: int, edges: Iterable[int]) -> int:
    for i, e in enumerate(edges):
        if v <= e:
            return i
    return len(list(edges))


def signature(game) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    rows = sum(max(L[0]["n_seq"], L[1]["n_seq"]) for L in game.layouts)
    nmax = max(max(L[0]["n_hands"], L[1]["n_hands"]) for L in game.layouts)
    return "|".join([arch, f"inst{_bucket(game.n_instances, (1, 16, 128, 1024))}",
                     f"rows{_bucket(rows, (256, 2048, 16384, 65536))}",
                     f"hands{_bucket(nmax, (512, 1024, 1280))}"])


def _load(path: str) -> Dict[str, list]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_schedule(game, kernel: int, rows: int, reps: int = 20, pair: bool = False) -> float:
    """Average microseconds of A y followed by A^T x under a schedule: two
    single-direction launches, as the solver makes them (or, with `pair`,
    one matvec-pair launch)."""
    import torch
    game.game_tune(kernel, rows)
    rng = np.random.default_rng(0)
    y = torch.from_numpy(rng.random(game.elems[1]).astype(np.float32)).cuda()
    x = torch.from_numpy(rng.random(game.elems[0]).astype(np.float32)).cuda()
    Ay = torch.empty(game.elems[0], dtype=torch.float32, device="cuda")
    ATx = torch.empty(game.elems[1], dtype=torch.float32, device="cuda")
    def once():
        if pair:
            game.matvec_pair(y, x, Ay, ATx)
        else:
            game.matvec_A(y, Ay)
            game.matvec_AT(x, ATx)

    for _ in range(3):
        once()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        once()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def time_iterations(game, kernel: int, rows: int, iters: int = 256) -> float:
    """Average microseconds of one solver iteration under a schedule (the
    graph-replayed sequence A y, Player 1's update, A^T x, Player 2's
    update), from a uniform start after one captured warm-up; the solver is
    left reset."""
    import torch
    game.game_tune(kernel, rows)
    game.solver_reset()
    game.solver_step(32)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    game.solver_step(iters)
    e1.record(s)
    torch.cuda.synchronize()
    game.solver_reset()
    return e0.elapsed_time(e1) * 1e3 / iters


def tune(game, candidates=None, reps: int = 20, cache_path: Optional[str] = None,
         use_cache: bool = True, objective: str = "products") -> Tuple[Tuple[int, int], Dict[str, float]]:
    """Pick and apply the fastest schedule.  Returns ((kernel, rows), timings).
    objective "products" times A y then A^T x (time_schedule); "iteration"
    times whole solver iterations (time_iterations; resets the solver), which
    also sees how the products overlap the regret updates in the graph."""
    if objective not in ("products", "iteration"):
        raise ValueError(f"unknown objective {objective!r}")
    cache_path = cache_path or os.environ.get(CACHE_ENV)
    key = signature(game) + ("" if objective == "products" else "|iteration")
    cache = _load(cache_path) if cache_path else {}
    if use_cache and key in cache:
        k, r = cache[key]
        game.game_tune(int(k), int(r))
        return (int(k), int(r)), {}
    timings = {}
    for k, r in (candidates or DEFAULT_CANDIDATES):
        timings[f"{k}:{r}"] = (time_schedule(game, k, r, reps) if objective == "products"
                               else time_iterations(game, k, r))
    best = min(timings, key=timings.get)
    k, r = (int(v) for v in best.split(":"))
    game.game_tune(k, r)
    if cache_path:
        cache[key] = [k, r]
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return (k, r), timings
