"""Solver checkpoints on disk.

A checkpoint is one ``.npz`` file (plain arrays, no pickled objects) holding
everything the solver's next iteration depends on: per player the regrets,
the current plan and the weighted sums of the average strategy, the iteration
count and the weight total, each instance's own weight total (instances that
retired early stop accumulating), the active flags, the solver parameters and
the matvec schedule.  The game's shape (per instance and player: sequences,
hands, row stride) is stored too, and a checkpoint is only loaded into a game
of the same shape.
"""
from __future__ import annotations

import json
from typing import Optional

import numpy as np

FORMAT = "pmx-solver-checkpoint"
VERSION = 1


def game_shape(game) -> np.ndarray:
    """int64 [instances, 6]: (sequences, hands, stride) of player 1, then of player 2."""
    return np.array([[L[p][k] for p in range(2) for k in ("n_seq", "n_hands", "stride")] for L in game.layouts],
                    dtype=np.int64)


def save(game, path: str, params: Optional[dict] = None, active=None) -> None:
    """Write the game's solver state to ``path`` (.npz).  ``params``: the
    solver parameters in force (``{"kind": "rm+"}`` or ``{"kind": "dcfr",
    "alpha": .., "beta": .., "gamma": ..}``), ``active``: the instance flags
    (None: all active)."""
    st = [game.solver_get_state(p) for p in range(2)]
    n = game.n_instances
    act = np.ones(n, np.int32) if active is None else np.ascontiguousarray(active, np.int32)
    if act.shape != (n,):
        raise ValueError("one active flag per instance")
    meta = {"format": FORMAT, "version": VERSION, "params": params or {"kind": "rm+"},
            "t": int(st[0]["t"]), "wsum": float(st[0]["wsum"]), "tuning": list(game.game_get_tuning())}
    with open(path, "wb") as f:
        np.savez(f, meta=np.array(json.dumps(meta)), shape=game_shape(game), weights=game.solver_get_weights(),
                 active=act,
                 regret0=st[0]["regret"], plan0=st[0]["plan"], avg0=st[0]["avg_sum"],
                 regret1=st[1]["regret"], plan1=st[1]["plan"], avg1=st[1]["avg_sum"])


def read(path: str) -> dict:
    """The checkpoint's arrays and metadata, checked for format and version."""
    with np.load(path, allow_pickle=False) as z:
        data = {k: z[k] for k in z.files}
    try:
        meta = json.loads(str(data.pop("meta")))
    except (KeyError, ValueError) as e:
        raise ValueError(f"{path}: not a solver checkpoint") from e
    if meta.get("format") != FORMAT or meta.get("version") != VERSION:
        raise ValueError(f"{path}: format {meta.get('format')!r} version {meta.get('version')!r} "
                         f"is not {FORMAT!r} version {VERSION}")
    data["meta"] = meta
    return data


def check_shape(game, data: dict) -> None:
    """Raise ValueError unless the checkpoint was written for a game of this shape."""
    want = game_shape(game)
    got = np.asarray(data["shape"])
    if got.shape != want.shape or not np.array_equal(got, want):
        raise ValueError("the checkpoint was written for a game of another shape "
                         f"({got.shape[0]} instances against {want.shape[0]}, or other sizes)")
    for p in range(2):
        for key, dt in (("regret", np.float32), ("plan", np.float32), ("avg", np.float64)):
            a = data[f"{key}{p}"]
            if a.shape != (game.elems[p],) or a.dtype != dt:
                raise ValueError(f"checkpoint array {key}{p} has shape {a.shape} / {a.dtype}")


def load(game, path: str) -> dict:
    """Restore a checkpoint into ``game`` (same shape): state, weights, active
    flags, solver parameters and schedule.  Returns the metadata."""
    data = read(path)
    check_shape(game, data)
    meta = data["meta"]
    k, r = meta["tuning"]
    game.game_tune(int(k), int(r))
    prm = dict(meta["params"])
    kind = prm.pop("kind", "rm+")
    game.solver_set_params(kind, **prm)
    for p in range(2):
        game.solver_set_state(p, regret=data[f"regret{p}"], plan=data[f"plan{p}"], avg_sum=data[f"avg{p}"],
                              t=meta["t"], wsum=meta["wsum"])
    game.solver_set_weights(data["weights"])
    game.solver_set_active(data["active"])
    return meta
