"""Benchmark: matvec pairs/s and time to gap 1e-4 * pot on one MI355X.

A step is one alternating RM+ iteration of the whole hot path on the river
endgame (52-card deck, 5-card board, 1081 hands per player, bets
{0.5, 1, 2} x pot + all-in, 3 raises): the structured product A y, Player 1's
treeplex update, A^T x, Player 2's update.  Each step performs exactly one
matvec pair, so `value` (pairs/s) is whole-job iterations per second with all
inputs resident in HBM.  Extra fields report the isolated matvec-pair kernel
(its roofline), the time to a saddle gap of 1e-4 * pot from a uniform start,
and the CPU oracle timed on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published


def algorithmic_bytes_pair(layouts):
    """Bytes one matvec pair must move: read y and x, write A y and A^T x
    (FP32, n_seq x n_hands each), plus 16 B of hand metadata per hand and
    direction (positions, cards, weight)."""
    tot = 0
    for L in layouts:
        for p in range(2):
            tot += 2 * 4 * L[p]["n_seq"] * L[p]["n_hands"]
            tot += 2 * 16 * L[p]["n_hands"]
    return tot


def cpu_baseline(desc, budget_s=15.0):
    """The oracle's FP64 matvec pair (A y and A^T x from the definition),
    timed on this host for about budget_s seconds."""
    from oracle import payoff
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    o = payoff.Game(desc)
    rng = np.random.default_rng(0)
    y = rng.random((o.S[1], o.N[1]))
    x = rng.random((o.S[0], o.N[0]))
    o.matvec_A(y)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.matvec_A(y)
        o.matvec_AT(x)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "matvec pairs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} FP64 matvec pairs of the river endgame (definition-level sum over "
                      f"61 terminals x 1081 x 1081 hand pairs), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    from paper_2112_03804_amd import instances as I
    from paper_2112_03804_amd import pmx

    desc = I.config(1)
    pot = 2 * desc.contrib
    stream = torch.cuda.current_stream()
    t_create = time.perf_counter()
    g = pmx.Game(desc)
    t_create = time.perf_counter() - t_create

    # ---- whole hot path: K solver iterations (one matvec pair each) --------
    g.solver_reset()
    g.solver_step(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.solver_step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    value = args.steps / (ms / 1e3)

    # ---- the matvec-pair kernel alone (roofline) ---------------------------
    rng = np.random.default_rng(1)
    L = [g.layouts[0]]
    y = torch.from_numpy(rng.random(g.elems[1]).astype(np.float32)).cuda()
    x = torch.from_numpy(rng.random(g.elems[0]).astype(np.float32)).cuda()
    Ay = torch.empty(g.elems[0], dtype=torch.float32, device="cuda")
    ATx = torch.empty(g.elems[1], dtype=torch.float32, device="cuda")
    for _ in range(50):
        g.matvec_pair(y, x, Ay, ATx)
    reps = 2000
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        g.matvec_pair(y, x, Ay, ATx)
    e1.record(stream)
    torch.cuda.synchronize()
    pair_us = e0.elapsed_time(e1) * 1e3 / reps
    bytes_pair = algorithmic_bytes_pair(L)
    achieved = bytes_pair / (pair_us * 1e-6) / 1e9

    # ---- time to gap 1e-4 * pot from a uniform start -----------------------
    target = 1e-4 * pot
    g.solver_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    gap = float("inf")
    while iters < 200000:
        g.solver_step(25)
        iters += 25
        gap = float(g.saddle_gap()[0][0])
        if gap <= target:
            break
    ttg = time.perf_counter() - t0

    out = {
        "metric": "matvec pairs/s (A·y+Aᵀx) & time to gap 1e-4·pot: plain vs batched/warm-start",
        "value": value,
        "unit": "matvec pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 scan accumulation)",
        "data": "synthetic",
        "config": {"workload": "river endgame: 52-card deck, 5-card board, 1081 hands/player, "
                               "bets {0.5,1,2}xpot + all-in, max 3 raises, pot 100, stacks 400; "
                               "step = one RM+ iteration (A y, P1 update, A^T x, P2 update)",
                   "n_seq": [L[0][0]["n_seq"], L[0][1]["n_seq"]],
                   "n_hands": [L[0][0]["n_hands"], L[0][1]["n_hands"]]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_matvec (matvec_pair launch)", "us_per_launch": pair_us,
                     "algorithmic_bytes_per_launch": bytes_pair},
        "time_to_gap": {"target": "1e-4*pot", "seconds": ttg, "iterations": iters,
                        "gap_over_pot": gap / pot, "solver": "plain RM+, uniform start, "
                        "FP64 gap checked every 25 iterations"},
        "game_create_s": t_create,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(desc, args.cpu_budget)
    g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
