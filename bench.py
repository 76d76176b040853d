"""Benchmark: matvec pairs/s and time to gap 1e-4 * pot on one MI355X.

A step is one alternating RM+ iteration of the whole hot path over the batch
of 512 uneven river endgames (hands U[200, 1081] per player, 1-3 bet sizes,
raise caps 2-4, pots U[20, 400], stack/pot U[1, 10]), all in one game: the
structured products A y of every instance, Player 1's treeplex updates,
A^T x, Player 2's updates.  Each step performs one matvec pair per instance,
so `value` (instance matvec pairs/s) is 512 x steps per second with all
inputs resident in HBM.  Extra fields report the isolated matvec-pair kernel
on the batch (its roofline), the batch's time to a saddle gap of
1e-4 * pot against the plain single-instance solver run on every one of the
512 instances, the learned warm start, the single river endgame, the
turn + river precision run, and the CPU oracle timed on this host.

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

# HBM bytes per matvec-pair launch from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE), each scaled by what the counter reads for a plain copy of
# known size (profiles/matvec_pair_traffic_counters.md).  They describe the
# kernel sources whose code (comments and whitespace removed) has the SHA-1
# recorded here and are reported as null for any other version of that code.
TRAFFIC = {"sources_sha1": "c20201a0c633536cff3f342b511300e6ece60a70",
           "river": {"4:1": 1421393, "3:1": 1623947},
           "batch": {"4:1": 351616011, "4:2": 351270363}}
TRAFFIC_SOURCES = ("paper_2112_03804_amd/csrc/pmx_device.hip", "paper_2112_03804_amd/csrc/host_build.cpp")
# the schedules of the counter probe (the autotuner's usual choices; traffic
# is reported for these only) and the batch schedule of the trace probe
PROBE_RIVER_SCHEDULES = ((4, 1), (3, 1))
PROBE_BATCH_SCHEDULES = ((4, 1), (4, 2))
PROBE_BATCH_SCHEDULE = (4, 1)


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def sources_sha1(root=None):
    """SHA-1 of the kernel sources' code: comments and whitespace removed, so
    that an edit of the comments keeps the measured traffic."""
    import hashlib
    import re
    h = hashlib.sha1()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(root or ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def kernel_label(sched):
    """The matvec kernel a schedule (kernel, rows) launches."""
    k, r = int(sched[0]), int(sched[1])
    if k == 4:
        return f"k_mvg (matvec_pair launch, schedule 4:{r}, grouped layout)"
    return f"k_mvc (matvec_pair launch, schedule {k}:{r}, chunk-aligned layout)"


def measured_traffic(key, sched=None):
    """The counted HBM bytes of a matvec-pair launch, or None when the
    kernel sources differ from those the counters were taken with or the
    schedule is not one of those counted."""
    if TRAFFIC["sources_sha1"] != sources_sha1():
        return None
    v = TRAFFIC.get(key)
    if isinstance(v, dict):
        return v.get(f"{sched[0]}:{sched[1]}") if sched is not None else None
    return v


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


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, river_desc, batch_descs, gpu_iters=None, precision=None):
    """The oracle on this host's cores (a reported baseline, not the target):

    * its FP64 matvec pairs (A y and A^T x from the definition, summed over
      terminals and hand pairs) on an even sample of the batch's instances,
      each timed in turn for about --cpu-budget seconds in all: instance
      pairs per second on that sample, the headline's unit;
    * the same on the single river endgame, with its thread pool and on one
      thread, and the oracle's river time to 1e-4 * pot extrapolated from
      that rate and the GPU solver's iteration count;
    * the 13-card game solved by the oracle's FP64 RM+ to 1e-6 * pot;
    * the oracle's FP64 saddle gap of the turn + river precision run's
      averages, beside the GPU's (the error the precision run reports)."""
    from oracle import payoff
    from oracle import solver as osolver
    from paper_2112_03804_amd import instances as I
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = 1
    budget_s = args.cpu_budget
    rng = np.random.default_rng(0)

    # batch sample: one pair per sampled instance, round robin, until the budget
    step = max(1, len(batch_descs) // args.cpu_batch_sample)
    idx = list(range(0, len(batch_descs), step))[:args.cpu_batch_sample]
    games = []
    for i in idx:
        o = payoff.Game(batch_descs[i])
        games.append((o, rng.random((o.S[1], o.N[1])), rng.random((o.S[0], o.N[0]))))
    n_pairs, t_used = 0, 0.0
    t0 = time.perf_counter()
    while n_pairs == 0 or time.perf_counter() - t0 < budget_s:
        for o, y, x in games:
            o.matvec_A(y)
            o.matvec_AT(x)
            n_pairs += 1
    t_used = time.perf_counter() - t0
    out = {"value": n_pairs / t_used, "unit": "instance matvec pairs/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{len(idx)} of the batch's {len(batch_descs)} instances (one in {step}), "
                     f"{n_pairs // len(idx)} FP64 matvec pairs each (definition-level sums over terminals x "
                     f"hand pairs), {t_used:.1f} s",
           "host": {"nproc": os.cpu_count(), "model": _cpu_model()}}
    del games

    # the single river endgame
    o = payoff.Game(river_desc)
    y = rng.random((o.S[1], o.N[1]))
    x = rng.random((o.S[0], o.N[0]))
    o.matvec_A(y)

    def rate(budget):
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget:
            o.matvec_A(y)
            o.matvec_AT(x)
            n += 1
        return n, time.perf_counter() - t0

    n, dt = rate(max(2.0, budget_s / 3))
    river = {"value": n / dt, "unit": "matvec pairs/s", "cores": int(threads),
             "sample": f"{n} FP64 matvec pairs of the river endgame, {dt:.1f} s"}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            n1, dt1 = rate(max(2.0, budget_s / 6))
        river["single_thread"] = {"value": n1 / dt1, "unit": "matvec pairs/s", "sample": f"{n1} pairs, {dt1:.1f} s"}
    if gpu_iters:
        river["time_to_gap_extrapolated"] = {
            "target": "1e-4*pot", "iterations": gpu_iters, "seconds": gpu_iters / (n / dt),
            "note": "the GPU solver's RM+ iteration count times the oracle's time per matvec pair "
                    "(regret updates and gap checks not counted)"}
    out["river"] = river
    # the 13-card game solved by the oracle's plain FP64 RM+ (gap every 100
    # iterations, stopped after 10 s)
    if not args.no_tiny:
        tiny = I.config(0)
        ot = payoff.Game(tiny)
        pot = 2 * tiny.contrib
        sol = osolver.RMPlus(ot)
        t0 = time.perf_counter()
        it, gap = 0, float("inf")
        while it < 200000 and time.perf_counter() - t0 < 10.0:
            for _ in range(100):
                sol.step()
            it += 100
            gap = float(sol.gap()[0])
            if gap <= 1e-6 * pot:
                break
        out["tiny_time_to_gap"] = {"target": "1e-6*pot", "seconds": time.perf_counter() - t0, "iterations": it,
                                   "gap_over_pot": gap / pot, "reached": gap <= 1e-6 * pot}
    # the oracle's gap of the precision run's averages
    if precision is not None:
        xa, ya = precision["averages"]
        od = payoff.Game(I.config(2))
        t0 = time.perf_counter()
        rgap, rb1, rb2 = osolver.saddle_gap(od, xa, ya)
        pot = 2 * od.desc.contrib
        out["precision_run_oracle_gap"] = {"gap_over_pot": rgap / pot, "br1": rb1, "br2": rb2,
                                           "seconds": time.perf_counter() - t0}
    return out


def batched_leg(args, stream):
    """The headline workload: 512 uneven river endgames in one game.  The
    timed steps (whole solver iterations over the batch), the matvec-pair
    kernel's roofline over the batch, the batched time to 1e-4 * pot for
    every instance, and the plain single-instance solver on every instance
    of the same batch (or on an even sample of --plain-sample of them)."""
    import torch
    from paper_2112_03804_amd import autotune
    from paper_2112_03804_amd import instances as I
    from paper_2112_03804_amd import pmx
    from paper_2112_03804_amd import warmstart as ws

    descs = I.load_json(args.instances) if args.instances else I.batched_configs(args.batch)
    t_create = time.perf_counter()
    g = pmx.Game(descs)
    t_create = time.perf_counter() - t_create
    L = g.layouts
    default_sched = g.game_get_tuning()
    # the schedule of the fastest solver iteration (the headline's unit)
    sched, sched_us = autotune.tune(g, use_cache=False, objective="iteration")
    log(f"batch: {len(descs)} instances, schedule {sched}; {args.warmup} warm-up and {args.steps} timed steps")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # ---- the timed steps: whole solver iterations over the batch ----------
    g.solver_reset()
    g.solver_step(args.warmup)
    torch.cuda.synchronize()
    e0.record(stream)
    g.solver_step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    it_ms = ms / args.steps
    # ---- the matvec pair alone (roofline) --------------------------------
    rng = np.random.default_rng(2)
    y = torch.from_numpy(rng.random(g.elems[1]).astype(np.float32)).cuda()
    x = torch.from_numpy(rng.random(g.elems[0]).astype(np.float32)).cuda()
    Ay = torch.empty(g.elems[0], dtype=torch.float32, device="cuda")
    ATx = torch.empty(g.elems[1], dtype=torch.float32, device="cuda")
    for _ in range(10):
        g.matvec_pair(y, x, Ay, ATx)
    reps = 200
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        g.matvec_pair(y, x, Ay, ATx)
    e1.record(stream)
    torch.cuda.synchronize()
    pair_us = e0.elapsed_time(e1) * 1e3 / reps
    bytes_pair = algorithmic_bytes_pair(L)
    achieved = bytes_pair / (pair_us * 1e-6) / 1e9
    del y, x, Ay, ATx
    # ---- batched time to gap: every instance at or below 1e-4 of its pot;
    # solved instances are retired from the iteration
    log(f"batch: {it_ms:.3f} ms per step, matvec pair {pair_us:.1f} us; solving to 1e-4 * pot")
    g.solver_reset()
    ttg_batched, iters, done_at = ws.solve_to_gap(g, 1e-4, check_every=32, max_iters=args.max_iters)
    log(f"batch: time to gap {ttg_batched:.2f} s ({iters} iterations); without retirement")
    g.solver_reset()
    ttg_noretire, iters_nr, _ = ws.solve_to_gap(g, 1e-4, check_every=32, max_iters=args.max_iters,
                                                retire=False)
    # the same with discounted CFR (the paper's solver family) instead of RM+
    log(f"batch: without retirement {ttg_noretire:.2f} s; DCFR")
    g.solver_set_params("dcfr")
    g.solver_reset()
    ttg_dcfr, iters_dcfr, _ = ws.solve_to_gap(g, 1e-4, check_every=32, max_iters=args.max_iters)
    g.solver_set_params("rm+")
    g.close()
    # ---- the plain single-instance solver on the same instances -----------
    n_plain = len(descs) if args.plain_sample <= 0 else min(args.plain_sample, len(descs))
    sample = list(range(0, len(descs), max(1, len(descs) // n_plain)))[:n_plain]
    log(f"batch: DCFR {ttg_dcfr:.2f} s; plain single-instance solver on {len(sample)} instances")
    plain_s, plain_it = [], []
    for k, i in enumerate(sample):
        gi = pmx.Game(descs[i])
        pot = 2 * descs[i].contrib
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it = 0
        while it < args.max_iters:
            gi.solver_step(32)
            it += 32
            if gi.saddle_gap()[0][0] <= 1e-4 * pot:
                break
        plain_s.append(time.perf_counter() - t0)
        plain_it.append(it)
        gi.close()
        if (k + 1) % 64 == 0:
            log(f"batch: plain solver, {k + 1}/{len(sample)} instances, {sum(plain_s):.1f} s")
    plain_total = float(np.sum(plain_s)) * (len(descs) / len(sample))
    big = None
    if args.batch_big > 0:
        # a batch four times larger than the Infinity Cache holds: the same
        # tuned schedule, the matvec pair alone
        log(f"batch: matvec pair on {args.batch_big} instances")
        gb = pmx.Game(I.batched_configs(args.batch_big))
        gb.game_tune(*sched)
        yb = torch.from_numpy(rng.random(gb.elems[1]).astype(np.float32)).cuda()
        xb = torch.from_numpy(rng.random(gb.elems[0]).astype(np.float32)).cuda()
        Ayb = torch.empty(gb.elems[0], dtype=torch.float32, device="cuda")
        ATxb = torch.empty(gb.elems[1], dtype=torch.float32, device="cuda")
        for _ in range(5):
            gb.matvec_pair(yb, xb, Ayb, ATxb)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(50):
            gb.matvec_pair(yb, xb, Ayb, ATxb)
        e1.record(stream)
        torch.cuda.synchronize()
        big_us = e0.elapsed_time(e1) * 1e3 / 50
        big_bytes = algorithmic_bytes_pair(gb.layouts)
        big_gbs = big_bytes / (big_us * 1e-6) / 1e9
        big = {"instances": args.batch_big, "schedule": list(sched), "us_per_launch": big_us,
               "algorithmic_bytes_per_launch": big_bytes, "achieved_gbs": big_gbs,
               "frac": big_gbs / HBM_PEAK_GBS}
        gb.close()
        del yb, xb, Ayb, ATxb
    n_seq = [[l[p]["n_seq"] for l in L] for p in range(2)]
    n_hands = [[l[p]["n_hands"] for l in L] for p in range(2)]
    return {
        "workload": (f"{len(descs)} instances of the spec {os.path.basename(args.instances)} in one game"
                     if args.instances else
                     f"{len(descs)} river endgames in one game: hands U[200,1081] per player, 1-3 bet "
                     "sizes from {0.33,0.5,0.75,1,1.5,2}xpot + all-in, raise caps 2-4, pots U[20,400], "
                     "stack/pot U[1,10]"),
        "instances": len(descs),
        "sizes": {"sequences_per_player_mean": [float(np.mean(s)) for s in n_seq],
                  "hands_per_player_mean": [float(np.mean(h)) for h in n_hands],
                  "entries_per_vector_total": [int(sum(a * b for a, b in zip(n_seq[p], n_hands[p])))
                                               for p in range(2)]},
        "game_create_s": t_create,
        "schedule": {"default": list(default_sched), "tuned": list(sched),
                     "us_per_iteration_by_schedule": sched_us},
        "steps": args.steps, "warmup": args.warmup, "ms": ms,
        "iteration_ms": it_ms,
        "matvec_pairs_per_s": len(descs) / (it_ms * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None if args.instances else measured_traffic("batch", sched),
                     "kernel": kernel_label(sched),
                     "us_per_launch": pair_us, "algorithmic_bytes_per_launch": bytes_pair},
        "time_to_gap_batched_s": ttg_batched,
        "time_to_gap_batched_no_retirement_s": ttg_noretire,
        "time_to_gap_batched_dcfr_s": ttg_dcfr,
        "iterations_batched_dcfr": iters_dcfr,
        "iterations_batched": iters,
        "instances_reached": int((done_at >= 0).sum()),
        "iterations_per_instance_p50_p90_max": [float(np.percentile(done_at[done_at > 0], q))
                                                for q in (50, 90, 100)] if (done_at > 0).any() else None,
        "plain_single_instance": {"instances": len(sample), "of": len(descs),
                                  "sum_s": float(np.sum(plain_s)), "mean_s": float(np.mean(plain_s)),
                                  "mean_iterations": float(np.mean(plain_it)),
                                  "sum_over_batch_s": plain_total,
                                  "extrapolated": len(sample) < len(descs),
                                  "solver": "plain RM+ on one instance, uniform start, FP64 gap every 32 "
                                            "iterations"},
        "speedup_batched_vs_plain": plain_total / ttg_batched,
        "speedup_batched_dcfr_vs_plain": plain_total / ttg_dcfr,
        "matvec_pair_beyond_infinity_cache": big,
    }


def turn_river_leg(args, stream):
    """The turn + river endgame: one instance of 19,480 sequences x 1128 hands
    per player (352 MB per matvec pair): tuned matvec-pair roofline, solver
    iteration time, and the precision run: discounted CFR from a uniform
    start toward an FP64 saddle gap of 1e-8 * pot, the gap checked at doubling
    iteration counts up to 16384 and every 2048 after, within a time budget."""
    import torch
    from paper_2112_03804_amd import autotune
    from paper_2112_03804_amd import instances as I
    from paper_2112_03804_amd import pmx

    desc = I.config(2)
    t_create = time.perf_counter()
    g = pmx.Game(desc)
    t_create = time.perf_counter() - t_create
    sched, sched_us = autotune.tune(g, candidates=[(2, 4), (2, 8), (3, 4), (3, 8), (4, 1), (4, 2)], reps=10,
                                    use_cache=False)
    bytes_pair = algorithmic_bytes_pair(g.layouts)
    pair_us = autotune.time_schedule(g, *sched, reps=20, pair=True)   # the matvec-pair launch (roofline)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g.solver_reset()
    g.solver_step(4)
    torch.cuda.synchronize()
    e0.record(stream)
    g.solver_step(args.turn_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    it_ms = e0.elapsed_time(e1) / args.turn_steps
    gap = float(g.saddle_gap()[0][0])
    # precision run
    pot = 2 * desc.contrib
    g.solver_set_params("dcfr")
    g.solver_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, nxt, traj, reached = 0, 256, [], False
    while True:
        g.solver_step(nxt - it)
        it = nxt
        gp = float(g.saddle_gap()[0][0]) / pot
        el = time.perf_counter() - t0
        traj.append([it, round(el, 3), gp])
        log(f"turn+river precision run: {it} iterations, {el:.1f} s, gap/pot {gp:.3e}")
        if gp <= 1e-8:
            reached = True
            break
        # next check: double up to 16384 iterations, then every 2048 (a check
        # costs a few ms), within what the measured rate allows in budget
        per_it = el / it
        left = args.turn_budget - el
        if left < 256 * per_it:
            break
        nxt = it + min(it if it < 16384 else 2048, int(left / per_it) // 256 * 256)
    out = {"workload": "turn + river endgame: 4-card board, 48 river cards, 1128 hands/player, "
                       "bets {0.33,0.75,1.5}xpot + all-in, max 3 raises per street, pot 100, stacks 400",
           "game_create_s": t_create,
           "schedule": {"tuned": list(sched), "us_A_then_AT_by_schedule": sched_us},
           "roofline": {"bound": "hbm", "achieved": bytes_pair / (pair_us * 1e-6) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": bytes_pair / (pair_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                        "kernel": kernel_label(sched),
                        "us_per_launch": pair_us, "algorithmic_bytes_per_launch": bytes_pair},
           "matvec_pairs_per_s": 1e6 / pair_us,
           "iteration_ms": it_ms,
           "gap_over_pot_after": {"iterations": 4 + args.turn_steps, "gap_over_pot": gap / (2 * desc.contrib)},
           "precision_run": {"solver": "DCFR (alpha 1.5, beta 0, gamma 2), uniform start, FP32 gradients "
                                       "with FP64-carried scans; gap from FP64 matvecs and FP64 best responses",
                             "target_gap_over_pot": 1e-8, "reached": reached,
                             "iterations": it, "seconds": traj[-1][1], "gap_over_pot": traj[-1][2],
                             "trajectory_iters_s_gap": traj, "budget_s": args.turn_budget}}
    # the run's FP64 averages, for the oracle's gap on the host
    out["_averages"] = (g.unpack(0, g.get_average_strategy(0))[0], g.unpack(1, g.get_average_strategy(1))[0])
    g.close()
    return out


def warm_leg(args, stream, batched):
    """Learned warm start on the batched workload: label instances with the
    plain batched solver (to --warm-label-gap of the pot), train the BF16
    network on the GPU, then solve the 512 held-out instances (the batched
    workload) from the network's prior under RM+ and under DCFR, each with
    the uniform start as the per-instance fallback (a probe of both starts;
    an instance keeps the prior only where its FP64 gap is finite and below
    the uniform start's).  `batched` holds the uniform-start baselines of the
    same instances; None measures them here."""
    import torch
    from paper_2112_03804_amd import instances as I
    from paper_2112_03804_amd import pmx
    from paper_2112_03804_amd import warmstart as ws

    t0 = time.perf_counter()
    train_descs = I.batched_configs(args.warm_train, seed=11)
    ds = ws.make_dataset(train_descs, batch=512, target=args.warm_label_gap, kind=args.warm_label_kind,
                         max_iters=args.warm_label_iters,
                         progress=lambda a, n: log(f"warm start: labelled {a}/{n} instances"))
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = ws.WarmMLP(seed=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"warm start: {ds.rows} rows; training")
    hist = ws.train(net, ds, steps=args.warm_steps, batch_rows=8192, lr=1e-3,
                    log_every=max(1, args.warm_steps // 10),
                    progress=lambda st, ls: log(f"warm start: step {st}, loss {ls:.4f}"))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    rows_trained = args.warm_steps * 8192
    flops_per_row = 2 * (ws.D_IN * ws.WIDTH + ws.WIDTH * ws.WIDTH + ws.WIDTH * ws.K) * 3   # forward + backward
    n_rows = ds.rows
    del ds
    descs = I.batched_configs(args.batch)
    g = pmx.Game(descs)
    g.game_tune(4, 1)
    base = {}
    if batched is None:
        for kind in ("rm+", "dcfr"):
            g.solver_set_params(kind)
            g.solver_reset()
            base[kind], _, _ = ws.solve_to_gap(g, 1e-4, check_every=32, max_iters=args.max_iters)
            log(f"warm start: uniform {kind} {base[kind]:.2f} s")
    else:
        base = {"rm+": batched["time_to_gap_batched_s"], "dcfr": batched["time_to_gap_batched_dcfr_s"]}
    res = {}
    for kind in ("rm+", "dcfr"):
        g.solver_set_params(kind)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        keep, gap_u, gap_w = ws.apply_prior_with_fallback(g, net, args.warm_scale, args.warm_avg,
                                                          probe=args.warm_probe)
        sec, iters, done = ws.solve_to_gap(g, 1e-4, check_every=32, max_iters=args.max_iters,
                                           start_iters=args.warm_probe)
        t_warm = time.perf_counter() - t2
        r = {"time_to_gap_warm_batched_s": t_warm, "iterations": iters,
             "instances_reached": int((done >= 0).sum()),
             "instances_kept_prior": int(keep.sum()),
             "probe_iterations": args.warm_probe,
             "iterations_per_instance_p50_p90_max": [float(np.percentile(done[done >= 0], q))
                                                     for q in (50, 90, 100)] if (done >= 0).any() else None,
             "speedup_vs_batched_uniform": base[kind] / t_warm,
             "time_to_gap_batched_uniform_s": base[kind]}
        if batched is not None:
            r["speedup_vs_plain_single_instance_rm+"] = (batched["plain_single_instance"]["sum_over_batch_s"]
                                                         / t_warm)
        res[kind] = r
        log(f"warm start: {kind} {t_warm:.2f} s from the prior ({int(keep.sum())} of {len(keep)} kept it)")
    g.solver_set_params("rm+")
    g.close()
    return {"workload": f"network trained on {len(train_descs)} synthetic river endgames drawn as the batch "
                        f"(other seeds), evaluated on the batch's {args.batch} instances",
            "train_instances": len(train_descs),
            "labels": f"average strategies of the plain batched {args.warm_label_kind.upper()} solver run to "
                      f"{args.warm_label_gap:g} * pot (at most {args.warm_label_iters} iterations)",
            "dataset_rows": n_rows, "data_s": t_data,
            "train_steps": args.warm_steps, "train_rows_per_step": 8192, "train_s": t_train,
            "loss_history": hist,
            "train_tflops": rows_trained * flops_per_row / t_train / 1e12,
            "prior": {"regret_scale": args.warm_scale, "avg_weight": args.warm_avg,
                      "fallback": "uniform start per instance, judged by the FP64 gap after the probe"},
            "rm+": res["rm+"], "dcfr": res["dcfr"]}


def pmc_probe(args):
    """Launches for hardware-counter runs (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE):
    a plain 256 MiB device-to-device copy (known bytes: calibrates the counters),
    then matvec-pair launches on the river endgame at each of
    PROBE_RIVER_SCHEDULES and on the batch at each of PROBE_BATCH_SCHEDULES."""
    import torch
    from paper_2112_03804_amd import instances as I
    from paper_2112_03804_amd import pmx
    n = 64 << 20
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    games = [(f"river {sc[0]}:{sc[1]}", pmx.Game(I.config(1)), sc) for sc in PROBE_RIVER_SCHEDULES]
    for sc in PROBE_BATCH_SCHEDULES:
        games.append((f"batch {sc[0]}:{sc[1]}", pmx.Game(I.batched_configs(args.batch)), sc))
    for name, g, sc in games:
        g.game_tune(*sc)
        rng = np.random.default_rng(0)
        y = torch.from_numpy(rng.random(g.elems[1]).astype(np.float32)).cuda()
        x = torch.from_numpy(rng.random(g.elems[0]).astype(np.float32)).cuda()
        Ay = torch.empty(g.elems[0], dtype=torch.float32, device="cuda")
        ATx = torch.empty(g.elems[1], dtype=torch.float32, device="cuda")
        for _ in range(10):
            g.matvec_pair(y, x, Ay, ATx)
        torch.cuda.synchronize()
        print(json.dumps({"probe": name, "algorithmic_bytes_per_launch": algorithmic_bytes_pair(g.layouts),
                          "copy_bytes_each_way": 4 * n}), flush=True)
        g.close()


def trace_probe(args):
    """Launches for a kernel trace of the solver iteration: the batch, the turn
    + river game, the river endgame and the river with Libratus' sizes, each
    at the schedule the bench's autotuner picks there (``--trace-game``
    selects one), a few graph-captured iterations after a warm-up, then one
    FP64 gap."""
    import torch
    from paper_2112_03804_amd import instances as I
    from paper_2112_03804_amd import pmx
    games = (("batch", lambda: pmx.Game(I.batched_configs(args.batch)), PROBE_BATCH_SCHEDULE, 64),
             ("turn_river", lambda: pmx.Game(I.config(2)), (3, 8), 32),
             ("river", lambda: pmx.Game(I.config(1)), (3, 1), 64),
             ("libratus_river", lambda: pmx.Game(I.libratus_river(stack=1000.0)), (3, 1), 64))
    for name, make, sched, iters in games:
        if args.trace_game and name != args.trace_game:
            continue
        g = make()
        g.game_tune(*sched)
        g.solver_reset()
        g.solver_step(32)
        torch.cuda.synchronize()
        g.solver_step(iters)
        torch.cuda.synchronize()
        g.saddle_gap()
        torch.cuda.synchronize()
        print(json.dumps({"probe": name, "schedule": list(sched), "iterations": 32 + iters}), flush=True)
        g.close()


def dcfr_sweep(args):
    """Discounted CFR parameters (Section 5 names the solver, not its
    parameters): time and iterations to 1e-4 * pot for alpha in {1, 1.5, 2},
    beta in {0, 0.5}, gamma in {1, 2, 3} (and RM+ beside them) on the river
    endgame and on the batch of 512 endgames (instances retire at the
    target); then RM+ against DCFR (1.5, 0, 2) to 1e-6 * pot on the turn +
    river game.  One JSON line per measurement, then a summary line."""
    import torch
    from paper_2112_03804_amd import instances as I
    from paper_2112_03804_amd import pmx
    from paper_2112_03804_amd import warmstart as ws

    grid = [(a, b, c) for a in (1.0, 1.5, 2.0) for b in (0.0, 0.5) for c in (1, 2, 3)]
    rows = []

    def emit(row):
        rows.append(row)
        print(json.dumps(row), flush=True)

    # river endgame: one instance, FP64 gap every 25 iterations
    desc = I.config(1)
    pot = 2 * desc.contrib
    g = pmx.Game(desc)
    g.solver_set_gap_guard(0)   # some settings are not monotone for long stretches
    for kind, prm in [("rm+", None)] + [("dcfr", p) for p in grid]:
        if prm:
            g.solver_set_params("dcfr", *prm)
        else:
            g.solver_set_params("rm+")
        g.solver_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, gap = 0, float("inf")
        while it < 200000:
            g.solver_step(25)
            it += 25
            gap = float(g.saddle_gap()[0][0])
            if gap <= 1e-4 * pot:
                break
        emit({"game": "river", "solver": kind, "alpha_beta_gamma": prm, "target": "1e-4*pot",
              "seconds": time.perf_counter() - t0, "iterations": it, "gap_over_pot": gap / pot})
    g.close()

    # the batch of 512 endgames
    g = pmx.Game(I.batched_configs(args.batch))
    g.game_tune(4, 1)
    g.solver_set_gap_guard(0)
    for kind, prm in [("rm+", None)] + [("dcfr", p) for p in grid]:
        if prm:
            g.solver_set_params("dcfr", *prm)
        else:
            g.solver_set_params("rm+")
        g.solver_reset()
        sec, iters, done = ws.solve_to_gap(g, 1e-4, check_every=32, max_iters=min(args.max_iters, 40000))
        emit({"game": f"batch of {args.batch}", "solver": kind, "alpha_beta_gamma": prm, "target": "1e-4*pot",
              "seconds": sec, "iterations": iters, "instances_reached": int((done >= 0).sum()),
              "iterations_per_instance_mean": float(done[done >= 0].mean()) if (done >= 0).any() else None})
    g.close()

    # turn + river: RM+ against DCFR to 1e-6 * pot
    desc = I.config(2)
    pot = 2 * desc.contrib
    g = pmx.Game(desc)
    g.game_tune(3, 8)
    g.solver_set_gap_guard(0)
    for kind, prm in (("rm+", None), ("dcfr", (1.5, 0.0, 2))):
        if prm:
            g.solver_set_params("dcfr", *prm)
        else:
            g.solver_set_params("rm+")
        g.solver_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, gap, traj = 0, float("inf"), []
        while time.perf_counter() - t0 < args.turn_budget:
            g.solver_step(256)
            it += 256
            gap = float(g.saddle_gap()[0][0])
            if it % 2048 == 0:
                traj.append([it, round(time.perf_counter() - t0, 3), gap / pot])
            if gap <= 1e-6 * pot:
                break
        emit({"game": "turn+river", "solver": kind, "alpha_beta_gamma": prm, "target": "1e-6*pot",
              "seconds": time.perf_counter() - t0, "iterations": it, "gap_over_pot": gap / pot,
              "reached": gap <= 1e-6 * pot, "trajectory_iters_s_gap": traj})
    g.close()
    best = {}
    for r in rows:
        if r["solver"] == "dcfr" and r["target"] == "1e-4*pot":
            b = best.get(r["game"])
            if b is None or r["seconds"] < b["seconds"]:
                best[r["game"]] = r
    print(json.dumps({"summary": "dcfr sweep",
                      "fastest": {k: {"alpha_beta_gamma": v["alpha_beta_gamma"], "seconds": v["seconds"],
                                      "iterations": v["iterations"]} for k, v in best.items()}}), flush=True)


def _time_to_gap(gm, kind, target, tpot):
    """Seconds and iterations of a single game's solver (uniform start) to an
    FP64 gap of target * pot, checked every 25 iterations."""
    import torch
    gm.solver_set_params(kind)
    gm.solver_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, gap = 0, float("inf")
    while iters < 200000:
        gm.solver_step(25)
        iters += 25
        gap = float(gm.saddle_gap()[0][0])
        if gap <= target * tpot:
            break
    gm.solver_set_params("rm+")
    return time.perf_counter() - t0, iters, gap


def libratus_leg(args, stream):
    """A river endgame closer to the paper's: hold'em hand ranking for the
    strengths and the asymmetric betting abstraction of its appendix
    (Libratus' sizes, all-in everywhere, no raise cap), pot 100, stacks 1000:
    solver iterations per second, the matvec pair, time to 1e-4 * pot, and
    Table 1's size metric (nnz of A against Technique B's factors)."""
    import torch
    from paper_2112_03804_amd import autotune, handeval
    from paper_2112_03804_amd import instances as I
    from paper_2112_03804_amd import pmx

    d = I.libratus_river(stack=1000.0)
    pot = 2 * d.contrib
    g = pmx.Game(d)
    sched, sched_us = autotune.tune(g, use_cache=False, objective="iteration")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g.solver_reset()
    g.solver_step(100)
    torch.cuda.synchronize()
    steps = 1000
    e0.record(stream)
    g.solver_step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    it_us = e0.elapsed_time(e1) * 1e3 / steps
    pair_us = autotune.time_schedule(g, *sched, reps=500, pair=True)
    bytes_pair = algorithmic_bytes_pair(g.layouts)
    ttg, iters, gap = _time_to_gap(g, "rm+", 1e-4, pot)
    ttg_d, iters_d, gap_d = _time_to_gap(g, "dcfr", 1e-4, pot)
    t0 = time.perf_counter()
    tb = g.tb_build()
    tb_s = time.perf_counter() - t0
    size_pp = tb["nnz_ahat"] + tb["nnz_u_pp"] + tb["nnz_m_pp"] + tb["nnz_v_pp"]
    L = g.layouts[0]
    classes = int(handeval.suit_classes(d.hands[0], d.board).max()) + 1
    out = {"workload": "river endgame, hold'em hand ranking on a seeded board, 1081 hands/player, Libratus' "
                       "asymmetric bet sizes (player 1 the AI) + all-in, no raise cap, pot 100, stacks 1000",
           "n_seq": [L[0]["n_seq"], L[1]["n_seq"]], "n_hands": [L[0]["n_hands"], L[1]["n_hands"]],
           "distinct_strengths": int(d.strength[0].max()) + 1,
           "suit_isomorphism_classes": classes,
           "schedule": {"tuned": list(sched), "us_per_iteration_by_schedule": sched_us},
           "iterations_per_s": 1e6 / it_us, "iteration_us": it_us,
           "matvec_pair": {"kernel": kernel_label(sched), "us_per_launch": pair_us,
                           "algorithmic_bytes_per_launch": bytes_pair,
                           "achieved_gbs": bytes_pair / (pair_us * 1e-6) / 1e9},
           "time_to_gap": {"target": "1e-4*pot", "seconds": ttg, "iterations": iters, "gap_over_pot": gap / pot,
                           "solver": "plain RM+, uniform start, FP64 gap checked every 25 iterations",
                           "dcfr": {"seconds": ttg_d, "iterations": iters_d, "gap_over_pot": gap_d / pot,
                                    "params": "alpha 1.5, beta 0, gamma 2"}},
           "technique_b_factors": {"nnz_A": tb["nnz_A"], "size_technique_b_postprocessed": size_pp,
                                   "nnz_A_over_size": tb["nnz_A"] / max(size_pp, 1), "build_s": tb_s}}
    g.close()
    log(f"libratus river: {out['iterations_per_s']:.0f} iterations/s, {out['n_seq']} sequences, "
        f"time to gap {ttg:.3f} s")
    return out


def river_leg(args, stream):
    """The single river endgame (52-card deck, 5-card board, 1081 hands per
    player, bets {0.5, 1, 2} x pot + all-in, 3 raises): solver iterations per
    second, the matvec-pair launch (0.86 MB, cache-resident and latency
    bound), time to 1e-4 * pot (RM+ and DCFR) and the 13-card game to
    1e-6 * pot."""
    import torch
    from paper_2112_03804_amd import autotune
    from paper_2112_03804_amd import instances as I
    from paper_2112_03804_amd import pmx

    desc = I.config(1)
    pot = 2 * desc.contrib
    t_create = time.perf_counter()
    g = pmx.Game(desc)
    t_create = time.perf_counter() - t_create
    # few rows: the chunk-aligned layout's one row per workgroup usually
    # beats the grouped layout's few long-lived workgroups; products of a few
    # microseconds are tuned on whole solver iterations
    sched, sched_us = autotune.tune(g, use_cache=False, objective="iteration")
    steps, warmup = 2000, 100
    g.solver_reset()
    g.solver_step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.solver_step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
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

    # Technique B's explicit factors (Table 1's size metric) and their FP64
    # product on the GPU beside the structured FP64 and FP32 products
    t0 = time.perf_counter()
    tb_sizes = g.tb_build()
    tb_build_s = time.perf_counter() - t0
    yd, xd = y.double(), x.double()
    Ayd = torch.empty(g.elems[0], dtype=torch.float64, device="cuda")
    ATxd = torch.empty(g.elems[1], dtype=torch.float64, device="cuda")

    def pair_time(fa, fat, reps=200):
        for _ in range(10):
            fa(yd, Ayd)
            fat(xd, ATxd)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fa(yd, Ayd)
            fat(xd, ATxd)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    tb_us = pair_time(g.matvec_A_tb, g.matvec_AT_tb)
    f64_us = pair_time(g.matvec_A_f64, g.matvec_AT_f64)
    nnz_tb = tb_sizes["nnz_ahat"] + tb_sizes["nnz_u"] + tb_sizes["nnz_m"] + tb_sizes["nnz_v"]
    nnz_tb_pp = tb_sizes["nnz_ahat"] + tb_sizes["nnz_u_pp"] + tb_sizes["nnz_m_pp"] + tb_sizes["nnz_v_pp"]
    technique_b = {"sizes": tb_sizes, "size_technique_b": nnz_tb, "size_technique_b_postprocessed": nnz_tb_pp,
                   "nnz_A_over_size": tb_sizes["nnz_A"] / max(nnz_tb_pp, 1), "build_s": tb_build_s,
                   "pair_us_explicit_factors_fp64": tb_us, "pair_us_structured_fp64": f64_us,
                   "pair_us_structured_fp32": pair_us,
                   "note": "explicit factors: CSR products for Ahat, U, V and M's chain solve (pointer jumping); "
                           "structured: the hand operators applied without forming any factor"}
    del yd, xd, Ayd, ATxd

    time_to_gap = _time_to_gap
    ttg, iters, gap = time_to_gap(g, "rm+", 1e-4, pot)
    ttg_d, iters_d, gap_d = time_to_gap(g, "dcfr", 1e-4, pot)
    out = {"workload": "river endgame: 52-card deck, 5-card board, 1081 hands/player, bets {0.5,1,2}xpot + "
                       "all-in, max 3 raises, pot 100, stacks 400",
           "n_seq": [L[0][0]["n_seq"], L[0][1]["n_seq"]], "n_hands": [L[0][0]["n_hands"], L[0][1]["n_hands"]],
           "game_create_s": t_create,
           "schedule": {"tuned": list(sched), "us_per_iteration_by_schedule": sched_us},
           "iterations_per_s": steps / (ms / 1e3), "iteration_us": ms * 1e3 / steps,
           "matvec_pair": {"kernel": kernel_label(g.game_get_tuning()),
                           "us_per_launch": pair_us, "algorithmic_bytes_per_launch": bytes_pair,
                           "achieved_gbs": bytes_pair / (pair_us * 1e-6) / 1e9,
                           "traffic": measured_traffic("river", g.game_get_tuning()),
                           "note": "0.86 MB per pair stays in the caches; the launch is latency bound"},
           "technique_b_factors": technique_b,
           "time_to_gap": {"target": "1e-4*pot", "seconds": ttg, "iterations": iters,
                           "gap_over_pot": gap / pot, "solver": "plain RM+, uniform start, "
                           "FP64 gap checked every 25 iterations",
                           "dcfr": {"seconds": ttg_d, "iterations": iters_d, "gap_over_pot": gap_d / pot,
                                    "params": "alpha 1.5, beta 0, gamma 2"}}}
    g.close()
    if not args.no_tiny:
        tiny = I.config(0)
        gt = pmx.Game(tiny)
        t_ttg, t_it, t_gap = time_to_gap(gt, "rm+", 1e-6, 2 * tiny.contrib)
        gt.close()
        out["tiny_time_to_gap"] = {"workload": "13-card deck, one card per hand, bet 1x pot, one raise, pot 2",
                                   "target": "1e-6*pot", "seconds": t_ttg, "iterations": t_it,
                                   "gap_over_pot": t_gap / (2 * tiny.contrib),
                                   "solver": "plain RM+, FP64 gap every 25"}
    log(f"river: {out['iterations_per_s']:.0f} iterations/s, pair {pair_us:.2f} us, time to gap {ttg:.3f} s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1024, help="timed solver iterations over the batch")
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--cpu-batch-sample", type=int, default=16,
                    help="instances of the batch in the oracle's timed sample")
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--instances", default=None,
                    help="JSON instance spec (instances.save_json) solved as the batch instead of the synthetic one")
    ap.add_argument("--plain-sample", type=int, default=0,
                    help="instances solved by the plain single-instance solver (0: all of the batch)")
    ap.add_argument("--batch-big", type=int, default=2048,
                    help="instances of the batch whose matvec pair is timed beyond the Infinity Cache (0: skip)")
    ap.add_argument("--max-iters", type=int, default=100000)
    ap.add_argument("--no-river", action="store_true")
    ap.add_argument("--no-turn", action="store_true")
    ap.add_argument("--no-libratus", action="store_true",
                    help="skip the river endgame with hand ranking and Libratus' bet sizes")
    ap.add_argument("--no-tiny", action="store_true", help="skip the 13-card game's time to gap")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only run the launches profiled for HBM traffic counters")
    ap.add_argument("--trace-probe", action="store_true",
                    help="only run solver iterations on the batch, the turn + river game and the rivers")
    ap.add_argument("--trace-game", default=None, choices=("batch", "turn_river", "river", "libratus_river"),
                    help="with --trace-probe: only this game")
    ap.add_argument("--dcfr-sweep", action="store_true",
                    help="only sweep the discounted-CFR parameters (river, batch, turn + river)")
    ap.add_argument("--turn-steps", type=int, default=20)
    ap.add_argument("--turn-budget", type=float, default=90.0,
                    help="seconds for the turn + river precision run")
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--warm-only", action="store_true",
                    help="only the warm-start leg (with its own uniform-start baselines)")
    ap.add_argument("--warm-train", type=int, default=2048)
    ap.add_argument("--warm-label-gap", type=float, default=1e-5)
    ap.add_argument("--warm-label-kind", choices=("rm+", "dcfr"), default="dcfr")
    ap.add_argument("--warm-label-iters", type=int, default=16384)
    ap.add_argument("--warm-steps", type=int, default=8000)
    ap.add_argument("--warm-probe", type=int, default=64)
    ap.add_argument("--warm-scale", type=float, default=1.0)
    ap.add_argument("--warm-avg", type=float, default=0.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    log("importing torch")
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    from paper_2112_03804_amd import instances as I

    if args.pmc_probe:
        pmc_probe(args)
        return
    if args.trace_probe:
        trace_probe(args)
        return
    if args.dcfr_sweep:
        dcfr_sweep(args)
        return
    if args.warm_only:
        print(json.dumps({"warm_start": warm_leg(args, torch.cuda.current_stream(), None)}), flush=True)
        return
    stream = torch.cuda.current_stream()
    log("batch leg (headline)")
    batched = batched_leg(args, stream)
    log("batch leg done")
    out = {
        "metric": "matvec pairs/s (A·y+Aᵀx) & time to gap 1e-4·pot: plain vs batched/warm-start",
        "value": batched["matvec_pairs_per_s"],
        "unit": "instance matvec pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": batched["iteration_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 scan accumulation)",
        "data": "synthetic",
        "config": {"workload": batched["workload"] + "; step = one RM+ iteration of every instance "
                               "(A y, P1 update, A^T x, P2 update)",
                   "instances": batched["instances"]},
        "roofline": batched["roofline"],
    }
    out["batched"] = batched
    if not args.no_warm and not args.instances:   # the warm start is trained for the synthetic batch
        out["warm_start"] = warm_leg(args, stream, batched)
        log("warm-start leg done")
    river_iters = None
    if not args.no_river:
        out["river"] = river_leg(args, stream)
        river_iters = out["river"]["time_to_gap"]["iterations"]
        log("river leg done")
    if not args.no_libratus:
        out["libratus_river"] = libratus_leg(args, stream)
        log("libratus river leg done")
    precision = None
    if not args.no_turn:
        tr = turn_river_leg(args, stream)
        precision = {"averages": tr.pop("_averages")}
        out["turn_river"] = tr
        log("turn+river leg done")
    if not args.no_cpu_baseline:
        cb = cpu_baseline(args, I.config(1), I.load_json(args.instances) if args.instances else
                          I.batched_configs(args.batch), gpu_iters=river_iters,
                          precision=precision)
        og = cb.pop("precision_run_oracle_gap", None)
        if og is not None:
            pr = out["turn_river"]["precision_run"]
            pr["oracle_gap_over_pot"] = og["gap_over_pot"]
            pr["gap_diff_over_pot"] = abs(og["gap_over_pot"] - pr["gap_over_pot"])
            pr["gap_diff_within_1e-9_pot"] = pr["gap_diff_over_pot"] <= 1e-9
            pr["oracle_gap_seconds"] = og["seconds"]
        out["cpu_baseline"] = cb
        log("CPU baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
