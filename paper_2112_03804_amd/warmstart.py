"""Learned warm start for the batched RM+ solver (not part of the paper).

A three-layer BF16 perceptron (64 -> 512 -> 512 -> 8, ReLU, FP32
accumulation) maps each (infoset, hand) row's betting and range features to
logits over the infoset's action slots; the masked softmax is a behavioural
prior that seeds the solver's regrets, current plans and averages
(``Game.warm_apply``).  Training targets are average strategies of the plain
solver on synthetic endgames (``Game.warm_targets``), weighted by belief
weight x reach.  Every arithmetic step runs in libpmx kernels (features,
targets, GEMMs on the matrix cores, softmax cross-entropy, Adam, prior
application); this module allocates device buffers and sequences the calls.
"""
from __future__ import annotations

import time
from typing import List, Sequence

import numpy as np

from . import pmx

D_IN, WIDTH, K = 64, 512, 8
PARAMS = ("W1", "b1", "W2", "b2", "W3", "b3")
SHAPES = {"W1": (WIDTH, D_IN), "b1": (WIDTH,), "W2": (WIDTH, WIDTH), "b2": (WIDTH,),
          "W3": (K, WIDTH), "b3": (K,)}


def _torch():
    import torch
    return torch


class WarmMLP:
    """Network parameters (FP32 master + BF16 copies) and Adam state on the GPU."""

    def __init__(self, seed: int = 0, init: dict = None):
        torch = _torch()
        rng = np.random.default_rng(seed)
        self.p, self.pb, self.m, self.v, self.g = {}, {}, {}, {}, {}
        for name in PARAMS:
            shp = SHAPES[name]
            if init is not None:
                host = np.asarray(init[name], dtype=np.float32)
            elif name.startswith("W"):
                a = np.sqrt(6.0 / shp[1])
                host = rng.uniform(-a, a, size=shp).astype(np.float32)
            else:
                host = np.zeros(shp, np.float32)
            self.p[name] = torch.from_numpy(host).cuda()
            self.m[name] = torch.zeros_like(self.p[name])
            self.v[name] = torch.zeros_like(self.p[name])
            self.g[name] = torch.zeros_like(self.p[name])
            if name.startswith("W"):
                self.pb[name] = torch.empty(shp, dtype=torch.bfloat16, device="cuda")
                pmx.check(pmx.lib().mlp_cast_bf16(self.p[name].numel(), pmx.dptr(self.p[name]),
                                                  pmx.dptr(self.pb[name]), pmx.stream_ptr()))
        self.step = 0
        self._ws = {}

    # -- buffers ------------------------------------------------------------
    def _work(self, M: int):
        torch = _torch()
        if self._ws.get("M", 0) < M:
            f32 = dict(dtype=torch.float32, device="cuda")
            b16 = dict(dtype=torch.bfloat16, device="cuda")
            self._ws = {
                "M": M,
                "H1": torch.empty((M, WIDTH), **f32), "H1b": torch.empty((M, WIDTH), **b16),
                "H2": torch.empty((M, WIDTH), **f32), "H2b": torch.empty((M, WIDTH), **b16),
                "Z3": torch.empty((M, K), **f32),
                "dZ3": torch.empty((M, K), **f32), "dZ3b": torch.empty((M, K), **b16),
                "dZ2": torch.empty((M, WIDTH), **f32), "dZ2b": torch.empty((M, WIDTH), **b16),
                "dZ1": torch.empty((M, WIDTH), **f32), "dZ1b": torch.empty((M, WIDTH), **b16),
                "loss": torch.empty(((M + 255) // 256,), **f32),
                # split-K partial products of the weight gradients and partial
                # column sums of the bias gradients
                "work": torch.empty((32 * WIDTH * WIDTH,), **f32),
            }
        return self._ws

    @staticmethod
    def gemm(M, N, Kd, A, lda, tA, B, ldb, tB, C=None, ldc=0, Cb=None, ldcb=0, bias=None, relu=False,
             mask=None, ldm=0, work=None):
        L = pmx.lib()
        pmx.check(L.mlp_gemm_bf16(M, N, Kd, pmx.dptr(A), lda, tA, pmx.dptr(B), ldb, tB, pmx.dptr(bias),
                                  1 if relu else 0, pmx.dptr(mask), ldm, pmx.dptr(C), ldc, pmx.dptr(Cb),
                                  ldcb, pmx.dptr(work), 0 if work is None else work.numel(),
                                  pmx.stream_ptr()))

    @staticmethod
    def colsum(M, N, dz, db, work):
        pmx.check(pmx.lib().mlp_colsum(M, N, pmx.dptr(dz), pmx.dptr(db), pmx.dptr(work), work.numel(),
                                       pmx.stream_ptr()))

    # -- forward / backward ------------------------------------------------
    def forward(self, Xb, M: int):
        """Logits [M, 8] (FP32) for BF16 inputs Xb [M, 64]; keeps activations."""
        w = self._work(M)
        self.gemm(M, WIDTH, D_IN, Xb, D_IN, 0, self.pb["W1"], D_IN, 1, C=w["H1"], ldc=WIDTH,
                  Cb=w["H1b"], ldcb=WIDTH, bias=self.p["b1"], relu=True)
        self.gemm(M, WIDTH, WIDTH, w["H1b"], WIDTH, 0, self.pb["W2"], WIDTH, 1, C=w["H2"], ldc=WIDTH,
                  Cb=w["H2b"], ldcb=WIDTH, bias=self.p["b2"], relu=True)
        self.gemm(M, K, WIDTH, w["H2b"], WIDTH, 0, self.pb["W3"], WIDTH, 1, C=w["Z3"], ldc=K,
                  bias=self.p["b3"])
        return w["Z3"]

    def loss_and_grad(self, Xb, T, Wt, M: int):
        """Weighted masked cross-entropy of a batch and the parameter gradients
        (left in self.g); returns the loss summed over rows."""
        L = pmx.lib()
        w = self._work(M)
        self.forward(Xb, M)
        pmx.check(L.mlp_softmax_xent(M, K, pmx.dptr(w["Z3"]), K, pmx.dptr(T), pmx.dptr(Wt),
                                     pmx.dptr(w["dZ3"]), pmx.dptr(w["dZ3b"]), pmx.dptr(w["loss"]),
                                     pmx.stream_ptr()))
        wk = w["work"]
        # layer 3
        self.gemm(K, WIDTH, M, w["dZ3b"], K, 1, w["H2b"], WIDTH, 0, C=self.g["W3"], ldc=WIDTH, work=wk)
        self.colsum(M, K, w["dZ3"], self.g["b3"], wk)
        self.gemm(M, WIDTH, K, w["dZ3b"], K, 0, self.pb["W3"], WIDTH, 0, C=w["dZ2"], ldc=WIDTH,
                  Cb=w["dZ2b"], ldcb=WIDTH, mask=w["H2"], ldm=WIDTH)
        # layer 2
        self.gemm(WIDTH, WIDTH, M, w["dZ2b"], WIDTH, 1, w["H1b"], WIDTH, 0, C=self.g["W2"], ldc=WIDTH, work=wk)
        self.colsum(M, WIDTH, w["dZ2"], self.g["b2"], wk)
        self.gemm(M, WIDTH, WIDTH, w["dZ2b"], WIDTH, 0, self.pb["W2"], WIDTH, 0, C=w["dZ1"], ldc=WIDTH,
                  Cb=w["dZ1b"], ldcb=WIDTH, mask=w["H1"], ldm=WIDTH)
        # layer 1
        self.gemm(WIDTH, D_IN, M, w["dZ1b"], WIDTH, 1, Xb, D_IN, 0, C=self.g["W1"], ldc=D_IN, work=wk)
        self.colsum(M, WIDTH, w["dZ1"], self.g["b1"], wk)
        return w["loss"][: (M + 255) // 256]

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
        self.step += 1
        L = pmx.lib()
        for name in PARAMS:
            pmx.check(L.mlp_adam(self.p[name].numel(), pmx.dptr(self.p[name]), pmx.dptr(self.g[name]),
                                 pmx.dptr(self.m[name]), pmx.dptr(self.v[name]), pmx.dptr(self.pb.get(name)),
                                 lr, b1, b2, eps, wd, self.step, pmx.stream_ptr()))

    def logits(self, Xb, M: int, chunk: int = 1 << 20):
        """Logits for M rows in chunks (inference)."""
        torch = _torch()
        out = torch.empty((M, K), dtype=torch.float32, device="cuda")
        for a in range(0, M, chunk):
            b = min(M, a + chunk)
            z = self.forward(Xb[a:b], b - a)
            out[a:b].copy_(z[: b - a])
        return out


class Dataset:
    """Rows of (features, targets, weights) from solved instances (device)."""

    def __init__(self):
        self.X, self.T, self.W = [], [], []

    def add_game(self, game):
        torch = _torch()
        for p in range(2):
            n = game.warm_num_rows(p)
            X = torch.empty((n, D_IN), dtype=torch.bfloat16, device="cuda")
            T = torch.empty((n, K), dtype=torch.float32, device="cuda")
            W = torch.empty((n,), dtype=torch.float32, device="cuda")
            game.warm_features(p, X)
            game.warm_targets(p, T, W)
            self.X.append(X)
            self.T.append(T)
            self.W.append(W)

    def finalize(self):
        torch = _torch()
        self.X = torch.cat(self.X)
        self.T = torch.cat(self.T)
        self.W = torch.cat(self.W)
        return self

    @property
    def rows(self):
        return int(self.X.shape[0])


def make_dataset(descs: Sequence, iters: int = 0, batch: int = 512, target: float = 0.0,
                 kind: str = "rm+", max_iters: int = 100000, progress=None) -> Dataset:
    """Solve the instances in batches and collect training rows from the
    average strategies: for `iters` iterations of the chosen solver, or, with
    `target` > 0, until every instance's FP64 gap is at most target * its pot
    (instances retire as they reach it; at most `max_iters` iterations)."""
    ds = Dataset()
    for a in range(0, len(descs), batch):
        g = pmx.Game(list(descs[a:a + batch]))
        g.solver_set_params(kind)
        if target > 0:
            solve_to_gap(g, target, check_every=64, max_iters=max_iters)
        else:
            g.solver_step(iters)
        ds.add_game(g)
        _torch().cuda.synchronize()
        g.close()
        if progress:
            progress(min(a + batch, len(descs)), len(descs))
    return ds.finalize()


def train(mlp: WarmMLP, ds: Dataset, steps: int, batch_rows: int = 8192, lr: float = 1e-3, seed: int = 0,
          log_every: int = 0, progress=None) -> List[float]:
    """Minibatch Adam on uniformly sampled rows; returns mean loss per logged
    interval (loss per unit weight)."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    L = pmx.lib()
    Xb = torch.empty((batch_rows, D_IN), dtype=torch.bfloat16, device="cuda")
    Tb = torch.empty((batch_rows, K), dtype=torch.float32, device="cuda")
    Wb = torch.empty((batch_rows,), dtype=torch.float32, device="cuda")
    idx_host = np.empty(batch_rows, np.int64)
    idx = torch.empty((batch_rows,), dtype=torch.int64, device="cuda")
    hist, acc, wacc = [], 0.0, 0.0
    for it in range(steps):
        idx_host[:] = rng.integers(0, ds.rows, size=batch_rows)
        idx.copy_(torch.from_numpy(idx_host))
        s = pmx.stream_ptr()
        pmx.check(L.mlp_gather_bf16(batch_rows, D_IN, pmx.dptr(idx), pmx.dptr(ds.X), pmx.dptr(Xb), s))
        pmx.check(L.mlp_gather_f32(batch_rows, K, pmx.dptr(idx), pmx.dptr(ds.T), pmx.dptr(Tb), s))
        pmx.check(L.mlp_gather_f32(batch_rows, 1, pmx.dptr(idx), pmx.dptr(ds.W), pmx.dptr(Wb), s))
        loss = mlp.loss_and_grad(Xb, Tb, Wb, batch_rows)
        mlp.adam(lr=lr)
        if log_every and (it + 1) % log_every == 0:
            acc = float(loss.sum().item())
            wacc = float(Wb.sum().item())
            hist.append(acc / max(wacc, 1e-12))
            if progress:
                progress(it + 1, hist[-1])
    return hist


def apply_prior(game, mlp: WarmMLP, regret_scale: float, avg_weight: float):
    """Features -> logits -> solver prior for both players of `game`."""
    torch = _torch()
    logits = []
    for p in range(2):
        n = game.warm_num_rows(p)
        X = torch.empty((n, D_IN), dtype=torch.bfloat16, device="cuda")
        game.warm_features(p, X)
        logits.append(mlp.logits(X, n))
    game.warm_apply(logits[0], logits[1], K, regret_scale, avg_weight)
    return logits


def _instance_rows(game, p: int) -> np.ndarray:
    """Row offsets of each instance among player p's network rows ((infoset,
    hand) pairs, instance by instance)."""
    n = [L[p]["n_infosets"] * L[p]["n_hands"] for L in game.layouts]
    return np.concatenate([[0], np.cumsum(n)]).astype(np.int64)


def apply_logits_with_fallback(game, logits, regret_scale: float, avg_weight: float, probe: int = 64):
    """Warm start with the uniform start as the fallback (per instance).

    The uniform start and the prior from `logits` (one [rows, 8] FP32 tensor
    per player) each run `probe` solver iterations; an instance keeps the
    prior's run only if its logits are finite and its FP64 gap after the
    probe is below the uniform run's; the others continue from the uniform
    run's state (regrets, plans, averages and weight totals, restored on the
    device from a snapshot).  The game ends `probe` iterations in either way.
    Returns the per-instance flags (True: the prior was kept) and both probe
    gaps."""
    torch = _torch()
    ni = game.n_instances
    game.solver_reset()
    game.solver_step(probe)
    gap_u = game.saddle_gap()[0]
    game.solver_snapshot()
    finite = np.ones(ni, dtype=bool)
    for p in range(2):
        off = _instance_rows(game, p)
        ok = torch.isfinite(logits[p]).all(dim=1).cpu().numpy()
        for i in range(ni):
            finite[i] &= bool(ok[off[i]:off[i + 1]].all())
    game.warm_apply(logits[0], logits[1], K, regret_scale, avg_weight)
    game.solver_step(probe)
    gap_w = game.saddle_gap()[0]
    keep = finite & (gap_w < gap_u)
    if not keep.all():
        game.solver_restore_instances((~keep).astype(np.int32))
    return keep, gap_u, gap_w


def apply_prior_with_fallback(game, mlp: WarmMLP, regret_scale: float, avg_weight: float, probe: int = 64):
    """The network's prior with the uniform start as fallback (see
    apply_logits_with_fallback)."""
    torch = _torch()
    logits = []
    for p in range(2):
        n = game.warm_num_rows(p)
        X = torch.empty((n, D_IN), dtype=torch.bfloat16, device="cuda")
        game.warm_features(p, X)
        logits.append(mlp.logits(X, n))
    return apply_logits_with_fallback(game, logits, regret_scale, avg_weight, probe)


def solve_to_gap(game, target_rel: float, check_every: int = 32, max_iters: int = 100000,
                 retire: bool = True, start_iters: int = 0):
    """Iterate until every instance's gap <= target_rel * its pot, retiring
    instances (``solver_set_active``) as they reach it; returns (seconds,
    iterations, per-instance first iteration at target).  `start_iters`
    counts iterations the game has already run (a probe) in the reported
    iteration numbers."""
    torch = _torch()
    pots = np.array([2 * d.contrib for d in game.descs])
    done = np.full(game.n_instances, -1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    gap = game.saddle_gap()[0]
    if start_iters:
        it = start_iters
    done[gap <= target_rel * pots] = it
    if retire:
        game.solver_set_active(done < 0)
    while (done < 0).any() and it < max_iters:
        game.solver_step(check_every)
        it += check_every
        gap = game.saddle_gap()[0]
        newly = (gap <= target_rel * pots) & (done < 0)
        done[newly] = it
        if retire and newly.any():
            game.solver_set_active(done < 0)
    return time.perf_counter() - t0, it, done
