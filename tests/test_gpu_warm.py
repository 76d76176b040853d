"""GPU tests of the warm-start network kernels and of the prior's plumbing.

* GEMM on the matrix cores against an FP32 product of the same BF16-rounded
  operands (every transpose combination, ragged sizes, all epilogues);
* loss and gradients of the three-layer network against the FP64 oracle
  (oracle/mlp.py, pinned by finite differences); BF16 activations bound the
  agreement to about 1e-2 relative;
* features, targets and the applied prior against definitions computed here
  and against the oracle's treeplex;
* a short training run lowers the loss.
"""
import numpy as np
import pytest

from paper_2112_03804_amd import instances as I
from oracle import mlp as omlp
from oracle import payoff, solver

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_03804_amd import pmx, warmstart
    pmx.lib()
    return pmx, warmstart


def _say(*a):
    print(*a, flush=True)


def bf16_round(a):
    """Round float32 values to the nearest BF16 (ties to even), as float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def to_bf16_dev(a):
    return torch.from_numpy(bf16_round(a)).cuda().to(torch.bfloat16)


@pytest.mark.parametrize("tA,tB", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K,split", [(77, 45, 83, 0), (130, 8, 512, 0), (64, 64, 32, 0), (5, 200, 3, 0),
                                         (128, 192, 640, 0), (8, 136, 3000, 1), (70, 64, 2050, 1),
                                         (200, 72, 8192, 1)])
def test_gemm_bf16_matches_fp32_product(tA, tB, M, N, K, split):
    """Every operand layout, ragged edges (unaligned leading dimensions take
    the element-wise loads), and split K through a workspace."""
    pmx, _ = _need()
    _say("gemm", tA, tB, M, N, K, split)
    rng = np.random.default_rng(M * 7 + N + K + 3 * tA + tB)
    A = bf16_round(rng.standard_normal((K, M) if tA else (M, K)).astype(np.float32))
    B = bf16_round(rng.standard_normal((N, K) if tB else (K, N)).astype(np.float32))
    bias = rng.standard_normal(N).astype(np.float32)
    mask = (rng.random((M, N)) > 0.3).astype(np.float32)
    opA = A.T if tA else A
    opB = B.T if tB else B
    ref = opA.astype(np.float64) @ opB.astype(np.float64) + bias
    ref = np.maximum(ref, 0.0) * (mask > 0)
    Ad, Bd = to_bf16_dev(A), to_bf16_dev(B)
    C = torch.full((M, N), 9.0, dtype=torch.float32, device="cuda")
    Cb = torch.zeros((M, N), dtype=torch.bfloat16, device="cuda")
    # device tensors stay referenced until the launch is enqueued
    bias_d = torch.from_numpy(bias).cuda()
    mask_d = torch.from_numpy(mask).cuda()
    work = torch.full((64 * M * N,), float("nan"), dtype=torch.float32, device="cuda") if split else None
    L = pmx.lib()
    pmx.check(L.mlp_gemm_bf16(M, N, K, pmx.dptr(Ad), M if tA else K, tA, pmx.dptr(Bd), K if tB else N, tB,
                              pmx.dptr(bias_d), 1, pmx.dptr(mask_d), N, pmx.dptr(C), N, pmx.dptr(Cb), N,
                              pmx.dptr(work), 0 if work is None else work.numel(), pmx.stream_ptr()))
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.float64)
    scale = np.abs(opA).astype(np.float64) @ np.abs(opB).astype(np.float64) + np.abs(bias)
    assert np.all(np.abs(got - ref) <= 1e-5 * scale + 1e-6)
    gotb = Cb.float().cpu().numpy()
    assert np.allclose(gotb, bf16_round(got.astype(np.float32)), rtol=0, atol=0)


@pytest.mark.parametrize("rows,cols", [(1, 5), (300, 8), (8192, 512), (1000, 300)])
def test_colsum_with_and_without_workspace(rows, cols):
    pmx, _ = _need()
    _say("colsum", rows, cols)
    rng = np.random.default_rng(rows + cols)
    dz = rng.standard_normal((rows, cols)).astype(np.float32)
    ref = dz.astype(np.float64).sum(axis=0)
    d = torch.from_numpy(dz).cuda()
    L = pmx.lib()
    for use_work in (False, True):
        db = torch.full((cols,), float("nan"), dtype=torch.float32, device="cuda")
        work = torch.full((((rows + 63) // 64) * cols,), float("nan"), dtype=torch.float32, device="cuda")
        pmx.check(L.mlp_colsum(rows, cols, pmx.dptr(d), pmx.dptr(db), pmx.dptr(work) if use_work else None,
                               work.numel() if use_work else 0, pmx.stream_ptr()))
        torch.cuda.synchronize()
        got = db.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - ref) <= 1e-5 * np.abs(dz).astype(np.float64).sum(axis=0) + 1e-6), use_work


def test_network_loss_and_gradients_match_fp64_oracle():
    pmx, ws = _need()
    _say("network gradients")
    rng = np.random.default_rng(0)
    M = 300
    p = omlp.init(ws.D_IN, ws.WIDTH, ws.K, seed=3)
    for b in ("b1", "b2", "b3"):
        p[b] = rng.normal(size=p[b].shape) * 0.05
    for w in ("W1", "W2", "W3"):
        p[w] = bf16_round(p[w].astype(np.float32)).astype(np.float64)
    X = bf16_round(rng.standard_normal((M, ws.D_IN)).astype(np.float32)).astype(np.float64)
    T = rng.random((M, ws.K))
    nact = rng.integers(2, ws.K + 1, size=M)
    for r in range(M):
        T[r, nact[r]:] = -1.0
        T[r, :nact[r]] /= T[r, :nact[r]].sum()
    W = rng.random(M) + 0.5
    loss, g, _ = omlp.loss_and_grad(p, X, T, W)
    net = ws.WarmMLP(init={k: v.astype(np.float32) for k, v in p.items()})
    Xd = torch.from_numpy(X.astype(np.float32)).cuda().to(torch.bfloat16)
    lp = net.loss_and_grad(Xd, torch.from_numpy(T.astype(np.float32)).cuda(),
                           torch.from_numpy(W.astype(np.float32)).cuda(), M)
    torch.cuda.synchronize()
    assert abs(float(lp.sum().item()) - loss) <= 1e-2 * abs(loss)
    for name in ws.PARAMS:
        got = net.g[name].cpu().numpy().astype(np.float64)
        rel = np.linalg.norm(got - g[name]) / max(np.linalg.norm(g[name]), 1e-30)
        assert rel <= 3e-2, (name, rel)


def _brute_hand_features(d, p):
    """Range features of each hand by direct enumeration of opponent hands."""
    q = 1 - p
    hp, hq = np.asarray(d.hands[p]), np.asarray(d.hands[q])
    mu_p, mu_q = np.asarray(d.range_[p]), np.asarray(d.range_[q])
    sp, sq = d.strength[p][0].astype(np.int64), d.strength[q][0].astype(np.int64)
    order = sorted(range(len(hp)), key=lambda h: (sp[h], h))
    rank = np.empty(len(hp), np.int64)
    rank[order] = np.arange(len(hp))
    out = np.zeros((len(hp), 5))
    T = mu_q.sum()
    for h in range(len(hp)):
        out[h, 0] = min(mu_p[h] / mu_p.mean(), 8.0) / 8.0
        out[h, 1] = rank[h] / (len(hp) - 1)
        share = np.array([bool(set(hp[h].tolist()) & set(hq[j].tolist())) for j in range(len(hq))])
        blocked = mu_q[share].sum()
        out[h, 2] = blocked / T
        comp = ~share
        cm = mu_q[comp].sum()
        out[h, 3] = mu_q[comp & (sq < sp[h])].sum() / cm
        out[h, 4] = mu_q[comp & (sq > sp[h])].sum() / cm
    return out


def test_features_targets_and_prior():
    pmx, ws = _need()
    d = I.small_river(6, deck_size=12, n_board=2, bet_fracs=(0.5, 1.0), max_raises=2)
    _say("warm features / targets / prior")
    g = pmx.Game(d)
    o = payoff.Game(d)
    for p in range(2):
        n = g.warm_num_rows(p)
        L = g.layouts[0][p]
        assert n == L["n_infosets"] * L["n_hands"]
        X = torch.empty((n, ws.D_IN), dtype=torch.bfloat16, device="cuda")
        g.warm_features(p, X)
        torch.cuda.synchronize()
        Xh = X.float().cpu().numpy().reshape(L["n_infosets"], L["n_hands"], ws.D_IN)
        hf = _brute_hand_features(d, p)
        for I_ in range(L["n_infosets"]):
            # one BF16 rounding step of slack: host and test sum in different orders
            assert np.allclose(Xh[I_, :, 59:], bf16_round(hf.astype(np.float32)), rtol=8e-3, atol=1e-6)
            assert np.all(Xh[I_, :, 0] == p)
            # valid action slots equal the infoset's action count
            assert np.allclose(Xh[I_, 0, 11::6][:8].sum(), L["infoset_nact"][I_])
    # targets from the average strategy after some iterations
    g.solver_step(64)
    for p in range(2):
        n = g.warm_num_rows(p)
        L = g.layouts[0][p]
        T = torch.empty((n, ws.K), dtype=torch.float32, device="cuda")
        W = torch.empty((n,), dtype=torch.float32, device="cuda")
        g.warm_targets(p, T, W)
        torch.cuda.synchronize()
        T = T.cpu().numpy().reshape(L["n_infosets"], L["n_hands"], ws.K)
        xbar = g.unpack(p, g.get_average_strategy(p))[0]
        for I_ in range(L["n_infosets"]):
            par, f, na = L["infoset_parent"][I_], L["infoset_first"][I_], L["infoset_nact"][I_]
            reach = np.ones(L["n_hands"]) if par < 0 else xbar[par]
            with np.errstate(invalid="ignore", divide="ignore"):
                b = np.where(reach[None, :] > 0, xbar[f:f + na] / reach[None, :], 1.0 / na)
            assert np.allclose(T[I_, :, :na].T, b, atol=2e-6)
            assert np.all(T[I_, :, na:] == -1.0)
    # the prior applied from random logits: plans are its realization
    rng = np.random.default_rng(1)
    logits = [torch.from_numpy(rng.standard_normal((g.warm_num_rows(p), ws.K)).astype(np.float32)).cuda()
              for p in range(2)]
    g.warm_apply(logits[0], logits[1], ws.K, 1.0, 0.0)
    tp = [solver.Treeplex(o, p) for p in range(2)]
    plans = []
    for p in range(2):
        L = g.layouts[0][p]
        Z = logits[p].cpu().numpy().reshape(L["n_infosets"], L["n_hands"], ws.K).astype(np.float64)
        b = np.zeros((o.S[p], o.N[p]))
        for I_ in range(L["n_infosets"]):
            f, na = L["infoset_first"][I_], L["infoset_nact"][I_]
            z = Z[I_, :, :na]
            e = np.exp(z - z.max(axis=1, keepdims=True))
            b[f:f + na] = (e / e.sum(axis=1, keepdims=True)).T
        x = tp[p].realization(b)
        st = g.solver_get_state(p)
        assert np.allclose(g.unpack(p, st["plan"])[0], x, atol=1e-6)
        assert st["t"] == 0
        plans.append(x)
    gap = g.saddle_gap()[0][0]
    rgap, _, _ = solver.saddle_gap(o, plans[0], plans[1])
    assert abs(gap - rgap) <= 1e-6 * 2 * d.contrib
    g.close()


def test_short_training_lowers_loss():
    pmx, ws = _need()
    descs = [I.river_config(seed=700 + i, n_keep=(150, 170), bet_fracs=(0.5, 1.0), max_raises=2,
                            pot=50.0, stack=150.0) for i in range(6)]
    _say("short training")
    ds = ws.make_dataset(descs, iters=256, batch=6)
    net = ws.WarmMLP(seed=0)
    hist = ws.train(net, ds, steps=300, batch_rows=2048, lr=1e-3, log_every=50)
    assert np.all(np.isfinite(hist))
    assert hist[-1] < 0.85 * hist[0], hist


def test_targets_of_retired_instance_use_its_own_weight():
    """Training weights (belief weight x average reach) of an instance retired
    early are those it had at retirement: its reach is its weighted sum over
    its own weight total, however long the others keep iterating."""
    pmx, ws = _need()
    descs = [I.river_config(seed=950 + i, n_keep=(90, 110), bet_fracs=(0.5, 1.0), max_raises=2,
                            pot=40.0, stack=120.0) for i in range(2)]
    g = pmx.Game(descs)
    g.solver_step(24)

    def weights(p):
        n = g.warm_num_rows(p)
        T = torch.empty((n, ws.K), dtype=torch.float32, device="cuda")
        W = torch.empty((n,), dtype=torch.float32, device="cuda")
        g.warm_targets(p, T, W)
        torch.cuda.synchronize()
        return T.cpu().numpy(), W.cpu().numpy()

    before = [weights(p) for p in range(2)]
    g.solver_set_active([0, 1])
    g.solver_step(40)
    after = [weights(p) for p in range(2)]
    for p in range(2):
        L = g.layouts[0][p]
        r0 = L["n_infosets"] * L["n_hands"]
        assert np.array_equal(before[p][0][:r0], after[p][0][:r0])
        assert np.array_equal(before[p][1][:r0], after[p][1][:r0])
        assert before[p][1][:r0].max() > 0
        assert not np.array_equal(before[p][1][r0:], after[p][1][r0:])
    g.close()


def test_adam_matches_the_oracle():
    """mlp_adam (FP32, with the BF16 weight copy) follows the oracle's FP64
    Adam over five steps with changing gradients and weight decay."""
    pmx, _ = _need()
    L = pmx.lib()
    rng = np.random.default_rng(17)
    n = 3001
    w0 = rng.standard_normal(n).astype(np.float32)
    wd = 0.01
    w = torch.from_numpy(w0.copy()).cuda()
    m = torch.zeros(n, dtype=torch.float32, device="cuda")
    v = torch.zeros(n, dtype=torch.float32, device="cuda")
    wb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    rw, rm, rv = w0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32) * (0.1 * t)
        gd = torch.from_numpy(g).cuda()
        pmx.check(L.mlp_adam(n, pmx.dptr(w), pmx.dptr(gd), pmx.dptr(m), pmx.dptr(v), pmx.dptr(wb), 1e-2, 0.9,
                             0.999, 1e-8, wd, t, pmx.stream_ptr()))
        rw, rm, rv = omlp.adam_step(rw, g.astype(np.float64), rm, rv, t, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8, wd=wd)
    torch.cuda.synchronize()
    got = w.cpu().numpy().astype(np.float64)
    assert np.abs(got - rw).max() <= 1e-5 * max(1.0, np.abs(rw).max())
    assert np.allclose(wb.float().cpu().numpy(), bf16_round(w.cpu().numpy()), rtol=0, atol=0)


def _target_logits(g, ws, p):
    """Logits whose softmax is the solver's current average behaviour."""
    n = g.warm_num_rows(p)
    T = torch.empty((n, ws.K), dtype=torch.float32, device="cuda")
    W = torch.empty((n,), dtype=torch.float32, device="cuda")
    g.warm_targets(p, T, W)
    return torch.where(T >= 0, torch.log(T.clamp_min(1e-6)), torch.full_like(T, -30.0))


def test_warm_start_fallback_per_instance():
    """A prior that is a near-equilibrium keeps its run; a prior that folds
    everything and one with a non-finite logit fall back to the uniform start:
    those instances end the probe exactly in the uniform run's state."""
    pmx, ws = _need()
    descs = [I.river_config(seed=810 + i, n_keep=(120, 140), bet_fracs=(0.5, 1.0), max_raises=2,
                            pot=40.0, stack=120.0) for i in range(3)]
    _say("warm start fallback")
    g = pmx.Game(descs)
    g.solver_set_params("dcfr")
    g.solver_step(2000)                       # a good prior: the averages of a long run
    logits = [_target_logits(g, ws, p) for p in range(2)]
    g.solver_set_params("rm+")
    for p in range(2):
        off = ws._instance_rows(g, p)
        Z = logits[p]
        # instance 1: fold (slot 0) everywhere; instance 2: one NaN logit
        Z[off[1]:off[2]] = -5.0
        Z[off[1]:off[2], 0] = 5.0
        Z[off[2], 1] = float("nan")
    probe = 32
    keep, gap_u, gap_w = ws.apply_logits_with_fallback(g, logits, 1.0, 0.0, probe=probe)
    assert keep.tolist() == [True, False, False], (keep, gap_u, gap_w)
    # the fallen-back instances stand where the uniform run stood
    u = pmx.Game(descs)
    u.solver_step(probe)
    for p in range(2):
        sg, su = g.solver_get_state(p), u.solver_get_state(p)
        for field in ("regret", "plan", "avg_sum"):
            a = g.unpack(p, sg[field])
            b = u.unpack(p, su[field])
            for i in (1, 2):
                assert np.array_equal(a[i], b[i]), field
        assert not np.array_equal(g.unpack(p, sg["avg_sum"])[0], u.unpack(p, su["avg_sum"])[0])
    assert np.array_equal(g.solver_get_weights()[1:], u.solver_get_weights()[1:])
    gap = g.saddle_gap()[0]
    ugap = u.saddle_gap()[0]
    assert gap[1] == ugap[1] and gap[2] == ugap[2]
    assert gap[0] < ugap[0]
    u.close()
    g.close()


def test_snapshot_restore_errors():
    """Restoring needs a snapshot taken at the same iteration count."""
    pmx, _ = _need()
    g = pmx.Game([I.small_river(0), I.small_river(1)])
    with pytest.raises(pmx.PmxError):
        g.solver_restore_instances([1, 0])
    g.solver_step(4)
    g.solver_snapshot()
    g.solver_step(1)
    with pytest.raises(pmx.PmxError):
        g.solver_restore_instances([1, 1])
    g.close()


def test_trained_prior_lowers_held_out_iterations():
    """A network trained on 256 solved endgames (DCFR averages at
    1e-5 * pot) lowers the total RM+ iterations to 1e-4 * pot on 32 held-out
    endgames of the batched distribution against the uniform start, with the
    same solver and batch."""
    pmx, ws = _need()
    _say("warm start gain: labelling")
    train = I.batched_configs(256, seed=23)
    ds = ws.make_dataset(train, batch=256, target=1e-5, kind="dcfr", max_iters=8192)
    net = ws.WarmMLP(seed=0)
    _say("warm start gain: training on", ds.rows, "rows")
    ws.train(net, ds, steps=800, batch_rows=8192, lr=1e-3)
    del ds
    held = I.batched_configs(32)
    g = pmx.Game(held)
    _, _, done_u = ws.solve_to_gap(g, 1e-4, check_every=32, max_iters=40000)
    g.solver_reset()
    ws.apply_prior(g, net, 1.0, 0.0)
    _, _, done_w = ws.solve_to_gap(g, 1e-4, check_every=32, max_iters=40000)
    g.close()
    _say(f"  iterations to 1e-4 * pot: uniform {done_u.sum()}, prior {done_w.sum()}")
    assert (done_u >= 0).all() and (done_w >= 0).all()
    assert done_w.sum() < 0.9 * done_u.sum(), (done_w.sum(), done_u.sum())
