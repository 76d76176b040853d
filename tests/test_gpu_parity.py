"""GPU parity of libpmx against the CPU oracle (calls go through the C ABI).

Tolerances (written here, derived in the design notes):
* FP32 matvec: |g - g_ref| <= 1e-5 * ||A||_inf * ||y||_inf (the stated bound)
  and, stricter, elementwise <= 1e-6 * (|A| |y|) + 1e-7 * ||A||_inf ||y||_inf:
  sums are carried across chunks in FP64, but inputs, chunk partial sums (at
  most 24 terms) and the stored prefix sums are FP32, and the
  inclusion-exclusion subtracts prefix sums of whole segments (all opponent
  hands, blocked ones included), so a few FP32 ulps of a segment total remain
  on an entry whatever its own size.
* FP64 matvec: elementwise <= 1e-12 * (|A| |y|) + 1e-15 * ||A||_inf ||y||_inf.
* Saddle gap, best responses: |diff| <= 1e-9 * pot.
* One RM+ step from a given state: regrets and plans within 1e-5 of their
  scale (FP32 state and gradients against the FP64 oracle).
"""
import numpy as np
import pytest

from paper_2112_03804_amd import instances as I
from oracle import payoff, solver

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_03804_amd import pmx
    pmx.lib()
    return pmx


def _say(*a):
    print(*a, flush=True)


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


SMALL = [
    ("kuhn", I.kuhn),
    ("tiny", I.tiny_config),
    ("small_river", lambda: I.small_river(0)),
    ("small_river_pruned", lambda: I.small_river(5, deck_size=11, n_keep=(20, 13))),
    ("turn_1card", lambda: I.small_turn_river(0)),
    ("turn_2card", lambda: I.small_turn_river(1, deck_size=9, n_board=3, cards_per_hand=2,
                                              bet_fracs=(0.5,), max_raises=0, stack=8.0)),
    ("turn_2card_deep", lambda: I.small_turn_river(4, deck_size=10, n_board=3, cards_per_hand=2,
                                                   bet_fracs=(0.5, 1.0), max_raises=1, stack=30.0,
                                                   zero_frac=0.2)),
    ("river_pruned_mid", lambda: I.river_config(seed=7, n_keep=(300, 517), bet_fracs=(0.33, 1.5),
                                                max_raises=2, stack=250.0)),
]


F32_FLOOR = 1e-7     # normalized by ||A||_inf ||y||_inf
F64_FLOOR = 1e-15


def _rand_vectors(o, rng, p):
    v = rng.standard_normal((o.S[p], o.N[p]))
    v[:, rng.random(o.N[p]) < 0.1] = 0.0
    return v.astype(np.float32).astype(np.float64)


def _assert_close(got, ref, mag, rel, floor, what):
    """Elementwise |got - ref| <= rel * mag + floor; report the worst entry."""
    err = np.abs(got - ref)
    bound = rel * mag + floor
    bad = err > bound
    if bad.any():
        i = np.unravel_index(np.argmax(err / np.maximum(bound, 1e-300)), err.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} entries off; worst at {i}: got {got[i]!r} "
                             f"ref {ref[i]!r} |A||v| {mag[i]!r} bound {bound[i]!r}")


def _check_matvecs(pmx, d, seed=0, full=True):
    o = payoff.Game(d)
    g = pmx.Game(d)
    rng = np.random.default_rng(seed)
    y = _rand_vectors(o, rng, 1)
    x = _rand_vectors(o, rng, 0)
    yd, xd = _dev(g.pack(1, [y]), np.float32), _dev(g.pack(0, [x]), np.float32)
    Ay = torch.zeros(g.elems[0], dtype=torch.float32, device="cuda")
    ATx = torch.zeros(g.elems[1], dtype=torch.float32, device="cuda")
    g.matvec_A(yd, Ay)
    g.matvec_AT(xd, ATx)
    Ay2 = torch.full_like(Ay, 7.0)
    ATx2 = torch.full_like(ATx, 7.0)
    g.matvec_pair(yd, xd, Ay2, ATx2)
    Ayd = torch.zeros(g.elems[0], dtype=torch.float64, device="cuda")
    ATxd = torch.zeros(g.elems[1], dtype=torch.float64, device="cuda")
    g.matvec_A_f64(_dev(g.pack(1, [y], np.float64), np.float64), Ayd)
    g.matvec_AT_f64(_dev(g.pack(0, [x], np.float64), np.float64), ATxd)
    torch.cuda.synchronize()
    ref_A, ref_AT = o.matvec_A(y), o.matvec_AT(x)
    mag_A, mag_AT = payoff.abs_matvec_A(o, y), payoff.abs_matvec_AT(o, x)
    normA = o.abs_row_sums().max()
    got_A = g.unpack(0, Ay.cpu().numpy())[0].astype(np.float64)
    got_AT = g.unpack(1, ATx.cpu().numpy())[0].astype(np.float64)
    assert np.abs(got_A - ref_A).max() <= 1e-5 * normA * np.abs(y).max()
    assert np.abs(got_AT - ref_AT).max() <= 1e-5 * o.abs_col_sums().max() * np.abs(x).max()
    # floor: rounding of segment totals in the inclusion-exclusion (FP32 data)
    fl_A = F32_FLOOR * normA * np.abs(y).max()
    fl_AT = F32_FLOOR * o.abs_col_sums().max() * np.abs(x).max()
    _assert_close(got_A, ref_A, mag_A, 1e-6, fl_A, "A y (fp32)")
    _assert_close(got_AT, ref_AT, mag_AT, 1e-6, fl_AT, "A^T x (fp32)")
    # the pair launch gives the same bits as the separate launches
    assert torch.equal(Ay, Ay2) and torch.equal(ATx, ATx2)
    # padding is written as zero
    for p, t in ((0, Ay), (1, ATx)):
        L = g.layouts[0][p]
        blk = t.cpu().numpy()[:L["n_seq"] * L["stride"]].reshape(L["n_seq"], L["stride"])
        assert np.all(blk[:, L["n_hands"]:] == 0)
    got_Ad = g.unpack(0, Ayd.cpu().numpy())[0]
    got_ATd = g.unpack(1, ATxd.cpu().numpy())[0]
    _assert_close(got_Ad, ref_A, mag_A, 1e-12, F64_FLOOR * normA * np.abs(y).max(), "A y (fp64)")
    _assert_close(got_ATd, ref_AT, mag_AT, 1e-12, F64_FLOOR * o.abs_col_sums().max() * np.abs(x).max(),
                  "A^T x (fp64)")
    g.close()


@pytest.mark.parametrize("name,fn", SMALL)
def test_matvec_small_games(name, fn):
    pmx = _need_gpu()
    _say("matvec parity", name)
    _check_matvecs(pmx, fn())


def test_matvec_river_full_size():
    pmx = _need_gpu()
    _say("matvec parity river 1081 hands")
    _check_matvecs(pmx, I.config(1), seed=3)


# river endgames with hand-ranking strengths and the asymmetric betting menu
# of the paper's appendix on Libratus' betting abstraction (166 and 82
# sequences per player)
LIBRATUS = [
    ("libratus_river_full", lambda: I.libratus_river(stack=1000.0)),
    ("libratus_river_ai2_pruned", lambda: I.libratus_river(seed=3, ai=1, stack=400.0, n_keep=(300, 260))),
]


@pytest.mark.parametrize("name,fn", LIBRATUS)
def test_matvec_libratus_menu_real_strengths(name, fn):
    pmx = _need_gpu()
    d = fn()
    _say("matvec parity", name)
    _check_matvecs(pmx, d, seed=5)
    o = payoff.Game(d)
    g = pmx.Game(d)
    rng = np.random.default_rng(6)
    y = _rand_vectors(o, rng, 1)
    x = _rand_vectors(o, rng, 0)
    ref_A, ref_AT = o.matvec_A(y), o.matvec_AT(x)
    mag_A, mag_AT = payoff.abs_matvec_A(o, y), payoff.abs_matvec_AT(o, x)
    fl_A = F32_FLOOR * o.abs_row_sums().max() * np.abs(y).max()
    fl_AT = F32_FLOOR * o.abs_col_sums().max() * np.abs(x).max()
    yd, xd = _dev(g.pack(1, [y]), np.float32), _dev(g.pack(0, [x]), np.float32)
    for sched in [(2, 1), (3, 1), (3, 4), (4, 2), (4, 8)]:
        _say("  schedule", sched)
        g.game_tune(*sched)
        Ay = torch.full((g.elems[0],), 3.0, dtype=torch.float32, device="cuda")
        ATx = torch.full((g.elems[1],), 3.0, dtype=torch.float32, device="cuda")
        g.matvec_pair(yd, xd, Ay, ATx)
        torch.cuda.synchronize()
        _assert_close(g.unpack(0, Ay.cpu().numpy())[0], ref_A, mag_A, 1e-6, fl_A, f"A y {sched}")
        _assert_close(g.unpack(1, ATx.cpu().numpy())[0], ref_AT, mag_AT, 1e-6, fl_AT, f"A^T x {sched}")
    g.close()


def test_isomorphic_hands_get_equal_values():
    """A monotone board (the three other suits permute freely) with ranges
    drawn per suit-isomorphism class and vectors constant on the classes:
    the oracle's and the device's A y and A^T x are constant on each class,
    so collapsing each class into one meta-hand (as the paper's experiments
    do) would lose nothing."""
    pmx = _need_gpu()
    from paper_2112_03804_amd import handeval
    board = [4 * r + 3 for r in (0, 3, 7, 9, 11)]          # 2s 5s 9s Js Ks
    d = I.river_config(seed=2, board=board, strengths="eval", iso_ranges=True, bet_fracs=(0.5, 1.0),
                       max_raises=2)
    _say("isomorphism invariance")
    cls = handeval.suit_classes(d.hands[0], d.board)
    assert np.array_equal(d.hands[0], d.hands[1]) and cls.max() + 1 < len(cls) // 2
    o = payoff.Game(d)
    g = pmx.Game(d)
    rng = np.random.default_rng(3)
    y = rng.random((o.S[1], cls.max() + 1))[:, cls]
    x = rng.random((o.S[0], cls.max() + 1))[:, cls]
    Ay = torch.zeros(g.elems[0], dtype=torch.float32, device="cuda")
    ATx = torch.zeros(g.elems[1], dtype=torch.float32, device="cuda")
    g.matvec_pair(_dev(g.pack(1, [y]), np.float32), _dev(g.pack(0, [x]), np.float32), Ay, ATx)
    Ayd = torch.zeros(g.elems[0], dtype=torch.float64, device="cuda")
    g.matvec_A_f64(_dev(g.pack(1, [y], np.float64), np.float64), Ayd)
    torch.cuda.synchronize()
    normA = o.abs_row_sums().max() * np.abs(y).max()
    normAT = o.abs_col_sums().max() * np.abs(x).max()
    for got, norm, rel in ((o.matvec_A(y), normA, 1e-12), (o.matvec_AT(x), normAT, 1e-12),
                           (g.unpack(0, Ay.cpu().numpy())[0].astype(np.float64), normA, 2e-6),
                           (g.unpack(1, ATx.cpu().numpy())[0].astype(np.float64), normAT, 2e-6),
                           (g.unpack(0, Ayd.cpu().numpy())[0], normA, 1e-12)):
        for c in range(cls.max() + 1):
            v = got[:, cls == c]
            assert np.abs(v - v[:, :1]).max() <= rel * norm, c
    g.close()


@pytest.mark.parametrize("name,fn", LIBRATUS)
def test_gap_and_step_libratus_menu(name, fn):
    """The FP64 gap of given strategies and one RM+ step from a given state
    on the menu games (trees deeper than one regret-update piece)."""
    pmx = _need_gpu()
    d = fn()
    _say("gap and step parity", name)
    o = payoff.Game(d)
    g = pmx.Game(d)
    rng = np.random.default_rng(12)
    x, y = _random_plans(o, rng)
    gap, b1, b2 = g.saddle_gap_of(_dev(g.pack(0, [x], np.float64), np.float64),
                                  _dev(g.pack(1, [y], np.float64), np.float64))
    rgap, rb1, rb2 = solver.saddle_gap(o, x, y)
    pot = 2 * d.contrib
    assert abs(b1[0] - rb1) <= 1e-9 * pot and abs(b2[0] - rb2) <= 1e-9 * pot
    assert abs(gap[0] - rgap) <= 1e-9 * pot and gap[0] >= 0
    ref = solver.RMPlus(o)
    t0, w0 = 3, 6.0
    for p in range(2):
        R = (rng.random((o.S[p], o.N[p])) * 3.0).astype(np.float32).astype(np.float64)
        xp = ref.tp[p].realization(ref.tp[p].behaviour_from_regret(R)).astype(np.float32).astype(np.float64)
        sm = rng.random((o.S[p], o.N[p]))
        ref.R[p], ref.x[p], ref.sum[p] = R, xp, sm.copy()
        g.solver_set_state(p, regret=g.pack(p, [R]), plan=g.pack(p, [xp]),
                           avg_sum=g.pack(p, [sm], np.float64), t=t0, wsum=w0)
    ref.t, ref.wsum = t0, w0
    g.solver_step(1)
    torch.cuda.synchronize()
    ref.step()
    for p in range(2):
        st = g.solver_get_state(p)
        R = g.unpack(p, st["regret"])[0]
        xp = g.unpack(p, st["plan"])[0]
        sm = g.unpack(p, st["avg_sum"])[0]
        scale = max(1.0, np.abs(ref.R[p]).max())
        assert np.abs(R - ref.R[p]).max() <= 1e-5 * scale, p
        assert np.abs(xp - ref.x[p]).max() <= 1e-5, p
        assert np.abs(sm - ref.sum[p]).max() <= 1e-6 * max(1.0, np.abs(ref.sum[p]).max()), p
    g.close()


@pytest.mark.parametrize("kernel", [2, 3, 4])
def test_matvec_max_hands(kernel):
    """The largest hand lists a game may hold (1280 per player, the top
    hands-per-thread class of each workgroup size) on a 57-card deck."""
    pmx = _need_gpu()
    d = I.river_config(seed=33, deck_size=57, bet_fracs=(0.75,), max_raises=1, n_keep=(1280, 1280),
                       name="river_max_hands")
    _say("matvec max hands, kernel", kernel)
    o = payoff.Game(d)
    g = pmx.Game(d)
    g.game_tune(kernel, 1)
    rng = np.random.default_rng(kernel)
    y = _rand_vectors(o, rng, 1)
    x = _rand_vectors(o, rng, 0)
    Ay = torch.zeros(g.elems[0], dtype=torch.float32, device="cuda")
    ATx = torch.zeros(g.elems[1], dtype=torch.float32, device="cuda")
    g.matvec_pair(_dev(g.pack(1, [y]), np.float32), _dev(g.pack(0, [x]), np.float32), Ay, ATx)
    Ayd = torch.zeros(g.elems[0], dtype=torch.float64, device="cuda")
    g.matvec_A_f64(_dev(g.pack(1, [y], np.float64), np.float64), Ayd)
    torch.cuda.synchronize()
    gA, gAT = g.unpack(0, Ay.cpu().numpy())[0], g.unpack(1, ATx.cpu().numpy())[0]
    gAd = g.unpack(0, Ayd.cpu().numpy())[0]
    normA = o.abs_row_sums().max() * np.abs(y).max()
    normAT = o.abs_col_sums().max() * np.abs(x).max()
    ref_A, ref_AT = o.matvec_A(y), o.matvec_AT(x)
    _assert_close(gA, ref_A, payoff.abs_matvec_A(o, y), 1e-6, F32_FLOOR * normA, "A y (fp32)")
    _assert_close(gAT, ref_AT, payoff.abs_matvec_AT(o, x), 1e-6, F32_FLOOR * normAT, "A^T x (fp32)")
    _assert_close(gAd, ref_A, payoff.abs_matvec_A(o, y), 1e-12, F64_FLOOR * normA, "A y (fp64)")
    g.close()


@pytest.mark.parametrize("kernel,rows", [(2, 1), (3, 2), (4, 1), (4, 8)])
def test_matvec_extreme_ragged_batch(kernel, rows):
    """One batch holding a 2-vs-3-hand instance, a 1280-hand instance on a
    57-card deck and a mid-size one (every hands-per-thread class at once);
    then one solver step of the batch equals each instance's own step."""
    pmx = _need_gpu()
    descs = [I.river_config(seed=41, n_keep=(2, 3), bet_fracs=(1.0,), max_raises=1),
             I.river_config(seed=42, deck_size=57, n_keep=(1280, 1277), bet_fracs=(0.5,), max_raises=1),
             I.river_config(seed=43, n_keep=(640, 333), bet_fracs=(0.33, 1.5), max_raises=2)]
    _say("extreme ragged batch", kernel, rows)
    g = pmx.Game(descs)
    g.game_tune(kernel, rows)
    os_ = [payoff.Game(d) for d in descs]
    rng = np.random.default_rng(77)
    ys = [_rand_vectors(o, rng, 1) for o in os_]
    xs = [_rand_vectors(o, rng, 0) for o in os_]
    Ay = torch.full((g.elems[0],), 5.0, dtype=torch.float32, device="cuda")
    ATx = torch.full((g.elems[1],), 5.0, dtype=torch.float32, device="cuda")
    g.matvec_pair(_dev(g.pack(1, ys), np.float32), _dev(g.pack(0, xs), np.float32), Ay, ATx)
    torch.cuda.synchronize()
    gA, gAT = g.unpack(0, Ay.cpu().numpy()), g.unpack(1, ATx.cpu().numpy())
    for i, o in enumerate(os_):
        fl = F32_FLOOR * o.abs_row_sums().max() * np.abs(ys[i]).max()
        _assert_close(gA[i], o.matvec_A(ys[i]), payoff.abs_matvec_A(o, ys[i]), 1e-6, fl, f"A y inst {i}")
        fl = F32_FLOOR * o.abs_col_sums().max() * np.abs(xs[i]).max()
        _assert_close(gAT[i], o.matvec_AT(xs[i]), payoff.abs_matvec_AT(o, xs[i]), 1e-6, fl, f"A^T x inst {i}")
    # the batch's iterates equal each instance solved on its own
    g.solver_step(7)
    torch.cuda.synchronize()
    for i, d in enumerate(descs):
        gi = pmx.Game(d)
        gi.game_tune(kernel, rows)
        gi.solver_step(7)
        torch.cuda.synchronize()
        for p in range(2):
            xb = g.unpack(p, g.solver_get_state(p)["plan"])[i]
            xi = gi.unpack(p, gi.solver_get_state(p)["plan"])[0]
            assert np.abs(xb - xi).max() <= 1e-6, (i, p)
        gi.close()
    g.close()


def test_matvec_batched_uneven():
    pmx = _need_gpu()
    descs = [I.river_config(seed=100 + i, n_keep=(40 + 37 * i, 200 - 13 * i),
                            bet_fracs=((0.5,), (0.33, 1.0), (0.75, 1.5, 2.0))[i % 3],
                            max_raises=2 + i % 3, pot=20.0 + 30 * i, stack=(1 + i) * 25.0)
             for i in range(6)]
    _say("matvec parity batch of", len(descs))
    g = pmx.Game(descs)
    os_ = [payoff.Game(d) for d in descs]
    rng = np.random.default_rng(9)
    ys = [_rand_vectors(o, rng, 1) for o in os_]
    xs = [_rand_vectors(o, rng, 0) for o in os_]
    Ay = torch.zeros(g.elems[0], dtype=torch.float32, device="cuda")
    ATx = torch.zeros(g.elems[1], dtype=torch.float32, device="cuda")
    g.matvec_pair(_dev(g.pack(1, ys), np.float32), _dev(g.pack(0, xs), np.float32), Ay, ATx)
    torch.cuda.synchronize()
    gA, gAT = g.unpack(0, Ay.cpu().numpy()), g.unpack(1, ATx.cpu().numpy())
    for i, o in enumerate(os_):
        fl = F32_FLOOR * o.abs_row_sums().max() * np.abs(ys[i]).max()
        _assert_close(gA[i], o.matvec_A(ys[i]), payoff.abs_matvec_A(o, ys[i]), 1e-6, fl, f"A y inst {i}")
        fl = F32_FLOOR * o.abs_col_sums().max() * np.abs(xs[i]).max()
        _assert_close(gAT[i], o.matvec_AT(xs[i]), payoff.abs_matvec_AT(o, xs[i]), 1e-6, fl,
                      f"A^T x inst {i}")
    g.close()


TR_SCHEDULES = [(2, 4), (2, 8), (3, 4), (3, 8), (4, 1), (4, 2), (4, 8)]   # the candidates the bench tunes over


def test_matvec_turn_river_full_size():
    """Every entry of A y and A^T x (FP32 under each schedule the bench
    tunes over, and FP64) on the full turn + river game, 19,480 sequences x
    1128 hands per player, against the oracle's definition-level sums."""
    pmx = _need_gpu()
    d = I.config(2)
    _say("matvec parity turn+river, every entry")
    o = payoff.Game(d)
    g = pmx.Game(d)
    rng = np.random.default_rng(21)
    y = _rand_vectors(o, rng, 1)
    x = _rand_vectors(o, rng, 0)
    yd, xd = _dev(g.pack(1, [y]), np.float32), _dev(g.pack(0, [x]), np.float32)
    ref_A, ref_AT = o.matvec_A(y), o.matvec_AT(x)
    mag_A, mag_AT = payoff.abs_matvec_A(o, y), payoff.abs_matvec_AT(o, x)
    normA, normAT = o.abs_row_sums().max(), o.abs_col_sums().max()
    fl_A, fl_AT = F32_FLOOR * normA * np.abs(y).max(), F32_FLOOR * normAT * np.abs(x).max()
    Ay = torch.empty(g.elems[0], dtype=torch.float32, device="cuda")
    ATx = torch.empty(g.elems[1], dtype=torch.float32, device="cuda")
    for sched in TR_SCHEDULES:
        _say("  schedule", sched)
        g.game_tune(*sched)
        Ay.fill_(7.0)
        ATx.fill_(7.0)
        g.matvec_pair(yd, xd, Ay, ATx)
        torch.cuda.synchronize()
        got_A = g.unpack(0, Ay.cpu().numpy())[0].astype(np.float64)
        got_AT = g.unpack(1, ATx.cpu().numpy())[0].astype(np.float64)
        assert np.abs(got_A - ref_A).max() <= 1e-5 * normA * np.abs(y).max()
        assert np.abs(got_AT - ref_AT).max() <= 1e-5 * normAT * np.abs(x).max()
        _assert_close(got_A, ref_A, mag_A, 1e-6, fl_A, f"A y (fp32, schedule {sched})")
        _assert_close(got_AT, ref_AT, mag_AT, 1e-6, fl_AT, f"A^T x (fp32, schedule {sched})")
    del Ay, ATx
    Ayd = torch.empty(g.elems[0], dtype=torch.float64, device="cuda")
    ATxd = torch.empty(g.elems[1], dtype=torch.float64, device="cuda")
    g.matvec_A_f64(_dev(g.pack(1, [y], np.float64), np.float64), Ayd)
    g.matvec_AT_f64(_dev(g.pack(0, [x], np.float64), np.float64), ATxd)
    torch.cuda.synchronize()
    _assert_close(g.unpack(0, Ayd.cpu().numpy())[0], ref_A, mag_A, 1e-12, F64_FLOOR * normA * np.abs(y).max(),
                  "A y (fp64)")
    _assert_close(g.unpack(1, ATxd.cpu().numpy())[0], ref_AT, mag_AT, 1e-12,
                  F64_FLOOR * normAT * np.abs(x).max(), "A^T x (fp64)")
    g.close()


# ---------------------------------------------------------------------------
# gap, single solver step, end-to-end solves
# ---------------------------------------------------------------------------

def _random_plans(o, rng):
    tp = [solver.Treeplex(o, p) for p in range(2)]
    return [tp[p].realization(tp[p].behaviour_from_regret(rng.random((o.S[p], o.N[p]))))
            for p in range(2)]


@pytest.mark.parametrize("name,fn", [SMALL[1], SMALL[3], SMALL[6], ("river", lambda: I.config(1))])
def test_gap_of_given_strategies(name, fn):
    pmx = _need_gpu()
    d = fn()
    _say("gap parity", name)
    o = payoff.Game(d)
    g = pmx.Game(d)
    rng = np.random.default_rng(4)
    x, y = _random_plans(o, rng)
    gap, b1, b2 = g.saddle_gap_of(_dev(g.pack(0, [x], np.float64), np.float64),
                                  _dev(g.pack(1, [y], np.float64), np.float64))
    rgap, rb1, rb2 = solver.saddle_gap(o, x, y)
    pot = 2 * d.contrib
    assert abs(b1[0] - rb1) <= 1e-9 * pot
    assert abs(b2[0] - rb2) <= 1e-9 * pot
    assert abs(gap[0] - rgap) <= 1e-9 * pot
    assert gap[0] >= 0
    g.close()


@pytest.mark.parametrize("name,fn", [SMALL[1], SMALL[2], SMALL[6], ("river", lambda: I.config(1))])
def test_single_solver_step_from_given_state(name, fn):
    pmx = _need_gpu()
    d = fn()
    _say("solver step parity", name)
    o = payoff.Game(d)
    g = pmx.Game(d)
    rng = np.random.default_rng(8)
    ref = solver.RMPlus(o)
    t0, w0 = 5, 15.0
    for p in range(2):
        R = (rng.random((o.S[p], o.N[p])) * 3.0).astype(np.float32).astype(np.float64)
        x = ref.tp[p].realization(ref.tp[p].behaviour_from_regret(R)).astype(np.float32).astype(np.float64)
        s = rng.random((o.S[p], o.N[p]))
        ref.R[p], ref.x[p], ref.sum[p] = R, x, s.copy()
        g.solver_set_state(p, regret=g.pack(p, [R]), plan=g.pack(p, [x]),
                           avg_sum=g.pack(p, [s], np.float64), t=t0, wsum=w0)
    ref.t, ref.wsum = t0, w0
    g.solver_step(1)
    torch.cuda.synchronize()
    ref.step()
    for p in range(2):
        st = g.solver_get_state(p)
        R = g.unpack(p, st["regret"])[0]
        x = g.unpack(p, st["plan"])[0]
        s = g.unpack(p, st["avg_sum"])[0]
        scale = max(1.0, np.abs(ref.R[p]).max())
        assert np.abs(R - ref.R[p]).max() <= 1e-5 * scale, p
        assert np.abs(x - ref.x[p]).max() <= 1e-5, p
        assert np.abs(s - ref.sum[p]).max() <= 1e-6 * max(1.0, np.abs(ref.sum[p]).max()), p
        assert st["t"] == t0 + 1 and st["wsum"] == w0 + t0 + 1
    g.close()


RM_KERNELS = {"lane": 0, "quad": 2 ** 31 - 1}   # solver_set_rm_quad: one lane / four lanes per hand


BIG_TREE = ("river_big_tree", lambda: I.river_config(seed=21, n_keep=(150, 170), bet_fracs=(0.33, 0.75, 1.5),
                                                      max_raises=4, stack=400.0))


@pytest.mark.parametrize("rmk", sorted(RM_KERNELS))
@pytest.mark.parametrize("kind", ["rm+", "dcfr"])
@pytest.mark.parametrize("rows", [8, 13, 64])
@pytest.mark.parametrize("name,fn", [SMALL[6], ("river", lambda: I.config(1)), BIG_TREE])
def test_single_step_any_piece_size(name, fn, rows, kind, rmk):
    """One solver step from a given state is the same whatever the cut of the
    treeplex into regret-update pieces (small cuts give several levels of
    pieces exchanging values through the stage buffer), with one lane or four
    lanes per hand."""
    pmx = _need_gpu()
    d = fn()
    _say("piece-size step parity", name, rows, kind, rmk)
    o = payoff.Game(d)
    g = pmx.Game(d)
    g.solver_set_task_rows(rows)
    g.solver_set_rm_quad(RM_KERNELS[rmk])
    g.solver_set_params(kind)
    rng = np.random.default_rng(21)
    ref = solver.RMPlus(o, kind=kind)
    t0, w0 = 6, 91.0
    for p in range(2):
        R = ((rng.random((o.S[p], o.N[p])) - 0.2) * 3.0).astype(np.float32).astype(np.float64)
        if kind == "rm+":
            R = np.maximum(R, 0.0)
        x = ref.tp[p].realization(ref.tp[p].behaviour_from_regret(R)).astype(np.float32).astype(np.float64)
        s = rng.random((o.S[p], o.N[p]))
        ref.R[p], ref.x[p], ref.sum[p] = R, x, s.copy()
        g.solver_set_state(p, regret=g.pack(p, [R]), plan=g.pack(p, [x]),
                           avg_sum=g.pack(p, [s], np.float64), t=t0, wsum=w0)
    ref.t, ref.wsum = t0, w0
    g.solver_step(1)
    torch.cuda.synchronize()
    ref.step()
    for p in range(2):
        st = g.solver_get_state(p)
        R = g.unpack(p, st["regret"])[0]
        x = g.unpack(p, st["plan"])[0]
        s = g.unpack(p, st["avg_sum"])[0]
        scale = max(1.0, np.abs(ref.R[p]).max())
        # regrets are continuous in the inputs: compared everywhere
        assert np.abs(R - ref.R[p]).max() <= 1e-5 * scale, p
        # the plan is the realization of the device's own regrets ...
        tp = ref.tp[p]
        assert np.abs(x - tp.realization(tp.behaviour_from_regret(R))).max() <= 1e-5, p
        # ... and the oracle's plan wherever it is well conditioned: where an
        # infoset's new regrets are all 0 (all its q equal, as under a river
        # card that blocks the hand, where the gradient is exactly 0) the
        # behaviour is the uniform convention and FP32 noise of ~1e-8 in g
        # may select another one, for the whole subtree below
        ok = np.ones_like(x, dtype=bool)
        for par, f, n in tp.inf:
            cond = np.maximum(ref.R[p][f:f + n], 0.0).sum(axis=0) > 1e-4 * scale
            ok[f:f + n] = (ok[par] if par >= 0 else True) & cond[None, :]
        assert ok.mean() > 0.5
        assert np.abs(x - ref.x[p])[ok].max() <= 1e-5, p
        assert np.abs(s - ref.sum[p]).max() <= 1e-6 * max(1.0, np.abs(ref.sum[p]).max()), p
    g.close()


@pytest.mark.parametrize("rmk", sorted(RM_KERNELS))
@pytest.mark.parametrize("kind", ["rm+", "dcfr"])
@pytest.mark.parametrize("tiny", [1e-30, 1e-42])
def test_single_step_tiny_regret_sums(tiny, kind, rmk):
    """Regret sums far below 1 (1e-30, and subnormal FP32 at 1e-42) give
    finite results: the walk's reciprocal is taken of a rescaled sum and no
    step passes through 1 / sum, which overflows FP32 for a subnormal sum (a
    hand whose gradient is 0 keeps its tiny regrets into the top-down pass).
    At 1e-30 the step matches the oracle to the usual tolerance; subnormal
    regrets times the gradient keep only a few bits, so at 1e-42 the check is
    finiteness and a plan that is the realization of the device's regrets."""
    pmx = _need_gpu()
    d = I.config(1)
    _say("tiny regret sums", tiny, kind, rmk)
    o = payoff.Game(d)
    g = pmx.Game(d)
    g.solver_set_params(kind)
    g.solver_set_rm_quad(RM_KERNELS[rmk])
    rng = np.random.default_rng(5)
    ref = solver.RMPlus(o, kind=kind)
    t0, w0 = 3, 6.0
    for p in range(2):
        R = (rng.random((o.S[p], o.N[p])) * tiny + tiny * 0.01).astype(np.float32).astype(np.float64)
        x = ref.tp[p].realization(ref.tp[p].behaviour_from_regret(R)).astype(np.float32).astype(np.float64)
        s = rng.random((o.S[p], o.N[p]))
        ref.R[p], ref.x[p], ref.sum[p] = R, x, s.copy()
        g.solver_set_state(p, regret=g.pack(p, [R]), plan=g.pack(p, [x]),
                           avg_sum=g.pack(p, [s], np.float64), t=t0, wsum=w0)
    ref.t, ref.wsum = t0, w0
    g.solver_step(1)
    torch.cuda.synchronize()
    ref.step()
    for p in range(2):
        st = g.solver_get_state(p)
        R = g.unpack(p, st["regret"])[0]
        x = g.unpack(p, st["plan"])[0]
        assert np.isfinite(R).all() and np.isfinite(x).all(), p
        scale = max(1.0, np.abs(ref.R[p]).max())
        if tiny >= 1e-37:
            assert np.abs(R - ref.R[p]).max() <= 1e-5 * scale, (p, np.abs(R - ref.R[p]).max())
        tp = ref.tp[p]
        assert np.abs(x - tp.realization(tp.behaviour_from_regret(R))).max() <= 1e-5, p
    g.close()


def test_piece_size_rejects_too_small():
    pmx = _need_gpu()
    g = pmx.Game(I.config(1))
    with pytest.raises(pmx.PmxError):
        g.solver_set_task_rows(2)      # an infoset of this tree has more actions
    with pytest.raises(pmx.PmxError):
        g.solver_set_task_rows(65)
    g.solver_step(3)                   # the previous cut is still in place
    torch.cuda.synchronize()
    g.close()


def test_rm_kernel_choice_rejects_negative():
    pmx = _need_gpu()
    g = pmx.Game(I.config(1))
    with pytest.raises(pmx.PmxError):
        g.solver_set_rm_quad(-1)
    g.solver_step(3)                   # the previous choice is still in place
    torch.cuda.synchronize()
    g.close()


@pytest.mark.parametrize("name,fn,target", [("tiny", I.tiny_config, 1e-6),
                                            ("kuhn", I.kuhn, 1e-5),
                                            ("river", lambda: I.config(1), 1e-4),
                                            ("turn_2card_deep", SMALL[6][1], 1e-4)])
def test_solve_to_target_and_certify(name, fn, target):
    pmx = _need_gpu()
    d = fn()
    _say("solve", name, "to", target)
    o = payoff.Game(d)
    g = pmx.Game(d)
    pot = 2 * d.contrib
    gap = np.inf
    # plain RM+ with linear averaging converges at about 1/T here: the 13-card
    # game needs ~1e5 iterations for 1e-6 * pot (the FP64 oracle needs as many)
    for k in range(300):
        g.solver_step(512)
        gap = g.saddle_gap()[0][0]
        if gap <= target * pot:
            break
    assert gap <= target * pot, gap / pot
    x = g.unpack(0, g.get_average_strategy(0))[0]
    y = g.unpack(1, g.get_average_strategy(1))[0]
    rgap, rb1, rb2 = solver.saddle_gap(o, x, y)
    assert abs(rgap - gap) <= 1e-9 * pot
    if d.deck_size <= 13:
        v, _ = solver.lp_value(o)
        assert rb2 - 1e-9 <= v <= rb1 + 1e-9
    g.close()


def test_batched_solver_per_instance_gaps():
    pmx = _need_gpu()
    descs = [I.river_config(seed=300 + i, n_keep=(60 + 50 * i, 250 - 30 * i),
                            bet_fracs=((0.5,), (0.33, 1.0), (0.75, 1.5, 2.0))[i % 3],
                            max_raises=2 + i % 3, pot=20.0 + 60 * i, stack=(1 + 2 * i) * 40.0)
             for i in range(5)]
    _say("batched solver, instances:", len(descs))
    g = pmx.Game(descs)
    os_ = [payoff.Game(d) for d in descs]
    g.solver_step(300)
    gap, b1, b2 = g.saddle_gap()
    xs = g.unpack(0, g.get_average_strategy(0))
    ys = g.unpack(1, g.get_average_strategy(1))
    for i, (o, d) in enumerate(zip(os_, descs)):
        rgap, rb1, rb2 = solver.saddle_gap(o, xs[i], ys[i])
        pot = 2 * d.contrib
        assert abs(gap[i] - rgap) <= 1e-9 * pot, i
        assert abs(b1[i] - rb1) <= 1e-9 * pot and abs(b2[i] - rb2) <= 1e-9 * pot, i
        assert gap[i] >= 0 and gap[i] < 0.05 * pot, (i, gap[i] / pot)
    # a batch iterates every instance exactly as a game of its own would
    g1 = pmx.Game(descs[2])
    g1.solver_step(300)
    x1 = g1.unpack(0, g1.get_average_strategy(0))[0]
    assert np.abs(x1 - xs[2]).max() <= 1e-6
    g.close()
    g1.close()


def test_solver_state_round_trip_and_reset():
    pmx = _need_gpu()
    d = I.small_river(2)
    _say("solver state round trip")
    g = pmx.Game(d)
    g.solver_step(40)
    st = [g.solver_get_state(p) for p in range(2)]
    gap_a = g.saddle_gap()[0][0]
    g.solver_step(40)
    gap_b = g.saddle_gap()[0][0]
    # restore the checkpoint and replay: identical results
    for p in range(2):
        g.solver_set_state(p, st[p]["regret"], st[p]["plan"], st[p]["avg_sum"], st[p]["t"], st[p]["wsum"])
    assert g.saddle_gap()[0][0] == gap_a
    g.solver_step(40)
    assert g.saddle_gap()[0][0] == gap_b
    g.solver_reset()
    g.solver_step(40)
    assert g.solver_get_state(0)["t"] == 40
    assert np.array_equal(g.solver_get_state(0)["avg_sum"], st[0]["avg_sum"])
    g.close()


@pytest.mark.parametrize("kernel,rows", [(2, 1), (2, 3), (3, 1), (3, 4), (4, 1), (4, 3), (4, 8)])
def test_matvec_schedules_agree(kernel, rows):
    """Every matvec schedule (the chunk-aligned layout with 256- or 512-thread
    workgroups, or the grouped layout; any chunk length) gives the oracle's
    products on a batch of uneven games, including a turn + river game whose
    rows span several board contexts."""
    pmx = _need_gpu()
    descs = [I.river_config(seed=500 + i, n_keep=(90 + 170 * i, 700 - 120 * i),
                            bet_fracs=((0.5,), (0.33, 1.0), (0.75, 1.5, 2.0))[i % 3],
                            max_raises=2 + i % 2, pot=30.0 + 40 * i, stack=(2 + i) * 35.0)
             for i in range(4)]
    descs.append(I.small_turn_river(4, deck_size=10, n_board=3, cards_per_hand=2,
                                    bet_fracs=(0.5, 1.0), max_raises=1, stack=30.0, zero_frac=0.2))
    _say("matvec schedule", kernel, rows)
    g = pmx.Game(descs)
    g.game_tune(kernel, rows)
    assert g.game_get_tuning() == (kernel, rows)
    os_ = [payoff.Game(d) for d in descs]
    rng = np.random.default_rng(kernel * 10 + rows)
    ys = [_rand_vectors(o, rng, 1) for o in os_]
    xs = [_rand_vectors(o, rng, 0) for o in os_]
    Ay = torch.full((g.elems[0],), 3.0, dtype=torch.float32, device="cuda")
    ATx = torch.full((g.elems[1],), 3.0, dtype=torch.float32, device="cuda")
    g.matvec_pair(_dev(g.pack(1, ys), np.float32), _dev(g.pack(0, xs), np.float32), Ay, ATx)
    Ayd = torch.zeros(g.elems[0], dtype=torch.float64, device="cuda")
    g.matvec_A_f64(_dev(g.pack(1, ys, np.float64), np.float64), Ayd)
    torch.cuda.synchronize()
    gA, gAT = g.unpack(0, Ay.cpu().numpy()), g.unpack(1, ATx.cpu().numpy())
    gAd = g.unpack(0, Ayd.cpu().numpy())
    for i, o in enumerate(os_):
        fl = F32_FLOOR * o.abs_row_sums().max() * np.abs(ys[i]).max()
        mag = payoff.abs_matvec_A(o, ys[i])
        ref = o.matvec_A(ys[i])
        _assert_close(gA[i], ref, mag, 1e-6, fl, f"A y inst {i}")
        _assert_close(gAd[i], ref, mag, 1e-12, F64_FLOOR / F32_FLOOR * fl, f"A y fp64 inst {i}")
        fl = F32_FLOOR * o.abs_col_sums().max() * np.abs(xs[i]).max()
        _assert_close(gAT[i], o.matvec_AT(xs[i]), payoff.abs_matvec_AT(o, xs[i]), 1e-6, fl,
                      f"A^T x inst {i}")
    # padding written as zero by every schedule
    flatA = Ay.cpu().numpy()
    for i in range(len(descs)):
        L = g.layouts[i][0]
        blk = flatA[L["vec_offset"]:L["vec_offset"] + L["n_seq"] * L["stride"]].reshape(L["n_seq"], L["stride"])
        assert np.all(blk[:, L["n_hands"]:] == 0)
    # the solver runs on the tuned schedule too (graph re-captured)
    g.solver_step(40)
    gap = g.saddle_gap()[0]
    assert np.all(gap >= 0)
    g.close()


@pytest.mark.parametrize("rmk", sorted(RM_KERNELS))
def test_retired_instances_stay_frozen(rmk):
    pmx = _need_gpu()
    descs = [I.river_config(seed=900 + i, n_keep=(120, 140), bet_fracs=(0.5, 1.0), max_raises=2,
                            pot=40.0, stack=120.0) for i in range(3)]
    _say("retirement", rmk)
    g = pmx.Game(descs)
    g.solver_set_rm_quad(RM_KERNELS[rmk])
    g.solver_step(40)
    before = [g.unpack(p, g.solver_get_state(p)["avg_sum"]) for p in range(2)]
    gap0 = g.saddle_gap()[0]
    g.solver_set_active([1, 0, 1])
    g.solver_step(40)
    after = [g.unpack(p, g.solver_get_state(p)["avg_sum"]) for p in range(2)]
    for p in range(2):
        assert np.array_equal(before[p][1], after[p][1])
        assert not np.array_equal(before[p][0], after[p][0])
        assert not np.array_equal(before[p][2], after[p][2])
    # halving the active set rebuilds the launch lists without the retired
    # instances; their state stays as it was
    g.solver_set_active([0, 0, 1])
    g.solver_step(8)
    mid = [g.unpack(p, g.solver_get_state(p)["avg_sum"]) for p in range(2)]
    for p in range(2):
        assert np.array_equal(after[p][0], mid[p][0]) and np.array_equal(after[p][1], mid[p][1])
        assert not np.array_equal(after[p][2], mid[p][2])
    # reactivated instances must be in the lists again
    g.solver_set_active([1, 1, 1])
    g.solver_step(8)
    end = [g.unpack(p, g.solver_get_state(p)["avg_sum"]) for p in range(2)]
    for p in range(2):
        for i in range(3):
            assert not np.array_equal(mid[p][i], end[p][i]), (p, i)
    # every instance retired: iterations still count, nothing changes
    g.solver_set_active([0, 0, 0])
    t0 = g.solver_get_state(0)["t"]
    g.solver_step(4)
    st = g.solver_get_state(0)
    assert st["t"] == t0 + 4
    assert all(np.array_equal(a, b) for a, b in zip(end[0], g.unpack(0, st["avg_sum"])))
    g.solver_reset()
    g.solver_step(8)
    assert all(np.abs(a).sum() > 0 for a in g.unpack(0, g.solver_get_state(0)["avg_sum"]))
    assert gap0.shape == (3,)
    g.close()


def _retire_descs(n):
    return [I.river_config(seed=930 + i, n_keep=(100, 120), bet_fracs=(0.5, 1.0), max_raises=2,
                           pot=40.0, stack=120.0) for i in range(n)]


def test_retired_average_keeps_its_own_weight():
    """A retired instance's averages are divided by the weights of the
    iterations it took part in, not by the batch's running total: its average
    strategy and gap stay as they were at retirement, and the gap of every
    instance matches the oracle's on the normalized averages."""
    pmx = _need_gpu()
    descs = _retire_descs(3)
    _say("retired averages")
    g = pmx.Game(descs)
    g.solver_step(24)
    avg0 = [g.unpack(p, g.get_average_strategy(p)) for p in range(2)]
    gap0 = g.saddle_gap()[0]
    g.solver_set_active([1, 0, 1])
    g.solver_step(40)
    w = g.solver_get_weights()
    assert w[1] == sum(range(1, 25)) and w[0] == w[2] == sum(range(1, 65))
    assert g.solver_get_state(0)["wsum"] == w[0]
    avg1 = [g.unpack(p, g.get_average_strategy(p)) for p in range(2)]
    gap1 = g.saddle_gap()[0]
    for p in range(2):
        assert np.array_equal(avg0[p][1], avg1[p][1])
    assert abs(gap1[1] - gap0[1]) <= 1e-12 * 2 * descs[1].contrib
    for i, d in enumerate(descs):
        o = payoff.Game(d)
        rgap, _, _ = solver.saddle_gap(o, avg1[0][i], avg1[1][i])
        assert abs(gap1[i] - rgap) <= 1e-9 * 2 * d.contrib, (i, gap1[i], rgap)
    # the totals travel with the state
    st = [g.solver_get_state(p) for p in range(2)]
    g.solver_reset()
    for p in range(2):
        g.solver_set_state(p, st[p]["regret"], st[p]["plan"], st[p]["avg_sum"], st[p]["t"], st[p]["wsum"])
    assert np.all(g.solver_get_weights() == st[0]["wsum"])
    g.solver_set_weights(w)
    assert np.array_equal(g.solver_get_weights(), w)
    assert np.allclose(g.saddle_gap()[0], gap1, rtol=0, atol=1e-12 * 2 * descs[0].contrib)
    with pytest.raises(pmx.PmxError):
        g.solver_set_weights(np.array([1.0, -1.0, 1.0]))
    g.close()


def test_gap_recomputes_only_changed_instances():
    """Gaps of retired instances are reused; the instances computed alone, on
    the solver's lists with and without retired instances, agree with a full
    recomputation."""
    pmx = _need_gpu()
    descs = _retire_descs(4)
    _say("partial gap")
    g = pmx.Game(descs)
    tol = 1e-12 * 2 * max(d.contrib for d in descs)

    def full():
        g.solver_set_weights(g.solver_get_weights())   # drops every kept value
        return g.saddle_gap()

    g.solver_step(16)
    g.saddle_gap()
    g.solver_set_active([1, 0, 1, 1])                  # lists keep the retired instance
    g.solver_step(16)
    part = g.saddle_gap()
    ref = full()
    for a, b in zip(part, ref):
        assert np.allclose(a, b, rtol=0, atol=tol)
    g.solver_set_active([0, 0, 1, 0])                  # lists rebuilt without three
    g.solver_step(16)
    part = g.saddle_gap()
    ref = full()
    for a, b in zip(part, ref):
        assert np.allclose(a, b, rtol=0, atol=tol)
    for i, d in enumerate(descs):
        o = payoff.Game(d)
        avg = [g.unpack(p, g.get_average_strategy(p))[i] for p in range(2)]
        rgap, _, _ = solver.saddle_gap(o, avg[0], avg[1])
        assert abs(part[0][i] - rgap) <= 1e-9 * 2 * d.contrib, (i, part[0][i], rgap)
    # a state import drops the kept values of retired instances too
    st = [g.solver_get_state(p) for p in range(2)]
    w = g.solver_get_weights()
    g.solver_reset()
    g.solver_step(4)
    g.solver_set_active([0, 0, 1, 0])
    other = g.saddle_gap()[0]
    assert not np.allclose(other, ref[0], rtol=0, atol=tol)
    for p in range(2):
        g.solver_set_state(p, st[p]["regret"], st[p]["plan"], st[p]["avg_sum"], st[p]["t"], st[p]["wsum"])
    g.solver_set_weights(w)
    assert np.allclose(g.saddle_gap()[0], ref[0], rtol=0, atol=tol)
    g.close()


def test_instance_retired_before_any_iteration_keeps_its_plan():
    pmx = _need_gpu()
    descs = _retire_descs(3)
    _say("retired at start")
    g = pmx.Game(descs)
    plan0 = [g.unpack(p, g.solver_get_state(p)["plan"]) for p in range(2)]
    gap0 = g.saddle_gap()[0]
    g.solver_set_active([1, 0, 1])
    g.solver_step(16)
    assert g.solver_get_weights()[1] == 0.0
    gap1 = g.saddle_gap()[0]
    assert abs(gap1[1] - gap0[1]) <= 1e-12 * 2 * descs[1].contrib
    for p in range(2):
        avg = g.unpack(p, g.get_average_strategy(p))
        assert np.array_equal(avg[1], plan0[p][1].astype(np.float64))
    o = payoff.Game(descs[0])
    avg = [g.unpack(p, g.get_average_strategy(p))[0] for p in range(2)]
    rgap, _, _ = solver.saddle_gap(o, avg[0], avg[1])
    assert abs(gap1[0] - rgap) <= 1e-9 * 2 * descs[0].contrib
    g.close()


@pytest.mark.parametrize("name,fn", [SMALL[2], SMALL[6], ("river", lambda: I.config(1))])
def test_dcfr_single_step_from_given_state(name, fn):
    pmx = _need_gpu()
    d = fn()
    _say("DCFR step parity", name)
    o = payoff.Game(d)
    g = pmx.Game(d)
    g.solver_set_params("dcfr", alpha=1.5, beta=0.0, gamma=2)
    rng = np.random.default_rng(13)
    ref = solver.RMPlus(o, kind="dcfr", alpha=1.5, beta=0.0, gamma=2)
    t0, w0 = 7, 140.0
    for p in range(2):
        R = ((rng.random((o.S[p], o.N[p])) - 0.3) * 3.0).astype(np.float32).astype(np.float64)
        x = ref.tp[p].realization(ref.tp[p].behaviour_from_regret(R)).astype(np.float32).astype(np.float64)
        s = rng.random((o.S[p], o.N[p]))
        ref.R[p], ref.x[p], ref.sum[p] = R, x, s.copy()
        g.solver_set_state(p, regret=g.pack(p, [R]), plan=g.pack(p, [x]),
                           avg_sum=g.pack(p, [s], np.float64), t=t0, wsum=w0)
    ref.t, ref.wsum = t0, w0
    g.solver_step(1)
    torch.cuda.synchronize()
    ref.step()
    for p in range(2):
        st = g.solver_get_state(p)
        R = g.unpack(p, st["regret"])[0]
        x = g.unpack(p, st["plan"])[0]
        s = g.unpack(p, st["avg_sum"])[0]
        scale = max(1.0, np.abs(ref.R[p]).max())
        assert np.abs(R - ref.R[p]).max() <= 1e-5 * scale, p
        assert np.abs(x - ref.x[p]).max() <= 1e-5, p
        assert np.abs(s - ref.sum[p]).max() <= 1e-6 * max(1.0, np.abs(ref.sum[p]).max()), p
        assert st["wsum"] == w0 + (t0 + 1) ** 2
    g.close()


def test_dcfr_solve_river_certified():
    pmx = _need_gpu()
    d = I.config(1)
    _say("DCFR solve river")
    o = payoff.Game(d)
    g = pmx.Game(d)
    g.solver_set_params("dcfr")
    pot = 2 * d.contrib
    gap = np.inf
    for _ in range(100):
        g.solver_step(64)
        gap = g.saddle_gap()[0][0]
        if gap <= 1e-4 * pot:
            break
    assert gap <= 1e-4 * pot
    x = g.unpack(0, g.get_average_strategy(0))[0]
    y = g.unpack(1, g.get_average_strategy(1))[0]
    rgap, _, _ = solver.saddle_gap(o, x, y)
    assert abs(rgap - gap) <= 1e-9 * pot
    g.close()


def _technique_b_products(o, y, x):
    """A y and A^T x through Technique B's postprocessed factors
    (Ahat + U M^-1 V^T), moved back to sequence-major layout."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import spsolve_triangular
    from oracle import sparsify
    Ahat, U, M, V, order = sparsify.factors(o)
    U, M, V = sparsify.postprocess(U, M, V)
    M = sp.csr_matrix(M)
    (S1, S2), (N1, N2) = o.S, o.N
    yh = y.T.reshape(-1)                               # hand-major: h2 * S2 + s2
    z = spsolve_triangular(M, V.T @ yh, lower=True, unit_diagonal=True)
    a = (Ahat @ yh + U @ z).reshape(N1, S1)            # Player 1's hands in `order`
    Ay = np.empty((N1, S1))
    Ay[order] = a
    xh = np.empty((N1, S1))
    xh[:] = x.T[order]
    xh = xh.reshape(-1)
    w = spsolve_triangular(sp.csr_matrix(M.T), U.T @ xh, lower=False, unit_diagonal=True)
    ATx = (Ahat.T @ xh + V @ w).reshape(N2, S2)
    return Ay.T, ATx.T


@pytest.mark.parametrize("name,fn", [("river_pruned_mid", SMALL[7][1]), ("river", lambda: I.config(1))])
def test_matvec_matches_technique_b_factors(name, fn):
    """The structured matvecs against the paper's own sparsified form of A
    (the factor route agrees with the oracle's direct sum to about 5e-17 of
    ||A|| ||v|| on these games, so the usual FP64 bound holds)."""
    pmx = _need_gpu()
    d = fn()
    _say("technique B cross-check", name)
    o = payoff.Game(d)
    rng = np.random.default_rng(17)
    y = _rand_vectors(o, rng, 1)
    x = _rand_vectors(o, rng, 0)
    ref_A, ref_AT = _technique_b_products(o, y, x)
    g = pmx.Game(d)
    Ay = torch.zeros(g.elems[0], dtype=torch.float32, device="cuda")
    ATx = torch.zeros(g.elems[1], dtype=torch.float32, device="cuda")
    g.matvec_pair(_dev(g.pack(1, [y]), np.float32), _dev(g.pack(0, [x]), np.float32), Ay, ATx)
    Ayd = torch.zeros(g.elems[0], dtype=torch.float64, device="cuda")
    ATxd = torch.zeros(g.elems[1], dtype=torch.float64, device="cuda")
    g.matvec_A_f64(_dev(g.pack(1, [y], np.float64), np.float64), Ayd)
    g.matvec_AT_f64(_dev(g.pack(0, [x], np.float64), np.float64), ATxd)
    torch.cuda.synchronize()
    normA = o.abs_row_sums().max() * np.abs(y).max()
    normAT = o.abs_col_sums().max() * np.abs(x).max()
    magA, magAT = payoff.abs_matvec_A(o, y), payoff.abs_matvec_AT(o, x)
    _assert_close(g.unpack(0, Ay.cpu().numpy())[0], ref_A, magA, 1e-6, F32_FLOOR * normA, "A y (fp32)")
    _assert_close(g.unpack(1, ATx.cpu().numpy())[0], ref_AT, magAT, 1e-6, F32_FLOOR * normAT, "A^T x (fp32)")
    _assert_close(g.unpack(0, Ayd.cpu().numpy())[0], ref_A, magA, 1e-12, F64_FLOOR * normA, "A y (fp64)")
    _assert_close(g.unpack(1, ATxd.cpu().numpy())[0], ref_AT, magAT, 1e-12, F64_FLOOR * normAT, "A^T x (fp64)")
    g.close()


def test_turn_river_gap_full_size_certified():
    """The FP64 saddle gap and best responses of the full turn + river game
    (19,480 sequences x 1128 hands per player) agree with the oracle to
    1e-9 * pot, on random strategies and on the averages of 1024 DCFR
    iterations (the solver and gap of the precision run)."""
    pmx = _need_gpu()
    d = I.config(2)
    _say("turn+river gap, full size")
    o = payoff.Game(d)
    g = pmx.Game(d)
    pot = 2 * d.contrib
    rng = np.random.default_rng(12)
    x, y = _random_plans(o, rng)
    gap, b1, b2 = g.saddle_gap_of(_dev(g.pack(0, [x], np.float64), np.float64),
                                  _dev(g.pack(1, [y], np.float64), np.float64))
    rgap, rb1, rb2 = solver.saddle_gap(o, x, y)
    _say(f"  random strategies: gap/pot {gap[0] / pot:.6e}, oracle {rgap / pot:.6e}")
    assert abs(b1[0] - rb1) <= 1e-9 * pot and abs(b2[0] - rb2) <= 1e-9 * pot
    assert abs(gap[0] - rgap) <= 1e-9 * pot
    g.solver_set_params("dcfr")
    g.solver_step(1024)
    gap, b1, b2 = g.saddle_gap()
    xa = g.unpack(0, g.get_average_strategy(0))[0]
    ya = g.unpack(1, g.get_average_strategy(1))[0]
    rgap, rb1, rb2 = solver.saddle_gap(o, xa, ya)
    _say(f"  DCFR averages after 1024 iterations: gap/pot {gap[0] / pot:.6e}, oracle {rgap / pot:.6e}")
    assert abs(b1[0] - rb1) <= 1e-9 * pot and abs(b2[0] - rb2) <= 1e-9 * pot
    assert abs(gap[0] - rgap) <= 1e-9 * pot
    assert 0 <= gap[0] < 1e-3 * pot
    g.close()


def test_gap_guard_flags_a_growing_gap():
    """Failure detection: the gap of a solve that keeps growing is an error.
    Halving the weight totals doubles every average (a best-response value is
    positively homogeneous), so each check finds the gap grown: the third
    growth in a row raises with guard 3, never with the guard off, and an
    ordinary solve checked 20 times under the default guard raises nothing.
    A non-finite average is an error whatever the guard."""
    pmx = _need_gpu()
    d = I.small_river(0)
    _say("gap guard")
    g = pmx.Game(d)
    for _ in range(20):
        g.solver_step(16)
        g.saddle_gap()
    w = g.solver_get_weights()
    g.solver_set_gap_guard(3)
    g0 = g.saddle_gap()[0][0]
    for k in range(2):
        w = w * 0.5
        g.solver_set_weights(w)
        assert g.saddle_gap()[0][0] > g0
    w = w * 0.5
    g.solver_set_weights(w)
    with pytest.raises(pmx.PmxError, match="grew"):
        g.saddle_gap()
    g.solver_set_gap_guard(0)
    for _ in range(4):
        w = w * 0.5
        g.solver_set_weights(w)
        g.saddle_gap()
    with pytest.raises(pmx.PmxError):
        g.solver_set_gap_guard(-1)
    # a NaN in the averages: a non-finite best response
    st = g.solver_get_state(0)
    s = st["avg_sum"].copy()
    s[0] = np.nan
    g.solver_set_state(0, regret=st["regret"], plan=st["plan"], avg_sum=s, t=st["t"], wsum=st["wsum"])
    g.solver_set_weights(w)
    with pytest.raises(pmx.PmxError, match="non-finite"):
        g.saddle_gap()
    g.close()


@pytest.mark.parametrize("name,fn", [("small_river_pruned", SMALL[3][1]), ("river_pruned_mid", SMALL[7][1]),
                                     ("river", lambda: I.config(1))])
def test_matvec_through_explicit_technique_b_factors(name, fn):
    """The library's own explicit Technique-B factors (CSR products for Ahat,
    U, V and M's chain solve by pointer jumping, FP64) give the oracle's A y
    and A^T x elementwise, and the structured FP64 products."""
    pmx = _need_gpu()
    d = fn()
    _say("explicit factors", name)
    o = payoff.Game(d)
    g = pmx.Game(d)
    sizes = g.tb_build()
    rng = np.random.default_rng(5)
    y = _rand_vectors(o, rng, 1)
    x = _rand_vectors(o, rng, 0)
    yd, xd = _dev(g.pack(1, [y], np.float64), np.float64), _dev(g.pack(0, [x], np.float64), np.float64)
    Ay = torch.full((g.elems[0],), 3.0, dtype=torch.float64, device="cuda")
    ATx = torch.full((g.elems[1],), 3.0, dtype=torch.float64, device="cuda")
    g.matvec_A_tb(yd, Ay)
    g.matvec_AT_tb(xd, ATx)
    torch.cuda.synchronize()
    ref_A, ref_AT = o.matvec_A(y), o.matvec_AT(x)
    normA = o.abs_row_sums().max() * np.abs(y).max()
    normAT = o.abs_col_sums().max() * np.abs(x).max()
    _assert_close(g.unpack(0, Ay.cpu().numpy())[0], ref_A, payoff.abs_matvec_A(o, y), 1e-12, F64_FLOOR * normA,
                  "A y (explicit factors)")
    _assert_close(g.unpack(1, ATx.cpu().numpy())[0], ref_AT, payoff.abs_matvec_AT(o, x), 1e-12,
                  F64_FLOOR * normAT, "A^T x (explicit factors)")
    # padding rows are written as zero
    for p, t in ((0, Ay), (1, ATx)):
        L = g.layouts[0][p]
        blk = t.cpu().numpy()[:L["n_seq"] * L["stride"]].reshape(L["n_seq"], L["stride"])
        assert np.all(blk[:, L["n_hands"]:] == 0)
    assert sizes["nnz_v_pp"] <= sizes["nnz_v"] and sizes["m_dim_pp"] <= sizes["m_dim"]
    g.close()


def test_autotuner_picks_the_fastest_timed_schedule_and_caches_it(tmp_path):
    """Both objectives time every candidate, apply the fastest and store it
    under a key of their own; a second game of the same size class takes the
    stored choice without timing.  The iteration objective leaves the solver
    reset."""
    pmx = _need_gpu()
    from paper_2112_03804_amd import autotune
    d = I.river_config(seed=7, n_keep=(300, 517), bet_fracs=(0.33, 1.5))
    _say("autotuner")
    g = pmx.Game(d)
    cands = [(2, 1), (3, 1), (4, 1)]
    cache = str(tmp_path / "tune.json")
    for obj in ("products", "iteration"):
        sched, t = autotune.tune(g, candidates=cands, cache_path=cache, objective=obj)
        assert set(t) == {f"{k}:{r}" for k, r in cands} and all(v > 0 for v in t.values())
        assert t[f"{sched[0]}:{sched[1]}"] == min(t.values())
        assert g.game_get_tuning() == sched
        g2 = pmx.Game(d)
        g2.game_tune(2, 4)
        sched2, t2 = autotune.tune(g2, candidates=cands, cache_path=cache, objective=obj)
        assert sched2 == sched and t2 == {} and g2.game_get_tuning() == sched
        g2.close()
    st = g.solver_get_state(0)
    assert st["t"] == 0 and np.all(st["regret"] == 0)
    g.close()


@pytest.mark.parametrize("rows", [1, 2, 8])
def test_matvec_batch_with_two_wide_and_split_groups(rows):
    """A batch with enough output rows (at least 1024 per direction) for the
    two-wide groups and the split groups (prefix slots for the showdown
    components only, the identical hand read from its staging row): every
    entry of A y and A^T x against the oracle."""
    pmx = _need_gpu()
    descs = I.batched_configs(24, seed=8)
    _say("matvec parity, batch with two-wide and split groups, groups per chunk", rows)
    g = pmx.Game(descs)
    g.game_tune(4, rows)
    os_ = [payoff.Game(d) for d in descs]
    assert sum(o.S[0] for o in os_) >= 1024 and sum(o.S[1] for o in os_) >= 1024
    rng = np.random.default_rng(30 + rows)
    ys = [_rand_vectors(o, rng, 1) for o in os_]
    xs = [_rand_vectors(o, rng, 0) for o in os_]
    Ay = torch.full((g.elems[0],), 9.0, dtype=torch.float32, device="cuda")
    ATx = torch.full((g.elems[1],), 9.0, dtype=torch.float32, device="cuda")
    g.matvec_pair(_dev(g.pack(1, ys), np.float32), _dev(g.pack(0, xs), np.float32), Ay, ATx)
    # the single-direction launches the solver makes give the same bits
    Ay1 = torch.zeros_like(Ay)
    ATx1 = torch.zeros_like(ATx)
    g.matvec_A(_dev(g.pack(1, ys), np.float32), Ay1)
    g.matvec_AT(_dev(g.pack(0, xs), np.float32), ATx1)
    torch.cuda.synchronize()
    assert torch.equal(Ay, Ay1) and torch.equal(ATx, ATx1)
    gA, gAT = g.unpack(0, Ay.cpu().numpy()), g.unpack(1, ATx.cpu().numpy())
    for i, o in enumerate(os_):
        fl = F32_FLOOR * o.abs_row_sums().max() * np.abs(ys[i]).max()
        _assert_close(gA[i], o.matvec_A(ys[i]), payoff.abs_matvec_A(o, ys[i]), 1e-6, fl, f"A y inst {i}")
        fl = F32_FLOOR * o.abs_col_sums().max() * np.abs(xs[i]).max()
        _assert_close(gAT[i], o.matvec_AT(xs[i]), payoff.abs_matvec_AT(o, xs[i]), 1e-6, fl, f"A^T x inst {i}")
    g.close()
