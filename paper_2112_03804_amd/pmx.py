"""ctypes binding of libpmx (the C ABI declared in include/pmx.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch tensors on the current HIP device (passed
by ``data_ptr()``); streams are taken from torch's current stream.  The
binding never computes a result itself and raises if the built library is
missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Sequence, Union

import numpy as np

from .instances import GameDesc

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmx.so")

PMX_OK, PMX_EINVAL, PMX_ENOMEM, PMX_EDEVICE, PMX_ESTATE, PMX_ENUMERIC = 0, -1, -2, -3, -4, -5
FOLD_P1, FOLD_P2, SHOWDOWN = 0, 1, 2

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_u8p = ctypes.POINTER(ctypes.c_uint8)
_c_f64p = ctypes.POINTER(ctypes.c_double)
_c_f32p = ctypes.POINTER(ctypes.c_float)


class GameDescC(ctypes.Structure):
    _fields_ = [
        ("deck_size", ctypes.c_int32), ("cards_per_hand", ctypes.c_int32),
        ("n_board", ctypes.c_int32), ("board", _c_u8p),
        ("n_river", ctypes.c_int32), ("river_cards", _c_u8p),
        ("n_hands", ctypes.c_int32 * 2), ("hand_cards", _c_u8p * 2),
        ("strength", _c_i32p * 2), ("range", _c_f64p * 2),
        ("contrib", ctypes.c_double), ("stack", ctypes.c_double * 2),
        ("n_bet_fracs", ctypes.c_int32), ("bet_fracs", _c_f64p),
        ("max_raises", ctypes.c_int32), ("allow_allin", ctypes.c_int32),
        ("bet_menu_len", _c_i32p), ("bet_menu", _c_f64p),
    ]


class LayoutC(ctypes.Structure):
    _fields_ = [
        ("n_seq", ctypes.c_int32), ("n_hands", ctypes.c_int32), ("stride", ctypes.c_int32),
        ("vec_offset", ctypes.c_int64), ("vec_elems", ctypes.c_int64),
        ("n_infosets", ctypes.c_int32),
        ("infoset_parent", _c_i32p), ("infoset_first", _c_i32p),
        ("infoset_nact", _c_i32p), ("infoset_board", _c_i32p),
    ]


class TerminalsC(ctypes.Structure):
    _fields_ = [
        ("n_terminals", ctypes.c_int32),
        ("seq1", _c_i32p), ("seq2", _c_i32p), ("kind", _c_i32p), ("board", _c_i32p),
        ("runout", _c_i32p), ("c1", _c_f64p), ("c2", _c_f64p),
    ]


class HandMetaC(ctypes.Structure):
    _fields_ = [
        ("n_hands", ctypes.c_int32), ("n_live", ctypes.c_int32),
        ("rank", _c_i32p), ("lt", _c_i32p), ("le", _c_i32p), ("self_", _c_i32p),
        ("beta", ctypes.c_double),
    ]


class TbSizesC(ctypes.Structure):
    _fields_ = [("nnz_A", ctypes.c_int64), ("nnz_ahat", ctypes.c_int64), ("nnz_u", ctypes.c_int64),
                ("nnz_m", ctypes.c_int64), ("nnz_v", ctypes.c_int64), ("nnz_u_pp", ctypes.c_int64),
                ("nnz_m_pp", ctypes.c_int64), ("nnz_v_pp", ctypes.c_int64), ("m_dim", ctypes.c_int64),
                ("m_dim_pp", ctypes.c_int64), ("chain_depth", ctypes.c_int32)]


class TbMatrixC(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("ptr", ctypes.POINTER(ctypes.c_int64)), ("idx", ctypes.POINTER(ctypes.c_int32)),
                ("val", ctypes.POINTER(ctypes.c_double))]


_lib = None

EXPORTS = [
    "game_create", "game_create_batch", "game_create_host", "game_destroy",
    "game_num_instances", "game_layout", "game_terminals", "game_hand_meta",
    "matvec_A", "matvec_AT", "matvec_A_f64", "matvec_AT_f64", "matvec_pair",
    "solver_reset", "solver_step", "saddle_gap", "saddle_gap_of", "saddle_gap_of_static",
    "solver_get_state", "solver_set_state", "solver_get_weights", "solver_set_weights",
    "get_average_strategy",
    "set_initial_strategy", "pmx_last_error", "game_tune", "game_get_tuning",
    "warm_num_rows", "warm_features", "warm_targets", "warm_apply",
    "mlp_gemm_bf16", "mlp_softmax_xent", "mlp_colsum", "mlp_adam", "mlp_gather_bf16",
    "mlp_gather_f32", "mlp_cast_bf16", "solver_set_active", "solver_set_params", "solver_set_task_rows", "solver_set_rm_quad",
    "solver_set_gap_guard", "tb_build", "tb_matrix", "matvec_A_tb", "matvec_AT_tb",
    "solver_snapshot", "solver_restore_instances",
]


def lib():
    """Load libpmx.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2112_03804_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.game_create.argtypes = [ctypes.POINTER(GameDescC), ctypes.POINTER(vp)]
    L.game_create_batch.argtypes = [ctypes.POINTER(GameDescC), ctypes.c_int32, ctypes.POINTER(vp)]
    L.game_create_host.argtypes = [ctypes.POINTER(GameDescC), ctypes.c_int32, ctypes.POINTER(vp)]
    L.game_destroy.argtypes = [vp]
    L.game_destroy.restype = None
    L.game_num_instances.argtypes = [vp, _c_i32p]
    L.game_layout.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(LayoutC)]
    L.game_terminals.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(TerminalsC)]
    L.game_hand_meta.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(HandMetaC)]
    for name in ("matvec_A", "matvec_AT", "matvec_A_f64", "matvec_AT_f64"):
        getattr(L, name).argtypes = [vp, vp, vp, vp]
    L.matvec_pair.argtypes = [vp, vp, vp, vp, vp, vp]
    L.solver_reset.argtypes = [vp, vp]
    L.solver_step.argtypes = [vp, ctypes.c_int32, vp]
    L.solver_set_active.argtypes = [vp, _c_i32p, vp]
    L.solver_set_params.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32]
    L.saddle_gap.argtypes = [vp, _c_f64p, _c_f64p, _c_f64p, vp]
    L.saddle_gap_of.argtypes = [vp, vp, vp, _c_f64p, _c_f64p, _c_f64p, vp]
    L.saddle_gap_of_static.argtypes = [vp, vp, vp, _c_f64p, _c_f64p, _c_f64p, vp]
    L.solver_get_state.argtypes = [vp, ctypes.c_int32, _c_f32p, _c_f32p, _c_f64p, _c_i32p, _c_f64p]
    L.solver_set_state.argtypes = [vp, ctypes.c_int32, _c_f32p, _c_f32p, _c_f64p, ctypes.c_int32,
                                   ctypes.c_double]
    L.solver_get_weights.argtypes = [vp, _c_f64p]
    L.solver_set_weights.argtypes = [vp, _c_f64p]
    L.get_average_strategy.argtypes = [vp, ctypes.c_int32, _c_f64p]
    L.set_initial_strategy.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_float, vp]
    L.game_tune.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.game_get_tuning.argtypes = [vp, _c_i32p, _c_i32p]
    L.solver_set_task_rows.argtypes = [vp, ctypes.c_int32]
    L.solver_set_rm_quad.argtypes = [vp, ctypes.c_int32]
    L.solver_set_gap_guard.argtypes = [vp, ctypes.c_int32]
    L.solver_snapshot.argtypes = [vp, vp]
    L.solver_restore_instances.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp]
    L.tb_build.argtypes = [vp, ctypes.POINTER(TbSizesC)]
    L.tb_matrix.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(TbMatrixC)]
    L.matvec_A_tb.argtypes = [vp, vp, vp, vp]
    L.matvec_AT_tb.argtypes = [vp, vp, vp, vp]
    i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.warm_num_rows.argtypes = [vp, i32, ctypes.POINTER(i64)]
    L.warm_features.argtypes = [vp, i32, vp, vp]
    L.warm_targets.argtypes = [vp, i32, vp, vp, vp]
    L.warm_apply.argtypes = [vp, vp, vp, i32, f32, ctypes.c_double, vp]
    L.mlp_gemm_bf16.argtypes = [i32, i32, i32, vp, i32, i32, vp, i32, i32, vp, i32, vp, i32, vp, i32,
                                vp, i32, vp, i64, vp]
    L.mlp_softmax_xent.argtypes = [i32, i32, vp, i32, vp, vp, vp, vp, vp, vp]
    L.mlp_colsum.argtypes = [i32, i32, vp, vp, vp, i64, vp]
    L.mlp_adam.argtypes = [i64, vp, vp, vp, vp, vp, f32, f32, f32, f32, f32, i32, vp]
    L.mlp_gather_bf16.argtypes = [i64, i32, vp, vp, vp, vp]
    L.mlp_gather_f32.argtypes = [i64, i32, vp, vp, vp, vp]
    L.mlp_cast_bf16.argtypes = [i64, vp, vp, vp]
    L.pmx_last_error.argtypes = []
    L.pmx_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


class PmxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pmx error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != PMX_OK:
        raise PmxError(rc, lib().pmx_last_error().decode())


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def check(rc):
    """Raise PmxError for a nonzero return code of a libpmx call."""
    _check(rc)


def dptr(t):
    """Device pointer of a torch tensor (NULL for None)."""
    return _dptr(t)


def stream_ptr(stream=None):
    return _stream(stream)


class _DescPack:
    """Keeps the numpy arrays behind a GameDescC alive."""

    def __init__(self, d: GameDesc):
        self.board = np.ascontiguousarray(d.board, dtype=np.uint8)
        self.rivers = np.ascontiguousarray(d.river_cards, dtype=np.uint8)
        self.cards = [np.ascontiguousarray(h, dtype=np.uint8) for h in d.hands]
        self.strength = [np.ascontiguousarray(s, dtype=np.int32) for s in d.strength]
        self.range = [np.ascontiguousarray(r, dtype=np.float64) for r in d.range_]
        self.fracs = np.ascontiguousarray(d.bet_fracs, dtype=np.float64)
        c = GameDescC()
        c.deck_size = d.deck_size
        c.cards_per_hand = d.cards_per_hand
        c.n_board = len(self.board)
        c.board = _ptr(self.board, ctypes.c_uint8)
        c.n_river = len(self.rivers)
        c.river_cards = _ptr(self.rivers, ctypes.c_uint8)
        for p in range(2):
            c.n_hands[p] = len(self.cards[p])
            c.hand_cards[p] = _ptr(self.cards[p], ctypes.c_uint8)
            c.strength[p] = _ptr(self.strength[p], ctypes.c_int32)
            c.range[p] = _ptr(self.range[p], ctypes.c_double)
        c.contrib = float(d.contrib)
        c.stack[0], c.stack[1] = float(d.stack[0]), float(d.stack[1])
        c.n_bet_fracs = len(self.fracs)
        c.bet_fracs = _ptr(self.fracs, ctypes.c_double)
        c.max_raises = int(d.max_raises)
        c.allow_allin = 1 if d.allow_allin else 0
        menu = getattr(d, "bet_menu", None)
        if menu is not None:
            if len(menu) != 2 or any(len(m) != 5 for m in menu):
                raise ValueError("bet_menu needs five lists of fractions per player")
            self.menu_len = np.array([len(menu[p][k]) for p in range(2) for k in range(5)], dtype=np.int32)
            self.menu = np.array([float(f) for p in range(2) for k in range(5) for f in menu[p][k]] or [0.0],
                                 dtype=np.float64)
            c.bet_menu_len = _ptr(self.menu_len, ctypes.c_int32)
            c.bet_menu = _ptr(self.menu, ctypes.c_double)
        self.c = c


class Game:
    """A game (one instance or a batch) owned by libpmx.

    ``device=False`` builds host-side structures only (usable without a GPU).
    """

    def __init__(self, descs: Union[GameDesc, Sequence[GameDesc]], device: bool = True):
        L = lib()
        if isinstance(descs, GameDesc):
            descs = [descs]
        self.descs = list(descs)
        packs = [_DescPack(d) for d in self.descs]
        arr = (GameDescC * len(packs))(*[p.c for p in packs])
        h = ctypes.c_void_p()
        if device:
            _check(L.game_create_batch(arr, len(packs), ctypes.byref(h)))
        else:
            _check(L.game_create_host(arr, len(packs), ctypes.byref(h)))
        self._h = h
        self.device = device
        self.n_instances = len(self.descs)
        self.layouts = [[self.layout(i, p) for p in range(2)] for i in range(self.n_instances)]
        self.elems = [self.layouts[0][p]["vec_elems"] for p in range(2)]

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().game_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- host-side queries --------------------------------------------------
    def layout(self, inst: int, player: int) -> dict:
        L = LayoutC()
        _check(lib().game_layout(self._h, inst, player, ctypes.byref(L)))
        n = L.n_infosets
        arr = lambda p: np.ctypeslib.as_array(p, shape=(n,)).copy() if n else np.zeros(0, np.int32)
        return dict(n_seq=L.n_seq, n_hands=L.n_hands, stride=L.stride, vec_offset=L.vec_offset,
                    n_infosets=n,
                    vec_elems=L.vec_elems, infoset_parent=arr(L.infoset_parent),
                    infoset_first=arr(L.infoset_first), infoset_nact=arr(L.infoset_nact),
                    infoset_board=arr(L.infoset_board))

    def terminals(self, inst: int) -> dict:
        T = TerminalsC()
        _check(lib().game_terminals(self._h, inst, ctypes.byref(T)))
        n = T.n_terminals
        g = lambda p: np.ctypeslib.as_array(p, shape=(n,)).copy()
        return dict(seq1=g(T.seq1), seq2=g(T.seq2), kind=g(T.kind), board=g(T.board),
                    runout=g(T.runout), c1=g(T.c1), c2=g(T.c2))

    def hand_meta(self, inst: int, ctx: int, player: int) -> dict:
        H = HandMetaC()
        _check(lib().game_hand_meta(self._h, inst, ctx, player, ctypes.byref(H)))
        n = H.n_hands
        rank = np.ctypeslib.as_array(H.rank, shape=(n,)).copy()
        # lt / le / self_ are strided views into 8-int records
        rec = np.ctypeslib.as_array(ctypes.cast(H.lt, _c_i32p), shape=(n * 8,)).reshape(n, 8).copy()
        return dict(n_live=H.n_live, rank=rank, lt=rec[:, 0], le=rec[:, 1], self_=rec[:, 7],
                    beta=H.beta)

    def game_tune(self, kernel: int, rows_per_chunk: int):
        _check(lib().game_tune(self._h, int(kernel), int(rows_per_chunk)))

    def solver_set_gap_guard(self, k: int):
        _check(lib().solver_set_gap_guard(self._h, int(k)))

    def solver_snapshot(self, stream=None):
        _check(lib().solver_snapshot(self._h, _stream(stream)))

    def solver_restore_instances(self, restore, stream=None):
        a = np.ascontiguousarray(restore, dtype=np.int32)
        if a.shape != (self.n_instances,):
            raise ValueError("one flag per instance")
        _check(lib().solver_restore_instances(self._h, _ptr(a, ctypes.c_int32), _stream(stream)))

    def solver_set_rm_quad(self, max_records: int):
        """Regret launches of at most max_records block records use the
        four-lanes-per-hand kernel (0: never)."""
        _check(lib().solver_set_rm_quad(self._h, int(max_records)))

    def solver_set_task_rows(self, rows: int):
        """Cut each treeplex into regret-update pieces of at most `rows` sequences."""
        _check(lib().solver_set_task_rows(self._h, int(rows)))

    def game_get_tuning(self):
        k, r = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().game_get_tuning(self._h, ctypes.byref(k), ctypes.byref(r)))
        return k.value, r.value

    # -- vector packing (host numpy <-> flat padded layout) ------------------
    def pack(self, player: int, per_instance: List[np.ndarray], dtype=np.float32) -> np.ndarray:
        out = np.zeros(self.elems[player], dtype=dtype)
        for i, v in enumerate(per_instance):
            L = self.layouts[i][player]
            blk = out[L["vec_offset"]:L["vec_offset"] + L["n_seq"] * L["stride"]].reshape(
                L["n_seq"], L["stride"])
            blk[:, :L["n_hands"]] = v
        return out

    def unpack(self, player: int, flat: np.ndarray) -> List[np.ndarray]:
        res = []
        for i in range(self.n_instances):
            L = self.layouts[i][player]
            blk = np.asarray(flat[L["vec_offset"]:L["vec_offset"] + L["n_seq"] * L["stride"]]).reshape(
                L["n_seq"], L["stride"])
            res.append(blk[:, :L["n_hands"]].copy())
        return res

    # -- device calls (torch tensors) ----------------------------------------
    def matvec_A(self, y, out, stream=None):
        _check(lib().matvec_A(self._h, _dptr(y), _dptr(out), _stream(stream)))

    def matvec_AT(self, x, out, stream=None):
        _check(lib().matvec_AT(self._h, _dptr(x), _dptr(out), _stream(stream)))

    def matvec_A_f64(self, y, out, stream=None):
        _check(lib().matvec_A_f64(self._h, _dptr(y), _dptr(out), _stream(stream)))

    def matvec_AT_f64(self, x, out, stream=None):
        _check(lib().matvec_AT_f64(self._h, _dptr(x), _dptr(out), _stream(stream)))

    def tb_build(self) -> dict:
        """Technique B's explicit factors (host sizes; device CSR forms for a
        device game).  Returns the sizes as a dict."""
        z = TbSizesC()
        _check(lib().tb_build(self._h, ctypes.byref(z)))
        return {f: getattr(z, f) for f, _ in TbSizesC._fields_}

    def tb_matrix(self, which: int):
        """One explicit factor as (indptr, indices, values, shape) host copies."""
        m = TbMatrixC()
        _check(lib().tb_matrix(self._h, int(which), ctypes.byref(m)))
        ptr = np.ctypeslib.as_array(m.ptr, shape=(m.rows + 1,)).copy()
        idx = np.ctypeslib.as_array(m.idx, shape=(m.nnz,)).copy() if m.nnz else np.zeros(0, np.int32)
        val = np.ctypeslib.as_array(m.val, shape=(m.nnz,)).copy() if m.nnz else np.zeros(0)
        return ptr, idx, val, (int(m.rows), int(m.cols))

    def matvec_A_tb(self, y, out, stream=None):
        _check(lib().matvec_A_tb(self._h, _dptr(y), _dptr(out), _stream(stream)))

    def matvec_AT_tb(self, x, out, stream=None):
        _check(lib().matvec_AT_tb(self._h, _dptr(x), _dptr(out), _stream(stream)))

    def matvec_pair(self, y, x, Ay, ATx, stream=None):
        _check(lib().matvec_pair(self._h, _dptr(y), _dptr(x), _dptr(Ay), _dptr(ATx), _stream(stream)))

    def solver_reset(self, stream=None):
        _check(lib().solver_reset(self._h, _stream(stream)))

    def solver_step(self, n_iters: int, stream=None):
        _check(lib().solver_step(self._h, int(n_iters), _stream(stream)))

    def solver_set_params(self, kind: str = "rm+", alpha: float = 1.5, beta: float = 0.0, gamma: int = 2):
        k = {"rm+": 0, "dcfr": 1}[kind]
        _check(lib().solver_set_params(self._h, k, float(alpha), float(beta), int(gamma)))

    def solver_set_active(self, active, stream=None):
        a = np.ascontiguousarray(active, dtype=np.int32)
        if a.shape != (self.n_instances,):
            raise ValueError("one flag per instance")
        _check(lib().solver_set_active(self._h, _ptr(a, ctypes.c_int32), _stream(stream)))

    def saddle_gap(self, stream=None):
        n = self.n_instances
        gap, b1, b2 = (np.zeros(n) for _ in range(3))
        _check(lib().saddle_gap(self._h, _ptr(gap, ctypes.c_double), _ptr(b1, ctypes.c_double),
                                _ptr(b2, ctypes.c_double), _stream(stream)))
        return gap, b1, b2

    def saddle_gap_of(self, x, y, stream=None):
        n = self.n_instances
        gap, b1, b2 = (np.zeros(n) for _ in range(3))
        _check(lib().saddle_gap_of(self._h, _dptr(x), _dptr(y), _ptr(gap, ctypes.c_double),
                                   _ptr(b1, ctypes.c_double), _ptr(b2, ctypes.c_double),
                                   _stream(stream)))
        return gap, b1, b2

    def saddle_gap_of_static(self, x, y, stream=None):
        n = self.n_instances
        gap, b1, b2 = (np.zeros(n) for _ in range(3))
        _check(lib().saddle_gap_of_static(self._h, _dptr(x), _dptr(y), _ptr(gap, ctypes.c_double),
                                          _ptr(b1, ctypes.c_double), _ptr(b2, ctypes.c_double),
                                          _stream(stream)))
        return gap, b1, b2

    def solver_get_state(self, player: int):
        n = self.elems[player]
        R = np.zeros(n, np.float32)
        x = np.zeros(n, np.float32)
        s = np.zeros(n, np.float64)
        t = ctypes.c_int32()
        w = ctypes.c_double()
        _check(lib().solver_get_state(self._h, player, _ptr(R, ctypes.c_float), _ptr(x, ctypes.c_float),
                                      _ptr(s, ctypes.c_double), ctypes.byref(t), ctypes.byref(w)))
        return dict(regret=R, plan=x, avg_sum=s, t=t.value, wsum=w.value)

    def solver_set_state(self, player: int, regret=None, plan=None, avg_sum=None, t=0, wsum=0.0):
        r = None if regret is None else np.ascontiguousarray(regret, np.float32)
        x = None if plan is None else np.ascontiguousarray(plan, np.float32)
        s = None if avg_sum is None else np.ascontiguousarray(avg_sum, np.float64)
        _check(lib().solver_set_state(self._h, player, _ptr(r, ctypes.c_float), _ptr(x, ctypes.c_float),
                                      _ptr(s, ctypes.c_double), int(t), float(wsum)))

    def solver_get_weights(self) -> np.ndarray:
        w = np.zeros(self.n_instances, np.float64)
        _check(lib().solver_get_weights(self._h, _ptr(w, ctypes.c_double)))
        return w

    def solver_set_weights(self, wsum):
        w = np.ascontiguousarray(wsum, np.float64)
        if w.shape != (self.n_instances,):
            raise ValueError(f"need {self.n_instances} weight totals, got shape {w.shape}")
        _check(lib().solver_set_weights(self._h, _ptr(w, ctypes.c_double)))

    def get_average_strategy(self, player: int) -> np.ndarray:
        out = np.zeros(self.elems[player], np.float64)
        _check(lib().get_average_strategy(self._h, player, _ptr(out, ctypes.c_double)))
        return out

    def warm_num_rows(self, player: int) -> int:
        n = ctypes.c_int64()
        _check(lib().warm_num_rows(self._h, player, ctypes.byref(n)))
        return n.value

    def warm_features(self, player: int, x_bf16, stream=None):
        _check(lib().warm_features(self._h, player, _dptr(x_bf16), _stream(stream)))

    def warm_targets(self, player: int, target, weight, stream=None):
        _check(lib().warm_targets(self._h, player, _dptr(target), _dptr(weight), _stream(stream)))

    def warm_apply(self, logits0, logits1, ldz: int, regret_scale: float, avg_weight: float, stream=None):
        _check(lib().warm_apply(self._h, _dptr(logits0), _dptr(logits1), int(ldz), float(regret_scale),
                                float(avg_weight), _stream(stream)))

    def set_initial_strategy(self, player: int, behav, scale: float = 1.0, stream=None):
        _check(lib().set_initial_strategy(self._h, player, _dptr(behav), float(scale), _stream(stream)))
