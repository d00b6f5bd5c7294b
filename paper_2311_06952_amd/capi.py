"""Thin ctypes binding of the C ABI in include/mhdeoct.h.

Only argument marshalling happens here: torch provides device memory and the
HIP stream, every computation runs in the HIP library.  There is no CPU
fallback: loading fails loudly if libmhdeoct.so is missing or does not export
the declared symbols.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmhdeoct.so")

MH_OK, MH_EINVAL, MH_ENOMEM, MH_EDEVICE, MH_EBUSY, MH_ECANCELED = 0, -1, -2, -3, -4, -5
MH_MAX_DEPTH = 10
MH_SEQUENTIAL, MH_BATCHED = 0, 1
MH_WS_CART, MH_WS_DEOCT, MH_WS_DEOCT_CART = 2, 4, 8

# Every entry point the header declares (checked by the CPU test suite).
EXPORTS = ("mh_version", "mh_ctx_create", "mh_ctx_destroy", "mh_last_error", "mh_ctx_profile",
           "mh_ctx_stats", "mh_rank_encode", "tree_decode", "fitness_eval", "mh_tileset_bytes",
           "mh_tileset_build", "fitness_eval_tiles", "de_init", "de_step", "subtree_solve",
           "mh_train", "split1", "mh_server_create", "mh_server_destroy", "mh_server_submit",
           "mh_server_footprint", "mh_server_pump", "mh_server_poll", "mh_autotune",
           "mh_tree_thresholds", "mh_predict", "tree_encode", "subtree_solve_pop",
           "mh_server_set_limits", "mh_server_cancel", "fitness_eval_static", "cart_tree")


class MhError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mhdeoct error {code}: {msg}")
        self.code = code


class DatasetC(C.Structure):
    _fields_ = [("n", C.c_uint32), ("F", C.c_uint32), ("K", C.c_uint32), ("ld", C.c_uint32),
                ("ranks", C.c_void_p), ("labels", C.c_void_p), ("n_unique", C.c_void_p),
                ("status", C.c_void_p)]


class DEParamsC(C.Structure):
    _fields_ = [("P", C.c_uint32), ("G", C.c_uint32), ("M", C.c_double), ("CR", C.c_double),
                ("seed", C.c_uint64), ("n_min", C.c_uint32), ("alpha", C.c_double)]


class TreeC(C.Structure):
    _fields_ = [("D", C.c_uint32), ("feat", C.c_uint8 * 1023), ("tau", C.c_uint32 * 1023),
                ("label", C.c_uint8 * 1024), ("correct", C.c_uint32), ("cost", C.c_double)]


class TuneC(C.Structure):
    _fields_ = [("persist", C.c_uint32), ("halves", C.c_uint32),
                ("persist_blocks_per_cu", C.c_uint32), ("fit_blocks_per_cu", C.c_uint32),
                ("ms_per_generation", C.c_double), ("n_candidates", C.c_uint32),
                ("ms", C.c_double * 16)]


class ResultC(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("status", C.c_int32), ("n", C.c_uint32),
                ("F", C.c_uint32), ("K", C.c_uint32), ("tree", TreeC),
                ("t_submit_ns", C.c_uint64), ("t_admit_ns", C.c_uint64),
                ("t_done_ns", C.c_uint64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmhdeoct.so and declare the signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} (run __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname; it must be the
    # one loaded, so that the library and torch share one runtime
    import torch  # noqa: F401
    lib = C.CDLL(path)
    V, U32, U64, I32, D = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_double
    sig = {
        "mh_version": ([], C.c_char_p),
        "mh_ctx_create": ([C.c_int, V, C.POINTER(V)], I32),
        "mh_ctx_destroy": ([V], None),
        "mh_last_error": ([V], C.c_char_p),
        "mh_ctx_profile": ([V, C.c_int], I32),
        "mh_ctx_stats": ([V, C.POINTER(U64), C.POINTER(D), C.POINTER(U64), C.POINTER(U64), C.c_int],
                         I32),
        "mh_rank_encode": ([V, V, U32, U32, U32, V, V, V], I32),
        "tree_decode": ([V, V, U32, U32, U32, V, V, V], I32),
        "fitness_eval": ([V, C.POINTER(DatasetC), V, U32, V, V, U32, U32, U32, D, V, V, V, V], I32),
        "fitness_eval_static": ([V, C.POINTER(DatasetC), V, U32, V, V, U32, U32, U32, D, V, V, V,
                                 V], I32),
        "mh_tileset_bytes": ([U32, U32, U32, C.POINTER(C.c_size_t)], I32),
        "mh_tileset_build": ([V, C.POINTER(DatasetC), V, U32, V, C.c_size_t], I32),
        "fitness_eval_tiles": ([V, V, V, V, V, U32, U32, U32, D, V, V, V, V], I32),
        "de_init": ([V, U32, U32, U32, U64, U64, V, U32, V], I32),
        "de_step": ([V, C.POINTER(DEParamsC), U32, U32, U64, U32, V, V, V, V, V, V], I32),
        "subtree_solve": ([V, C.POINTER(DatasetC), V, U32, U32, C.POINTER(DEParamsC), V, U32, U64,
                           C.POINTER(TreeC)], I32),
        "mh_train": ([V, C.POINTER(DatasetC), U32, U32, C.POINTER(DEParamsC), U32,
                      C.POINTER(TreeC)], I32),
        "split1": ([V, C.POINTER(DatasetC), V, U32, C.POINTER(C.c_uint8), C.POINTER(U32),
                    C.POINTER(U32)], I32),
        "cart_tree": ([V, C.POINTER(DatasetC), V, U32, U32, V, V], I32),
        "mh_server_create": ([V, U64, U32, C.POINTER(V)], I32),
        "mh_server_destroy": ([V], None),
        "mh_server_submit": ([V, U64, V, V, U32, U32, U32, U32, C.POINTER(DEParamsC)], I32),
        "mh_server_footprint": ([U32, U32, U32, U32, U32, C.POINTER(U64)], I32),
        "mh_server_pump": ([V, U32, C.POINTER(U32), C.POINTER(U32)], I32),
        "mh_server_poll": ([V, C.POINTER(ResultC), U32, C.POINTER(U32)], I32),
        "mh_server_set_limits": ([V, U32, U64], I32),
        "mh_server_cancel": ([V, U64], I32),
        "mh_autotune": ([V, C.POINTER(DatasetC), U32, C.POINTER(DEParamsC), U32, C.POINTER(TuneC)],
                        I32),
        "mh_tree_thresholds": ([V, C.POINTER(DatasetC), V, V, V, U32, V], I32),
        "mh_predict": ([V, V, U32, U32, V, V, V, U32, V, V, V], I32),
        "tree_encode": ([V, V, V, U32, U32, U32, V, V], I32),
        "subtree_solve_pop": ([V, C.POINTER(DatasetC), V, U32, U32, C.POINTER(DEParamsC), V, U32,
                               U64, C.POINTER(TreeC), V, V], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)  # AttributeError if a symbol is missing
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


# Live contexts and servers.  They are closed by an exit hook, while the HIP
# runtime (and any profiler attached to it) is still fully up: left to
# garbage collection at interpreter shutdown, their destroy calls (stream
# synchronisation, device and pinned-memory frees) could run after the
# runtime has begun to tear down.
_live_servers: "weakref.WeakSet" = weakref.WeakSet()
_live_contexts: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_all() -> None:
    for srv in list(_live_servers):
        try:
            srv.close()
        except Exception:
            pass
    for ctx in list(_live_contexts):
        try:
            ctx.close()
        except Exception:
            pass
    _default.clear()


# --------------------------------------------------------------------------
# torch-backed helpers (imported lazily so that the CPU suite can inspect the
# library without initialising a GPU)
# --------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """An mh_ctx bound to a device and a HIP stream (torch's current stream
    at creation unless one is given)."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU; none is visible")
        self.lib = load_library()
        self.device = device
        with torch.cuda.device(device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        rc = self.lib.mh_ctx_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != MH_OK:
            raise MhError(rc, self.lib.mh_last_error(None).decode())
        self.h = h
        _live_contexts.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.lib.mh_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int):
        if rc != MH_OK:
            raise MhError(rc, self.lib.mh_last_error(self.h).decode())

    def profile(self, enable: bool):
        self.check(self.lib.mh_ctx_profile(self.h, 1 if enable else 0))

    def stats(self, reset: bool = False):
        la, ev, ti = C.c_uint64(), C.c_uint64(), C.c_uint64()
        ms = C.c_double()
        self.check(self.lib.mh_ctx_stats(self.h, C.byref(la), C.byref(ms), C.byref(ev),
                                         C.byref(ti), 1 if reset else 0))
        return dict(launches=la.value, ms=ms.value, evals=ev.value, tiles=ti.value)


_default: dict[int, Context] = {}


def default_context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


@dataclass
class Dataset:
    """Rank-encoded training set resident on the device."""
    ranks: object      # torch.int32 [F][ld] (uint32 bits)
    labels: object     # torch.uint8 [n]
    n_unique: object   # torch.int32 [F] (uint32 bits)
    n: int
    F: int
    K: int
    status: object = None  # torch.int32 [1] from rank_encode(..., status=...), or None

    @property
    def ld(self) -> int:
        return int(self.ranks.shape[1])

    def cstruct(self) -> DatasetC:
        return DatasetC(self.n, self.F, self.K, self.ld, self.ranks.data_ptr(),
                        self.labels.data_ptr(), self.n_unique.data_ptr(),
                        None if self.status is None else self.status.data_ptr())


def rank_encode(X, ctx: Context | None = None, pad_to: int = 256, status=None, out=None):
    """mh_rank_encode: X float32 [n][F] (torch, on the device) -> (ranks
    int32 [F][ld], n_unique int32 [F]) with ld = n rounded up to pad_to (the
    padding columns are left unwritten).  With `status` (a device int32
    tensor of one element) the call does not wait: the device writes the
    NaN / failure status there (pass it on to Dataset).  `out` = (ranks,
    n_unique) of an earlier call with the same shape are written again instead
    of allocating new tensors."""
    torch = _torch()
    ctx = ctx or default_context()
    X = X.contiguous()
    n, F = X.shape
    ld = max(pad_to, ((n + pad_to - 1) // pad_to) * pad_to)
    if out is not None:
        ranks, nu = out
        if tuple(ranks.shape) != (F, ld) or tuple(nu.shape) != (F,):
            raise ValueError("out tensors do not match the input shape")
    else:
        ranks = torch.empty((F, ld), dtype=torch.int32, device=X.device)
        nu = torch.empty(F, dtype=torch.int32, device=X.device)
    ctx.check(ctx.lib.mh_rank_encode(ctx.h, _ptr(X), n, F, ld, _ptr(ranks), _ptr(nu),
                                     _ptr(status)))
    return ranks, nu


def dataset(X, y, K: int, ctx: Context | None = None) -> Dataset:
    """Upload float32 X [n][F] and labels y [n] and rank-encode on the device."""
    torch = _torch()
    ctx = ctx or default_context()
    dev = torch.device("cuda", ctx.device)
    Xt = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    yt = torch.as_tensor(np.ascontiguousarray(y, dtype=np.uint8)).to(dev)
    ranks, nu = rank_encode(Xt, ctx)
    return Dataset(ranks, yt, nu, int(Xt.shape[0]), int(Xt.shape[1]), int(K))


def tree_decode(genes, D: int, F: int, n_unique, ctx: Context | None = None):
    torch = _torch()
    ctx = ctx or default_context()
    SB = (1 << D) - 1
    genes = genes.contiguous().view(-1, 2 * SB)
    P = genes.shape[0]
    feat = torch.zeros((P, SB), dtype=torch.uint8, device=genes.device)
    tau = torch.zeros((P, SB), dtype=torch.int32, device=genes.device)
    ctx.check(ctx.lib.tree_decode(ctx.h, _ptr(genes), P, D, F, _ptr(n_unique), _ptr(feat),
                                  _ptr(tau)))
    return feat, tau


def tree_encode(feat, tau, D: int, F: int, n_unique, ctx: Context | None = None):
    """tree_encode: trees (feat, tau) [P][SB] -> genes [P][2*SB] float64 on
    the device (the inverse of tree_decode, for warm starts)."""
    torch = _torch()
    ctx = ctx or default_context()
    dev = torch.device("cuda", ctx.device)
    SB = (1 << D) - 1
    feat = _on_device(np.asarray(feat).reshape(-1, SB) if not isinstance(feat, torch.Tensor)
                      else feat.reshape(-1, SB), torch.uint8, dev)
    tau = tau if isinstance(tau, torch.Tensor) else np.asarray(tau, dtype=np.uint32).view(np.int32)
    tau = _on_device(tau, torch.int32, dev).reshape(-1, SB)
    P = int(feat.shape[0])
    genes = torch.empty((P, 2 * SB), dtype=torch.float64, device=dev)
    ctx.check(ctx.lib.tree_encode(ctx.h, _ptr(feat), _ptr(tau), P, D, F, _ptr(n_unique),
                                  _ptr(genes)))
    return genes


def fitness_eval(ds: Dataset, feat, tau, D: int, idx=None, n_min: int = 1, alpha: float = 0.0,
                 ctx: Context | None = None, want_counts: bool = True, static: bool = False):
    """fitness_eval (fitness_eval_static with static=True: no allocation in
    the library): returns (counts [P][SL][K] int32, correct [P] int32,
    label [P][SL] uint8, cost [P] float64), all on the device."""
    torch = _torch()
    ctx = ctx or default_context()
    SB = (1 << D) - 1
    SL = SB + 1
    feat = feat.contiguous().view(-1, SB)
    tau = tau.contiguous().view(-1, SB)
    P = feat.shape[0]
    dev = feat.device
    counts = torch.zeros((P, SL, ds.K), dtype=torch.int32, device=dev) if want_counts else None
    correct = torch.zeros(P, dtype=torch.int32, device=dev)
    label = torch.zeros((P, SL), dtype=torch.uint8, device=dev)
    cost = torch.zeros(P, dtype=torch.float64, device=dev)
    n_sub = ds.n if idx is None else int(idx.numel())
    dsc = ds.cstruct()
    fn = ctx.lib.fitness_eval_static if static else ctx.lib.fitness_eval
    ctx.check(fn(ctx.h, C.byref(dsc), _ptr(idx), n_sub, _ptr(feat), _ptr(tau), P, D, n_min, alpha,
                 _ptr(counts), _ptr(correct), _ptr(label), _ptr(cost)))
    return counts, correct, label, cost


class TileSet:
    """A prebuilt tiled sample layout (device buffer owned by torch)."""

    def __init__(self, ds: Dataset, idx=None, ctx: Context | None = None):
        torch = _torch()
        self.ctx = ctx or default_context()
        self.ds = ds
        n_sub = ds.n if idx is None else int(idx.numel())
        nb = C.c_size_t()
        self.ctx.check(self.ctx.lib.mh_tileset_bytes(n_sub, ds.F, ds.K, C.byref(nb)))
        self.buf = torch.empty(nb.value + 256, dtype=torch.uint8, device=ds.labels.device)
        off = (-self.buf.data_ptr()) % 256
        self.view = self.buf[off:off + nb.value]
        self.bytes = nb.value
        dsc = ds.cstruct()
        self.ctx.check(self.ctx.lib.mh_tileset_build(self.ctx.h, C.byref(dsc), _ptr(idx), n_sub,
                                                     _ptr(self.view), nb.value))

    def fitness(self, feat, tau, D: int, n_min: int = 1, alpha: float = 0.0, out=None):
        torch = _torch()
        SB = (1 << D) - 1
        P = feat.numel() // SB
        dev = feat.device
        if out is None:
            out = (None, None, None, torch.zeros(P, dtype=torch.float64, device=dev))
        counts, correct, label, cost = out
        ctx = self.ctx
        ctx.check(ctx.lib.fitness_eval_tiles(ctx.h, _ptr(self.view), _ptr(self.ds.n_unique),
                                             _ptr(feat), _ptr(tau), P, D, n_min, alpha,
                                             _ptr(counts), _ptr(correct), _ptr(label), _ptr(cost)))
        return out


def de_params(P, G, M=0.5, CR=0.9, seed=0, n_min=1, alpha=0.0) -> DEParamsC:
    return DEParamsC(P, G, M, CR, seed, n_min, alpha)


def de_init(P, D, F, seed, prob, warm=None, ctx: Context | None = None, device=0):
    torch = _torch()
    ctx = ctx or default_context()
    SB = (1 << D) - 1
    pop = torch.zeros((P, 2 * SB), dtype=torch.float64, device=torch.device("cuda", ctx.device))
    W = 0 if warm is None else int(warm.shape[0])
    ctx.check(ctx.lib.de_init(ctx.h, P, D, F, seed, prob, _ptr(warm), W, _ptr(pop)))
    return pop


def de_step(prm: DEParamsC, D, F, prob, g, pop, cost, trial=None, trial_cost=None,
            make_trial=True, ctx: Context | None = None):
    """One DE step; returns (best int32 [1] device tensor, next_trial or None).
    pop and cost are updated in place."""
    torch = _torch()
    ctx = ctx or default_context()
    best = torch.zeros(1, dtype=torch.int32, device=pop.device)
    nxt = torch.zeros_like(pop) if make_trial else None
    ctx.check(ctx.lib.de_step(ctx.h, C.byref(prm), D, F, prob, g, _ptr(pop), _ptr(cost),
                              _ptr(trial), _ptr(trial_cost), _ptr(best), _ptr(nxt)))
    return best, nxt


def _tree_dict(t: TreeC) -> dict:
    SB = (1 << t.D) - 1
    SL = SB + 1
    return dict(D=t.D, feat=np.array(t.feat[:SB], dtype=np.uint8),
                tau=np.array(t.tau[:SB], dtype=np.uint32),
                label=np.array(t.label[:SL], dtype=np.uint8), correct=int(t.correct),
                cost=float(t.cost))


def subtree_solve(ds: Dataset, D: int, prm: DEParamsC, idx=None, warm=None, prob: int = 0,
                  ctx: Context | None = None, with_pop: bool = False) -> dict:
    """DEOCT on the device; warm is a host float64 array [W][2*SB].  With
    with_pop the result also holds the final population (`pop`, float64
    [P][2*SB]) and its costs (`pop_cost`, [P]) as numpy arrays
    (subtree_solve_pop)."""
    ctx = ctx or default_context()
    n_sub = ds.n if idx is None else int(idx.numel())
    W = 0
    wp = None
    if warm is not None:
        warm = np.ascontiguousarray(warm, dtype=np.float64).reshape(-1, 2 * ((1 << D) - 1))
        W = warm.shape[0]
        wp = warm.ctypes.data_as(C.c_void_p)
    out = TreeC()
    dsc = ds.cstruct()
    if not with_pop:
        ctx.check(ctx.lib.subtree_solve(ctx.h, C.byref(dsc), _ptr(idx), n_sub, D, C.byref(prm), wp,
                                        W, prob, C.byref(out)))
        return _tree_dict(out)
    torch = _torch()
    dev = torch.device("cuda", ctx.device)
    pop = torch.empty((prm.P, 2 * ((1 << D) - 1)), dtype=torch.float64, device=dev)
    pcost = torch.empty(prm.P, dtype=torch.float64, device=dev)
    ctx.check(ctx.lib.subtree_solve_pop(ctx.h, C.byref(dsc), _ptr(idx), n_sub, D, C.byref(prm), wp,
                                        W, prob, C.byref(out), _ptr(pop), _ptr(pcost)))
    res = _tree_dict(out)
    res["pop"] = pop.cpu().numpy()
    res["pop_cost"] = pcost.cpu().numpy()
    return res


def _on_device(a, dtype, dev):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        return a.to(device=dev, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype).contiguous()


def tree_thresholds(ds: Dataset, X, tree: dict, ctx: Context | None = None):
    """mh_tree_thresholds: the float64 thresholds [SB] (on the device) that
    apply `tree` (a dict from subtree_solve / mh_train) to new rows; X is the
    float32 [n][F] training matrix ds was encoded from."""
    torch = _torch()
    ctx = ctx or default_context()
    dev = torch.device("cuda", ctx.device)
    D = int(tree["D"])
    Xd = _on_device(X, torch.float32, dev)
    if tuple(Xd.shape) != (ds.n, ds.F):
        raise ValueError(f"X has shape {tuple(Xd.shape)}, the dataset ({ds.n}, {ds.F})")
    feat = _on_device(tree["feat"], torch.uint8, dev)
    tau = _on_device(np.asarray(tree["tau"], dtype=np.uint32).view(np.int32), torch.int32, dev)
    thr = torch.empty((1 << D) - 1, dtype=torch.float64, device=dev)
    dsc = ds.cstruct()
    ctx.check(ctx.lib.mh_tree_thresholds(ctx.h, C.byref(dsc), _ptr(Xd), _ptr(feat), _ptr(tau), D,
                                         _ptr(thr)))
    return thr


def predict(X, tree: dict, thr, y=None, ctx: Context | None = None):
    """mh_predict: (pred uint8 [n] on the device, number of rows with
    pred == y, or None without y)."""
    torch = _torch()
    ctx = ctx or default_context()
    dev = torch.device("cuda", ctx.device)
    D = int(tree["D"])
    Xd = _on_device(X, torch.float32, dev)
    n, F = int(Xd.shape[0]), int(Xd.shape[1])
    feat = _on_device(tree["feat"], torch.uint8, dev)
    label = _on_device(tree["label"], torch.uint8, dev)
    thr = _on_device(thr, torch.float64, dev)
    yd = None if y is None else _on_device(y, torch.uint8, dev)
    pred = torch.empty(n, dtype=torch.uint8, device=dev)
    correct = None if y is None else torch.empty(1, dtype=torch.int32, device=dev)
    ctx.check(ctx.lib.mh_predict(ctx.h, _ptr(Xd), n, F, _ptr(feat), _ptr(thr), _ptr(label), D,
                                 _ptr(yd), _ptr(pred), _ptr(correct)))
    return pred, None if correct is None else int(correct.item())


def autotune(ds: Dataset, D: int, prm: DEParamsC, generations: int = 20,
             ctx: Context | None = None) -> dict:
    """mh_autotune: time the launch configurations on short runs and keep the
    fastest for this shape in the context."""
    ctx = ctx or default_context()
    out = TuneC()
    dsc = ds.cstruct()
    ctx.check(ctx.lib.mh_autotune(ctx.h, C.byref(dsc), D, C.byref(prm), generations,
                                  C.byref(out)))
    return dict(persist=int(out.persist), halves=int(out.halves),
                persist_blocks_per_cu=int(out.persist_blocks_per_cu),
                fit_blocks_per_cu=int(out.fit_blocks_per_cu),
                ms_per_generation=float(out.ms_per_generation),
                ms=[float(out.ms[i]) for i in range(out.n_candidates)])


def mh_train(ds: Dataset, D: int, D_MH: int, prm: DEParamsC, batched: bool = False,
             ctx: Context | None = None, warm: int = 0) -> dict:
    """Moving-horizon DEOCT; warm: MH_WS_* bits (warm starts of the subtree
    solves)."""
    ctx = ctx or default_context()
    out = TreeC()
    dsc = ds.cstruct()
    flags = (MH_BATCHED if batched else MH_SEQUENTIAL) | int(warm)
    ctx.check(ctx.lib.mh_train(ctx.h, C.byref(dsc), D, D_MH, C.byref(prm), flags, C.byref(out)))
    return _tree_dict(out)


def cart(ds: Dataset, D: int, idx=None, ctx: Context | None = None):
    """CART (Gini) of depth D on the samples idx (device tensor, all if None):
    (feat [2^D - 1] uint8, tau [2^D - 1] uint32) numpy arrays."""
    ctx = ctx or default_context()
    n_sub = ds.n if idx is None else int(idx.numel())
    SB = (1 << D) - 1
    feat = np.zeros(SB, dtype=np.uint8)
    tau = np.zeros(SB, dtype=np.uint32)
    dsc = ds.cstruct()
    ctx.check(ctx.lib.cart_tree(ctx.h, C.byref(dsc), _ptr(idx), n_sub, D,
                                C.c_void_p(feat.ctypes.data), C.c_void_p(tau.ctypes.data)))
    return feat, tau


def split1(ds: Dataset, idx=None, ctx: Context | None = None):
    ctx = ctx or default_context()
    n_sub = ds.n if idx is None else int(idx.numel())
    f, t, c = C.c_uint8(), C.c_uint32(), C.c_uint32()
    dsc = ds.cstruct()
    ctx.check(ctx.lib.split1(ctx.h, C.byref(dsc), _ptr(idx), n_sub, C.byref(f), C.byref(t),
                             C.byref(c)))
    return int(f.value), int(t.value), int(c.value)


def server_footprint(n: int, F: int, K: int, D: int, P: int) -> int:
    """Device bytes a served request of this shape holds while resident."""
    lib = load_library()
    b = C.c_uint64()
    rc = lib.mh_server_footprint(n, F, K, D, P, C.byref(b))
    if rc != MH_OK:
        raise MhError(rc, "invalid request shape")
    return int(b.value)


class Server:
    """mh_server: continuous-batching DEOCT requests on one context.  The
    context must not be used for other calls while the server lives."""

    def __init__(self, hbm_budget: int, max_slots: int, ctx: Context | None = None):
        self.ctx = ctx or default_context()
        h = C.c_void_p()
        self.ctx.check(self.ctx.lib.mh_server_create(self.ctx.h, int(hbm_budget), int(max_slots),
                                                     C.byref(h)))
        self.h = h
        self._inputs = {}  # req_id -> (X, y): kept alive until the result is polled
        _live_servers.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.mh_server_destroy(self.h)
            self.h = None
            self._inputs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, req_id: int, X, y, K: int, D: int, prm: DEParamsC):
        """X: float32 [n][F], y: uint8 [n], both torch tensors on the device."""
        X = X.contiguous()
        y = y.contiguous()
        n, F = int(X.shape[0]), int(X.shape[1])
        self.ctx.check(self.ctx.lib.mh_server_submit(self.h, int(req_id), _ptr(X), _ptr(y), n, F,
                                                     int(K), int(D), C.byref(prm)))
        self._inputs[int(req_id)] = (X, y)

    def set_limits(self, max_queued: int = 0, timeout_ns: int = 0):
        """mh_server_set_limits: queue back-pressure (MH_EBUSY) and a time
        limit after which requests are cancelled (0: none)."""
        self.ctx.check(self.ctx.lib.mh_server_set_limits(self.h, int(max_queued), int(timeout_ns)))

    def cancel(self, req_id: int):
        """mh_server_cancel: the request's result comes back with status
        MH_ECANCELED."""
        self.ctx.check(self.ctx.lib.mh_server_cancel(self.h, int(req_id)))

    def pump(self, ticks: int = 1):
        """Runs up to `ticks` scheduling rounds; returns (resident, queued)."""
        a, q = C.c_uint32(), C.c_uint32()
        self.ctx.check(self.ctx.lib.mh_server_pump(self.h, int(ticks), C.byref(a), C.byref(q)))
        return int(a.value), int(q.value)

    def poll(self, max_results: int = 64) -> list:
        buf = (ResultC * max_results)()
        k = C.c_uint32()
        self.ctx.check(self.ctx.lib.mh_server_poll(self.h, buf, max_results, C.byref(k)))
        out = []
        for i in range(k.value):
            r = buf[i]
            self._inputs.pop(int(r.req_id), None)
            out.append(dict(req_id=int(r.req_id), status=int(r.status), n=int(r.n), F=int(r.F),
                            K=int(r.K), tree=_tree_dict(r.tree), t_submit_ns=int(r.t_submit_ns),
                            t_admit_ns=int(r.t_admit_ns), t_done_ns=int(r.t_done_ns)))
        return out

    def drain(self, max_rounds: int = 10_000_000) -> list:
        """Pumps until nothing is resident or queued; returns every result."""
        res = []
        for _ in range(max_rounds):
            a, q = self.pump(16)
            res += self.poll(256)
            if a == 0 and q == 0:
                break
        res += self.poll(256)
        return res

