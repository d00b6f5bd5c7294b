"""CPU oracle for the MH-DEOCT fitness-evaluation path (arXiv 2311.06952).

TEST INFRASTRUCTURE ONLY.  This package is the CPU implementation that the
HIP library's results are compared against.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product package never
imports, links or calls anything here, and the two share no code.

The arithmetic lives in ``mhdeoct_oracle.c`` (plain C, ``-O2
-ffp-contract=off``; its fitness loop over individuals runs on OpenMP threads,
which changes no result).  This module only builds it and marshals numpy
arrays through ctypes.  Each wrapper names the passage of the paper that the C
function follows; the readings taken where the paper is silent are stated in
the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhdeoct_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp",
             "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class DEParams(C.Structure):
    _fields_ = [("P", C.c_uint32), ("G", C.c_uint32), ("M", C.c_double),
                ("CR", C.c_double), ("seed", C.c_uint64), ("n_min", C.c_uint32),
                ("alpha", C.c_double)]


_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = C.CDLL(_LIB)
    V = C.c_void_p
    lib.oracle_splitmix64_next.argtypes = [C.POINTER(C.c_uint64)]
    lib.oracle_splitmix64_next.restype = C.c_uint64
    lib.oracle_draw.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
    lib.oracle_draw.restype = C.c_uint64
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = C.c_int
    lib.oracle_u01.argtypes = [C.c_uint64]
    lib.oracle_u01.restype = C.c_double
    lib.oracle_uint.argtypes = [C.c_uint64, C.c_uint32]
    lib.oracle_uint.restype = C.c_uint32
    lib.oracle_rank_encode.argtypes = [_f32p, C.c_uint32, C.c_uint32, _u32p, _u32p]
    lib.oracle_decode.argtypes = [_f64p, C.c_uint32, C.c_uint32, C.c_uint32, _u32p, _u8p, _u32p]
    lib.oracle_decode.restype = None
    lib.oracle_route.argtypes = [_u32p, C.c_size_t, C.c_uint32, _u8p, _u32p, C.c_uint32]
    lib.oracle_route.restype = C.c_uint32
    lib.oracle_fitness.argtypes = [_u32p, C.c_size_t, _u8p, C.c_uint32, V, C.c_uint32,
                                   _u8p, _u32p, C.c_uint32, C.c_uint32, C.c_uint32,
                                   C.c_double, _u32p, _u32p, _u8p, _f64p]
    lib.oracle_split1.argtypes = [_u32p, C.c_size_t, _u32p, C.c_uint32, _u8p, C.c_uint32,
                                  V, C.c_uint32, C.POINTER(C.c_uint8),
                                  C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    lib.oracle_opt2.argtypes = [_u32p, C.c_size_t, _u32p, C.c_uint32, _u8p, C.c_uint32,
                                V, C.c_uint32, C.POINTER(C.c_uint32), _u8p, _u32p]
    lib.oracle_greedy_tree.argtypes = [_u32p, C.c_size_t, _u32p, C.c_uint32, _u8p,
                                       C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                       _u8p, _u32p]
    lib.oracle_de_init.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                   C.c_uint64, V, C.c_uint32, _f64p]
    lib.oracle_de_init.restype = None
    lib.oracle_argmin.argtypes = [_f64p, C.c_uint32]
    lib.oracle_argmin.restype = C.c_uint32
    lib.oracle_de_pick.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64,
                                   C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32),
                                   C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    lib.oracle_de_pick.restype = None
    lib.oracle_de_trial.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_double,
                                    C.c_double, C.c_uint64, C.c_uint64, C.c_uint32,
                                    _f64p, C.c_uint32, _f64p]
    lib.oracle_de_trial.restype = None
    lib.oracle_de_select.argtypes = [C.c_uint32, C.c_uint32, _f64p, _f64p, _f64p, _f64p]
    lib.oracle_de_select.restype = None
    lib.oracle_deoct.argtypes = [_u32p, C.c_size_t, _u32p, C.c_uint32, _u8p, C.c_uint32,
                                 V, C.c_uint32, C.c_uint32, C.POINTER(DEParams), V,
                                 C.c_uint32, C.c_uint64, _f64p, _u8p, _u32p, _u8p,
                                 C.POINTER(C.c_uint32), C.POINTER(C.c_double), V, V]
    lib.oracle_tree_thresholds.argtypes = [_f32p, C.c_uint32, C.c_uint32, _u8p, _u32p,
                                           C.c_uint32, _f64p]
    lib.oracle_predict.argtypes = [_f32p, C.c_uint32, C.c_uint32, _u8p, _f64p, _u8p,
                                   C.c_uint32, V, V]
    lib.oracle_predict.restype = C.c_uint32
    lib.oracle_tree_encode.argtypes = [_u8p, _u32p, C.c_uint32, C.c_uint32, C.c_uint32, _u32p,
                                       _f64p]
    lib.oracle_tree_encode.restype = None
    lib.oracle_mh_train.argtypes = [_u32p, C.c_size_t, _u32p, C.c_uint32, _u8p,
                                    C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                    C.POINTER(DEParams), C.c_uint32, _u8p, _u32p, _u8p,
                                    C.POINTER(C.c_uint32), C.POINTER(C.c_double)]
    lib.oracle_subtree.argtypes = [_u8p, _u32p, C.c_uint32, C.c_uint32, C.c_uint32, _u8p,
                                   _u32p]
    lib.oracle_cart.argtypes = [_u32p, C.c_size_t, _u32p, C.c_uint32, _u8p, C.c_uint32, V,
                                C.c_uint32, C.c_uint32, _u8p, _u32p]
    for name in ("oracle_rank_encode", "oracle_fitness", "oracle_split1", "oracle_opt2",
                 "oracle_greedy_tree", "oracle_deoct", "oracle_mh_train", "oracle_cart",
                 "oracle_subtree"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"{what} failed with status {rc}")


def _idx_arg(idx):
    if idx is None:
        return None, None
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    return idx, idx.ctypes.data_as(C.c_void_p)


class Dataset:
    """A rank-encoded training set held on the host (Section 2 notation):
    ``ranks`` column-major ``[F][n]`` uint32, ``n_unique`` ``[F]``,
    ``labels`` ``[n]`` uint8 in ``[0, K)``."""

    def __init__(self, ranks, n_unique, labels, K):
        self.ranks = np.ascontiguousarray(ranks, dtype=np.uint32)
        self.n_unique = np.ascontiguousarray(n_unique, dtype=np.uint32)
        self.labels = np.ascontiguousarray(labels, dtype=np.uint8)
        self.K = int(K)
        self.F, self.n = self.ranks.shape


# --------------------------------------------------------------------------
# random numbers (SplitMix64, Steele, Lea and Flood 2014)
# --------------------------------------------------------------------------
def splitmix64_sequence(seed: int, count: int) -> list[int]:
    lib = _load()
    st = C.c_uint64(seed)
    return [int(lib.oracle_splitmix64_next(C.byref(st))) for _ in range(count)]


def threads() -> int:
    """Threads of the oracle's parallel fitness loop (OpenMP)."""
    return int(_load().oracle_threads())


def draw(seed: int, prob: int, g: int, r: int, slot: int) -> int:
    return int(_load().oracle_draw(seed, prob, g, r, slot))


def u01(u: int) -> float:
    return float(_load().oracle_u01(u))


def uint(u: int, m: int) -> int:
    return int(_load().oracle_uint(u, m))


# --------------------------------------------------------------------------
# threshold sets, decoding, routing, fitness
# --------------------------------------------------------------------------
def rank_encode(X: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Section 3.1 threshold sets as dense ranks: X row-major [n][F] float32 ->
    (ranks [F][n] uint32, n_unique [F] uint32)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, F = X.shape
    ranks = np.zeros((F, n), dtype=np.uint32)
    nu = np.zeros(F, dtype=np.uint32)
    _check(_load().oracle_rank_encode(X, n, F, ranks, nu), "rank_encode")
    return ranks, nu


def dataset_from_X(X, y, K) -> Dataset:
    ranks, nu = rank_encode(X)
    return Dataset(ranks, nu, y, K)


def decode(genes: np.ndarray, D: int, F: int, n_unique) -> tuple[np.ndarray, np.ndarray]:
    """Eq. aenc and eq. benc: genes [P][2*SB] float64 -> (feat [P][SB] uint8,
    tau [P][SB] uint32)."""
    genes = np.ascontiguousarray(genes, dtype=np.float64)
    SB = (1 << D) - 1
    genes = genes.reshape(-1, 2 * SB)
    P = genes.shape[0]
    feat = np.zeros((P, SB), dtype=np.uint8)
    tau = np.zeros((P, SB), dtype=np.uint32)
    _load().oracle_decode(genes, P, D, F, np.ascontiguousarray(n_unique, dtype=np.uint32),
                          feat, tau)
    return feat, tau


def route(ds: Dataset, i: int, feat, tau, D: int) -> int:
    """Algorithm 1 walk for one sample; returns the 0-based leaf."""
    return int(_load().oracle_route(ds.ranks, ds.n, i,
                                    np.ascontiguousarray(feat, dtype=np.uint8),
                                    np.ascontiguousarray(tau, dtype=np.uint32), D))


def fitness(ds: Dataset, feat, tau, D: int, idx=None, n_min: int = 1, alpha: float = 0.0):
    """Eq. opt_c / eq. opt_all / Section 3.2 fitness for P trees.
    Returns (counts [P][SL][K], correct [P], label [P][SL], cost [P])."""
    feat = np.ascontiguousarray(feat, dtype=np.uint8)
    tau = np.ascontiguousarray(tau, dtype=np.uint32)
    SB = (1 << D) - 1
    SL = SB + 1
    feat = feat.reshape(-1, SB)
    tau = tau.reshape(-1, SB)
    P = feat.shape[0]
    idx, idx_p = _idx_arg(idx)
    n_sub = ds.n if idx is None else len(idx)
    counts = np.zeros((P, SL, ds.K), dtype=np.uint32)
    correct = np.zeros(P, dtype=np.uint32)
    label = np.zeros((P, SL), dtype=np.uint8)
    cost = np.zeros(P, dtype=np.float64)
    _check(_load().oracle_fitness(ds.ranks, ds.n, ds.labels, ds.K, idx_p, n_sub, feat, tau,
                                  P, D, n_min, alpha, counts, correct, label, cost),
           "fitness")
    return counts, correct, label, cost


def split1(ds: Dataset, idx=None):
    """Algorithm 2 horizon-1 branch: exact best depth-1 split under the 0-1
    loss.  Returns (feat, tau, correct)."""
    idx, idx_p = _idx_arg(idx)
    n_sub = ds.n if idx is None else len(idx)
    f, t, c = C.c_uint8(), C.c_uint32(), C.c_uint32()
    _check(_load().oracle_split1(ds.ranks, ds.n, ds.n_unique, ds.F, ds.labels, ds.K, idx_p,
                                 n_sub, C.byref(f), C.byref(t), C.byref(c)), "split1")
    return int(f.value), int(t.value), int(c.value)


def opt2(ds: Dataset, idx=None):
    """Exhaustive depth-2 optimum (test only).  Returns (correct, feat[3], tau[3])."""
    idx, idx_p = _idx_arg(idx)
    n_sub = ds.n if idx is None else len(idx)
    c = C.c_uint32()
    feat = np.zeros(3, dtype=np.uint8)
    tau = np.zeros(3, dtype=np.uint32)
    _check(_load().oracle_opt2(ds.ranks, ds.n, ds.n_unique, ds.F, ds.labels, ds.K, idx_p,
                               n_sub, C.byref(c), feat, tau), "opt2")
    return int(c.value), feat, tau


def cart(ds: Dataset, D: int, idx=None):
    """CART of depth D (Gini, reading R15) on the samples idx (all if None):
    (feat [SB], tau [SB])."""
    SB = (1 << D) - 1
    idx, idx_p = _idx_arg(idx)
    n_sub = ds.n if idx is None else len(idx)
    feat = np.zeros(SB, dtype=np.uint8)
    tau = np.zeros(SB, dtype=np.uint32)
    _check(_load().oracle_cart(ds.ranks, ds.n, ds.n_unique, ds.F, ds.labels, ds.K, idx_p, n_sub,
                               D, feat, tau), "cart")
    return feat, tau


def subtree(feat, tau, D: int, t: int, De: int):
    """The depth-De subtree rooted at heap node t (1-based) of a depth-D
    tree: (feat [2^De - 1], tau [2^De - 1])."""
    SBe = (1 << De) - 1
    sf = np.zeros(SBe, dtype=np.uint8)
    st = np.zeros(SBe, dtype=np.uint32)
    _load().oracle_subtree(np.ascontiguousarray(feat, dtype=np.uint8),
                           np.ascontiguousarray(tau, dtype=np.uint32), D, t, De, sf, st)
    return sf, st


def greedy_tree(ds: Dataset, D: int, n_min: int = 1):
    SB = (1 << D) - 1
    feat = np.zeros(SB, dtype=np.uint8)
    tau = np.zeros(SB, dtype=np.uint32)
    _check(_load().oracle_greedy_tree(ds.ranks, ds.n, ds.n_unique, ds.F, ds.labels, ds.K,
                                      ds.n, D, n_min, feat, tau), "greedy_tree")
    return feat, tau


# --------------------------------------------------------------------------
# differential evolution
# --------------------------------------------------------------------------
def de_params(P, G, M=0.5, CR=0.9, seed=0, n_min=1, alpha=0.0) -> DEParams:
    return DEParams(P, G, M, CR, seed, n_min, alpha)


def de_init(P, D, F, seed, prob, warm=None):
    SB = (1 << D) - 1
    m = 2 * SB
    pop = np.zeros((P, m), dtype=np.float64)
    W = 0
    wp = None
    if warm is not None:
        warm = np.ascontiguousarray(warm, dtype=np.float64).reshape(-1, m)
        W = warm.shape[0]
        wp = warm.ctypes.data_as(C.c_void_p)
    _load().oracle_de_init(P, D, F, seed, prob, wp, W, pop)
    return pop


def argmin(cost) -> int:
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    return int(_load().oracle_argmin(cost, len(cost)))


def de_pick(P, m, seed, prob, g, r):
    """(r1, r2, q_rand) of individual r at generation g (reading R8)."""
    a, b, c = C.c_uint32(), C.c_uint32(), C.c_uint32()
    _load().oracle_de_pick(P, m, seed, prob, g, r, C.byref(a), C.byref(b), C.byref(c))
    return int(a.value), int(b.value), int(c.value)


def de_trial(pop, D, F, M, CR, seed, prob, g, best):
    pop = np.ascontiguousarray(pop, dtype=np.float64)
    trial = np.zeros_like(pop)
    _load().oracle_de_trial(pop.shape[0], D, F, M, CR, seed, prob, g, pop, best, trial)
    return trial


def de_select(pop, cost, trial, trial_cost):
    """In place on pop and cost (eq. selection)."""
    P, m = pop.shape
    _load().oracle_de_select(P, m, pop, cost, np.ascontiguousarray(trial),
                             np.ascontiguousarray(trial_cost, dtype=np.float64))


def deoct(ds: Dataset, D: int, prm: DEParams, idx=None, warm=None, prob: int = 0,
          with_trace: bool = False, with_pop: bool = False):
    """Algorithm 4.  Returns a dict with the best genes, tree, labels, correct,
    cost, and optionally the best-cost trace and the final population."""
    SB = (1 << D) - 1
    m = 2 * SB
    idx, idx_p = _idx_arg(idx)
    n_sub = ds.n if idx is None else len(idx)
    W = 0
    wp = None
    if warm is not None:
        warm = np.ascontiguousarray(warm, dtype=np.float64).reshape(-1, m)
        W = warm.shape[0]
        wp = warm.ctypes.data_as(C.c_void_p)
    best = np.zeros(m, dtype=np.float64)
    feat = np.zeros(SB, dtype=np.uint8)
    tau = np.zeros(SB, dtype=np.uint32)
    label = np.zeros(SB + 1, dtype=np.uint8)
    correct = C.c_uint32()
    cost = C.c_double()
    trace = np.zeros(prm.G + 1, dtype=np.float64) if with_trace else None
    pop = np.zeros((prm.P, m), dtype=np.float64) if with_pop else None
    _check(_load().oracle_deoct(ds.ranks, ds.n, ds.n_unique, ds.F, ds.labels, ds.K, idx_p,
                                n_sub, D, C.byref(prm), wp, W, prob, best, feat, tau, label,
                                C.byref(correct), C.byref(cost),
                                trace.ctypes.data_as(C.c_void_p) if with_trace else None,
                                pop.ctypes.data_as(C.c_void_p) if with_pop else None),
           "deoct")
    out = dict(genes=best, feat=feat, tau=tau, label=label, correct=int(correct.value),
               cost=float(cost.value))
    if with_trace:
        out["trace"] = trace
    if with_pop:
        out["pop"] = pop
        # each final individual's objective, from the oracle's own decode and
        # fitness (eq. opt_all with the soft constraints of Section 3.2)
        f, t = decode(pop, D, ds.F, ds.n_unique)
        out["pop_cost"] = fitness(ds, f, t, D, idx=idx, n_min=prm.n_min, alpha=prm.alpha)[3]
    return out


MH_WS_CART, MH_WS_DEOCT, MH_WS_DEOCT_CART = 2, 4, 8


def mh_train(ds: Dataset, D: int, D_MH: int, prm: DEParams, flags: int = 0):
    """Algorithm 2 (sequential, node by node), with the warm starts of `flags`
    (MH_WS_CART, MH_WS_DEOCT, MH_WS_DEOCT_CART).  Returns a dict with the
    tree, leaf labels, correct and cost."""
    SB = (1 << D) - 1
    feat = np.zeros(SB, dtype=np.uint8)
    tau = np.zeros(SB, dtype=np.uint32)
    label = np.zeros(SB + 1, dtype=np.uint8)
    correct = C.c_uint32()
    cost = C.c_double()
    _check(_load().oracle_mh_train(ds.ranks, ds.n, ds.n_unique, ds.F, ds.labels, ds.K, ds.n,
                                   D, D_MH, C.byref(prm), flags, feat, tau, label,
                                   C.byref(correct), C.byref(cost)), "mh_train")
    return dict(feat=feat, tau=tau, label=label, correct=int(correct.value),
                cost=float(cost.value))


# --------------------------------------------------------------------------
# applying a trained tree to new samples (test accuracy)
# --------------------------------------------------------------------------
def tree_thresholds(X, feat, tau, D: int) -> np.ndarray:
    """Section 3.1 threshold sets in raw units for one tree trained on X
    (row-major [n][F] float32): the f64 value beta_t each split compares
    against (reading R13)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, F = X.shape
    SB = (1 << D) - 1
    thr = np.zeros(SB, dtype=np.float64)
    _check(_load().oracle_tree_thresholds(X, n, F, np.ascontiguousarray(feat, dtype=np.uint8),
                                          np.ascontiguousarray(tau, dtype=np.uint32), D, thr),
           "tree_thresholds")
    return thr


def predict(X, feat, thr, label, D: int, y=None):
    """Section 2 routing with raw thresholds: returns (pred [n] uint8, number
    of rows with pred == y, or 0 without y)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, F = X.shape
    pred = np.zeros(n, dtype=np.uint8)
    yv = None if y is None else np.ascontiguousarray(y, dtype=np.uint8)
    correct = _load().oracle_predict(X, n, F, np.ascontiguousarray(feat, dtype=np.uint8),
                                     np.ascontiguousarray(thr, dtype=np.float64),
                                     np.ascontiguousarray(label, dtype=np.uint8), D,
                                     None if yv is None else yv.ctypes.data_as(C.c_void_p),
                                     pred.ctypes.data_as(C.c_void_p))
    return pred, int(correct)


def tree_encode(feat, tau, D: int, F: int, n_unique) -> np.ndarray:
    """The inverse of eq. aenc / eq. benc (reading R14): trees (feat, tau)
    [P][SB] -> genes [P][2*SB] float64 that decode back to them."""
    SB = (1 << D) - 1
    feat = np.ascontiguousarray(feat, dtype=np.uint8).reshape(-1, SB)
    tau = np.ascontiguousarray(tau, dtype=np.uint32).reshape(-1, SB)
    P = feat.shape[0]
    genes = np.zeros((P, 2 * SB), dtype=np.float64)
    _load().oracle_tree_encode(feat, tau, P, D, F, np.ascontiguousarray(n_unique, dtype=np.uint32),
                               genes)
    return genes
