"""CPU oracle of the IPLS sort: TEST INFRASTRUCTURE ONLY.

Loads ``libipls_oracle.so`` (plain sequential C, built from ``ipls_oracle.c`` with gcc and no
FMA contraction) and wraps it for numpy arrays.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module; the GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ipls_oracle.c")
LIB = os.path.join(HERE, "libipls_oracle.so")
CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-Wall"]

F64, F32, U64 = 0, 1, 2
MODEL_LINEAR, MODEL_MSD, MODEL_CLOSED, MODEL_L2PL, MODEL_TREE = 0, 1, 2, 3, 4
_DT = {np.dtype(np.float64): F64, np.dtype(np.float32): F32, np.dtype(np.uint64): U64}


class Params(C.Structure):
    _fields_ = [("num_buckets", C.c_uint32), ("base_case_max", C.c_uint32), ("sample_divisor", C.c_uint32),
                ("sample_min", C.c_uint32), ("sample_max", C.c_uint64), ("seed", C.c_uint64),
                ("model", C.c_uint32), ("leaves", C.c_uint32), ("train_iters", C.c_uint32), ("sample_policy", C.c_uint32),
                ("equality", C.c_uint32), ("inherit", C.c_uint32), ("bucket_policy", C.c_uint32)]


class Model(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("K", C.c_uint32), ("a", C.c_double), ("b", C.c_double), ("D", C.c_uint64),
                ("umin", C.c_uint64), ("shift", C.c_uint32), ("degenerate", C.c_uint32), ("S", C.c_uint64),
                ("max_load_linear", C.c_uint64), ("max_load_l2pl", C.c_uint64), ("neq", C.c_uint32),
                ("Km", C.c_uint32), ("const0", C.c_uint32), ("pad_", C.c_uint32), ("heavy", C.c_uint64 * 16),
                ("tree_strict", C.c_uint32), ("pad2_", C.c_uint32), ("split", C.c_uint64 * 255)]


class Stats(C.Structure):
    _fields_ = [("passes", C.c_uint64), ("max_level", C.c_uint64), ("closed", C.c_uint64),
                ("fallback", C.c_uint64), ("base_cases", C.c_uint64), ("l2pl_used", C.c_uint64),
                ("level1_max_load", C.c_uint64), ("keys_partitioned", C.c_uint64),
                ("inherited", C.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


DEFAULT_SEED = 0x1F5A_2208_0690_2000


def params(K=256, T=4096, divisor=100, sample_min=0, sample_max=0, seed=DEFAULT_SEED, model=0, leaves=256,
           train_iters=4, sample_policy=0, equality=0, inherit=0, bucket_policy=1) -> Params:
    return Params(K, T, divisor, sample_min, sample_max, seed, model, leaves, train_iters, sample_policy, equality,
                  inherit, bucket_policy)


def bucket_count(n: int, p: Params) -> int:
    return int(lib().oracle_bucket_count(n, C.byref(p)))


CTX_SRC = os.path.join(HERE, "cpu_context.cpp")
CTX_LIB = os.path.join(HERE, "libcpu_context.so")


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    if force or not os.path.exists(CTX_LIB) or os.path.getmtime(CTX_LIB) < os.path.getmtime(CTX_SRC):
        tmp = CTX_LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", CTX_SRC, "-o", tmp])
        os.replace(tmp, CTX_LIB)
    return LIB


def std_sorts_seconds(x: np.ndarray) -> dict:
    """Context baselines: seconds of std::sort and std::stable_sort of copies of the fp64 array x,
    each on one thread."""
    build()
    L = C.CDLL(CTX_LIB)
    out = {}
    for name in ("ctx_std_sort_f64", "ctx_std_stable_sort_f64"):
        f = getattr(L, name)
        f.restype = C.c_double
        f.argtypes = [C.c_void_p, C.c_size_t]
        a = np.array(x, dtype=np.float64, copy=True)
        out[name[4:-4]] = float(f(a.ctypes.data, a.size))
        assert np.all(a[1:] >= a[:-1])
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        u64, u32, i32, dbl = C.c_uint64, C.c_uint32, C.c_int, C.c_double
        sig = {
            "oracle_mix64": (u64, [u64]),
            "oracle_sample_size": (u64, [u64, C.POINTER(Params)]),
            "oracle_bucket_count": (u32, [u64, C.POINTER(Params)]),
            "oracle_log2": (C.c_double, [u64]),
            "oracle_sample_positions": (None, [u64, u64, u64, u64, P]),
            "oracle_sorted_sample": (None, [P, u64, i32, u64, u64, u64, P]),
            "oracle_keymap": (None, [P, C.c_size_t, i32, P, P]),
            "oracle_fmcd": (i32, [P, u64, u32, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(u64)]),
            "oracle_sort": (i32, [P, P, u64, i32, C.POINTER(Params), C.POINTER(Stats)]),
            "oracle_sort_segmented": (i32, [P, P, P, u64, i32, C.POINTER(Params), C.POINTER(Stats)]),
            "oracle_fit_bucket": (i32, [P, u64, i32, C.POINTER(Params), u64, C.POINTER(Model), P, P]),
            "oracle_partition": (i32, [P, P, u64, i32, C.POINTER(Params), C.POINTER(Model), P]),
            "oracle_classify_linear": (None, [P, u64, i32, dbl, dbl, u32, P]),
            "oracle_child_sample": (i32, [P, u64, i32, C.POINTER(Params), u32, P, C.POINTER(C.c_uint64)]),
            "oracle_classify_model": (None, [P, u64, i32, C.POINTER(Model), P, P, u32, P]),
            "oracle_stable_layout": (None, [P, u64, i32, P, u32, P]),
            "oracle_buffered_layout": (None, [P, u64, i32, P, u32, u32, P]),
            "oracle_l2pl_geometry": (None, [P, u64, u32, dbl, dbl, P, P, P, P]),
            "oracle_l2pl_grad": (None, [P, u64, u32, u32, P, P, P, P, P, P]),
            "oracle_l2pl_train": (i32, [P, u64, u32, u32, u32, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dt(keys: np.ndarray) -> int:
    return _DT[keys.dtype]


def ord_keys(keys: np.ndarray) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    out = np.empty(keys.size, np.uint64)
    lib().oracle_keymap(_p(keys), keys.size, _dt(keys), _p(out), None)
    return out


def val_keys(keys: np.ndarray) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    out = np.empty(keys.size, np.float64)
    lib().oracle_keymap(_p(keys), keys.size, _dt(keys), None, _p(out))
    return out


def mix64(z: int) -> int:
    return int(lib().oracle_mix64(z))


def sample_size(n: int, p: Params) -> int:
    return int(lib().oracle_sample_size(n, C.byref(p)))


def log2(n: int) -> float:
    return float(lib().oracle_log2(n))


def sample_positions(n: int, lo_rel: int, S: int, seed: int) -> np.ndarray:
    out = np.empty(S, np.uint64)
    lib().oracle_sample_positions(n, lo_rel, S, seed, _p(out))
    return out


def sorted_sample(keys: np.ndarray, S: int, seed: int, lo_rel: int = 0) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    out = np.empty(S, np.float64)
    lib().oracle_sorted_sample(_p(keys), keys.size, _dt(keys), lo_rel, S, seed, _p(out))
    return out


def fmcd(x: np.ndarray, K: int):
    """FMCD on a sorted fp64 sample: (a, b, D), or None when S < 3 or K < 4."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    a, b, D = C.c_double(), C.c_double(), C.c_uint64()
    rc = lib().oracle_fmcd(_p(x), x.size, K, C.byref(a), C.byref(b), C.byref(D))
    return None if rc else (a.value, b.value, int(D.value))


def sort(keys: np.ndarray, payload: np.ndarray | None = None, p: Params | None = None):
    """Sorted copies of (keys, payload) and the oracle's stats."""
    p = p or params()
    k = np.array(keys, copy=True)
    pl = None if payload is None else np.array(payload, dtype=np.uint32, copy=True)
    st = Stats()
    rc = lib().oracle_sort(_p(k), _p(pl), k.size, _dt(k), C.byref(p), C.byref(st))
    if rc:
        raise ValueError("oracle_sort rejected its arguments")
    return k, pl, st.as_dict()


def sort_segmented(keys: np.ndarray, offsets: np.ndarray, payload: np.ndarray | None = None,
                   p: Params | None = None):
    p = p or params()
    k = np.array(keys, copy=True)
    pl = None if payload is None else np.array(payload, dtype=np.uint32, copy=True)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    st = Stats()
    rc = lib().oracle_sort_segmented(_p(k), _p(pl), _p(off), off.size - 1, _dt(k), C.byref(p), C.byref(st))
    if rc:
        raise ValueError("oracle_sort_segmented rejected its arguments")
    return k, pl, st.as_dict()


def fit_bucket(keys: np.ndarray, p: Params | None = None, lo_rel: int = 0):
    """Model of the bucket `keys` (sample, sort, fit, degenerate handling): (Model, root, leaf)."""
    p = p or params()
    keys = np.ascontiguousarray(keys)
    m = Model()
    M = p.leaves or 256
    root = np.zeros(2, np.float64)
    leaf = np.zeros(4 * M, np.float64)
    rc = lib().oracle_fit_bucket(_p(keys), keys.size, _dt(keys), C.byref(p), lo_rel, C.byref(m), _p(root), _p(leaf))
    if rc:
        raise ValueError("oracle_fit_bucket rejected its arguments")
    return m, root, leaf


def child_sample(keys: np.ndarray, c: int, p: Params) -> np.ndarray:
    """The sorted sample (as ords) that bucket c of the first level inherits; empty when it draws a
    fresh one."""
    keys = np.ascontiguousarray(keys)
    out = np.zeros(max(sample_size(keys.size, p), 1), np.uint64)
    ln = C.c_uint64()
    if lib().oracle_child_sample(_p(keys), keys.size, _dt(keys), C.byref(p), c, _p(out), C.byref(ln)):
        raise ValueError("oracle_child_sample rejected its arguments")
    return out[: ln.value].copy()


def partition(keys: np.ndarray, payload: np.ndarray | None = None, p: Params | None = None):
    """One distribution pass of the whole array: (keys, payload, counts, Model)."""
    p = p or params()
    k = np.array(keys, copy=True)
    pl = None if payload is None else np.array(payload, dtype=np.uint32, copy=True)
    counts = np.zeros(p.num_buckets, np.uint64)
    m = Model()
    rc = lib().oracle_partition(_p(k), _p(pl), k.size, _dt(k), C.byref(p), C.byref(m), _p(counts))
    if rc:
        raise ValueError("oracle_partition rejected its arguments")
    return k, pl, counts, m


def classify_linear(keys: np.ndarray, a: float, b: float, K: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    out = np.empty(keys.size, np.uint32)
    lib().oracle_classify_linear(_p(keys), keys.size, _dt(keys), a, b, K, _p(out))
    return out


def classify_model(keys: np.ndarray, m: Model, root=None, leaf=None, M: int = 256) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    out = np.empty(keys.size, np.uint32)
    lib().oracle_classify_model(_p(keys), keys.size, _dt(keys), C.byref(m), _p(root), _p(leaf), M, _p(out))
    return out


def stable_layout(keys: np.ndarray, bucket: np.ndarray, K: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    b = np.ascontiguousarray(bucket, dtype=np.uint32)
    out = np.empty_like(keys)
    lib().oracle_stable_layout(_p(keys), keys.size, _dt(keys), _p(b), K, _p(out))
    return out


def buffered_layout(keys: np.ndarray, bucket: np.ndarray, K: int, bsize: int) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    b = np.ascontiguousarray(bucket, dtype=np.uint32)
    out = np.empty_like(keys)
    lib().oracle_buffered_layout(_p(keys), keys.size, _dt(keys), _p(b), K, bsize, _p(out))
    return out


def l2pl_geometry(x: np.ndarray, M: int, ra: float, rb: float):
    x = np.ascontiguousarray(x, dtype=np.float64)
    first = np.zeros(M + 1, np.uint64)
    c = np.zeros(M, np.float64)
    h = np.zeros(M, np.float64)
    m2 = np.zeros(M, np.float64)
    lib().oracle_l2pl_geometry(_p(x), x.size, M, ra, rb, _p(first), _p(c), _p(h), _p(m2))
    return first, c, h, m2


def l2pl_grad(x: np.ndarray, K: int, M: int, first, c, h, ab: np.ndarray):
    """(grad (2M), loss (M)) of every leaf's mean-squared error at (alpha, beta) = ab."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    ab = np.ascontiguousarray(ab, dtype=np.float64)
    g = np.zeros(2 * M, np.float64)
    loss = np.zeros(M, np.float64)
    lib().oracle_l2pl_grad(_p(x), x.size, K, M, _p(np.ascontiguousarray(first, np.uint64)),
                           _p(np.ascontiguousarray(c, np.float64)), _p(np.ascontiguousarray(h, np.float64)),
                           _p(ab), _p(g), _p(loss))
    return g, loss


def l2pl_train(x: np.ndarray, K: int, M: int, iters: int):
    """(root (2), leaf (4M: A, B, LO, HI), ab (2M)) or None when the root fit fails."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    root = np.zeros(2, np.float64)
    leaf = np.zeros(4 * M, np.float64)
    ab = np.zeros(2 * M, np.float64)
    rc = lib().oracle_l2pl_train(_p(x), x.size, K, M, iters, _p(root), _p(leaf), _p(ab))
    return None if rc else (root, leaf, ab)
