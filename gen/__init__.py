"""Seeded synthetic inputs for the sort, shared by the oracle tests, the GPU tests and the bench.

This module only draws numbers: it holds none of the sort's arithmetic (no key map, no sample,
no model, no classification).  Every generator is a pure function of (n, seed) so the CPU oracle
and the GPU path can be fed byte-identical inputs.

The distributions follow the synthetic suite of the Experimental Evaluation chapter (Uniform,
Normal, Log-Normal, Mix Gauss, Exponential, Chi-Squared, Root Dups, Two Dups, Zipf), with the
shapes of the workloads this library is measured on:

* ``uniform01``     i.i.d. U[0, 1) fp64
* ``normal``        N(0, 1) fp64
* ``lognormal``     LogNormal(mu=0, sigma) fp64, sigma = 0.5 by default (2.0 for the skewed stream)
* ``exponential``   Exp(lambda=2) fp64
* ``mixgauss``      equal-weight mixture of ``m`` N(mu_i, 1), mu_i ~ U[-100, 100] drawn from the seed
* ``uniform_int``   integers uniform in [0, 1e6) cast to fp64 (about 100 copies of each value at 1e8)
* ``u64_uniform``   uint64 uniform over [0, 2^64)
* ``zipf_u64``      uint64 ranks of a Zipf(s) law truncated to {1 .. 2^32} (rejection of larger draws)
* ``chi_squared``   chi^2(k=4) fp64
* ``root_dups``     A[i] = i mod floor(sqrt(n)) as fp64
* ``two_dups``      A[i] = (i^2 + n/2) mod n as fp64
"""
from __future__ import annotations

import math

import numpy as np

F64, F32, U64 = 0, 1, 2
NP_DTYPE = {F64: np.float64, F32: np.float32, U64: np.uint64}
DTYPE_CODE = {np.dtype(np.float64): F64, np.dtype(np.float32): F32, np.dtype(np.uint64): U64}

FP64_DISTS = ("normal", "lognormal", "exponential", "mixgauss", "uniform_int")
CONFIG1_DISTS = ("uniform01",) + FP64_DISTS


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(int(seed)))


def uniform01(n: int, seed: int) -> np.ndarray:
    return _rng(seed).random(n, dtype=np.float64)


def normal(n: int, seed: int) -> np.ndarray:
    return _rng(seed).standard_normal(n, dtype=np.float64)


def lognormal(n: int, seed: int, sigma: float = 0.5) -> np.ndarray:
    return _rng(seed).lognormal(0.0, sigma, n)


def exponential(n: int, seed: int, lam: float = 2.0) -> np.ndarray:
    return _rng(seed).exponential(1.0 / lam, n)


def mixgauss(n: int, seed: int, m: int = 5) -> np.ndarray:
    r = _rng(seed)
    means = r.uniform(-100.0, 100.0, m)
    comp = r.integers(0, m, n)
    out = r.standard_normal(n, dtype=np.float64)
    out += means[comp]
    return out


def uniform_int(n: int, seed: int, hi: int = 1_000_000) -> np.ndarray:
    return _rng(seed).integers(0, hi, n).astype(np.float64)


def chi_squared(n: int, seed: int, k: int = 4) -> np.ndarray:
    return _rng(seed).chisquare(k, n)


def root_dups(n: int, seed: int = 0) -> np.ndarray:
    m = max(1, math.isqrt(n))
    return (np.arange(n, dtype=np.uint64) % np.uint64(m)).astype(np.float64)


def two_dups(n: int, seed: int = 0) -> np.ndarray:
    i = np.arange(n, dtype=np.uint64)
    return ((i * i + np.uint64(n // 2)) % np.uint64(max(n, 1))).astype(np.float64)


def u64_uniform(n: int, seed: int) -> np.ndarray:
    return _rng(seed).integers(0, 2**64, n, dtype=np.uint64, endpoint=False)


def zipf_u64(n: int, seed: int, s: float = 1.1, vmax: int = 2**32) -> np.ndarray:
    """Zipf(s) ranks restricted to {1..vmax}: draws above vmax are rejected and drawn again."""
    r = _rng(seed)
    out = r.zipf(s, n)
    bad = np.nonzero(out > vmax)[0]
    while bad.size:
        out[bad] = r.zipf(s, bad.size)
        bad = bad[out[bad] > vmax]
    return out.astype(np.uint64)


GENERATORS = {
    "uniform01": uniform01,
    "normal": normal,
    "lognormal": lognormal,
    "exponential": exponential,
    "mixgauss": mixgauss,
    "uniform_int": uniform_int,
    "chi_squared": chi_squared,
    "root_dups": root_dups,
    "two_dups": two_dups,
    "u64_uniform": u64_uniform,
    "zipf_u64": zipf_u64,
    "lognormal2": lambda n, seed: lognormal(n, seed, sigma=2.0),
    "mixgauss20": lambda n, seed: mixgauss(n, seed, m=20),
}


def make(dist: str, n: int, seed: int) -> np.ndarray:
    return GENERATORS[dist](int(n), int(seed))


def as_dtype(x: np.ndarray, dtype: int) -> np.ndarray:
    """Request dtypes of the served stream: u64 = floor(|x| * 2^32), f32 = x rounded to nearest."""
    if dtype == F64:
        return np.ascontiguousarray(x, dtype=np.float64)
    if dtype == F32:
        return np.ascontiguousarray(x, dtype=np.float32)
    if x.dtype == np.uint64:
        return x
    return np.floor(np.abs(x) * 4294967296.0).astype(np.uint64)


def index_payload(n: int) -> np.ndarray:
    """uint32 payload equal to each key's original index."""
    return np.arange(n, dtype=np.uint32)


def special_f64() -> np.ndarray:
    """Edge values of IEEE binary64 (no NaN): signed zeros, infinities, subnormals, extremes."""
    f = np.finfo(np.float64)
    v = [0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, f.tiny, -f.tiny, 5e-324, -5e-324, f.max, -f.max,
         2.0**53, 2.0**53 + 2.0, -(2.0**53), 0.1, -0.1, 1e300, -1e300, 1e-300, -1e-300]
    return np.array(v, dtype=np.float64)


def segment_sizes_lognormal(nseg: int, seed: int, median: int = 4096, sigma: float = 1.39,
                            lo: int = 64, hi: int = 10_000_000) -> np.ndarray:
    """Sizes of the batched workload: clip(round(median * exp(sigma z)), lo, hi), z ~ N(0, 1)."""
    z = _rng(seed).standard_normal(nseg)
    return np.clip(np.rint(median * np.exp(sigma * z)), lo, hi).astype(np.int64)
