"""GPU parity of the base case, through the C ABI, bit for bit against the oracle.

Segments of at most T keys go straight to the base case, so one segmented sort of many such
segments reaches each of its paths:

* digits that cover every varying bit (integers over a short range): counting alone sorts;
* digits from the top varying bits and a rank inside each digit (a narrow float range);
* buckets whose top varying bits are mostly exponent bits (a float range over several binades),
  heavy duplicates, a lognormal with a wide sigma, infinities, NaNs, ranges whose width or scale
  overflows: a few digits take most keys, and the merge sort runs.

Each kind runs at every size class of the base case, for fp64, fp32 and u64, with and without a
payload.

The samples of a level are sorted by the same kernels, where a skewed sample is first counted again
with digits from a linear map of the value.  Sorts whose samples (600, 2000 and 4000 keys: one per
large size class) span such ranges check that path through the fitted lines: the output, the
number of levels and the largest first-level bucket must equal the oracle's.
"""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
import paper_2208_06902_amd as ipls  # noqa: E402
from gpu_util import dev, host, same_bits  # noqa: E402

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 64, 65, 300, 512, 513, 1000, 1024, 1025, 2000, 2048, 2049, 3000, 4095, 4096]


def kind_keys(kind, n, r):
    if kind == "narrow":
        return 1.0 + r.random(n) * 1e-3
    if kind == "binades":
        return r.standard_normal(n)
    if kind == "binades_pos":
        return r.exponential(0.5, n)
    if kind == "lognormal_wide":
        return r.lognormal(0.0, 2.0, n)
    if kind == "ints":
        return r.integers(0, 1000, n).astype(np.float64)
    if kind == "dups":
        return r.choice(np.array([1.5, 2.5, -3.0]), n)
    if kind == "zeros":
        k = r.standard_normal(n) * 1e-3
        k[r.random(n) < 0.3] = 0.0
        k[r.random(n) < 0.3] = -0.0
        return k
    if kind == "inf":
        k = r.standard_normal(n)
        k[r.integers(0, n, max(1, n // 200))] = np.inf
        k[r.integers(0, n, max(1, n // 200))] = -np.inf
        return k
    if kind == "nan":
        k = r.standard_normal(n)
        k[r.integers(0, n, max(1, n // 200))] = np.nan
        k[r.integers(0, n, max(1, n // 300))] = -np.nan
        return k
    if kind == "tiny":
        return r.standard_normal(n) * 1e-310  # subnormal range: the value map's scale overflows
    if kind == "huge":
        return r.standard_normal(n) * 1e307  # the range's width overflows
    raise ValueError(kind)


F_KINDS = ["narrow", "binades", "binades_pos", "lognormal_wide", "ints", "dups", "zeros", "inf", "nan", "tiny", "huge"]


def u64_keys(kind, n, r):
    if kind == "wide":
        return r.integers(0, 2**64, n, dtype=np.uint64)
    if kind == "low":
        return r.integers(0, 2**20, n, dtype=np.uint64)
    if kind == "skew":  # small values and a few huge ones: skewed under both digit functions
        k = r.integers(0, 2**20, n, dtype=np.uint64)
        k[r.integers(0, n, max(1, n // 100))] = np.uint64(2**63) + r.integers(0, 2**40, dtype=np.uint64)
        return k
    if kind == "around_2_63":  # one binade of the value map, many keys per double
        return np.uint64(2**63) + r.integers(0, 2**14, n, dtype=np.uint64) * np.uint64(4096)
    raise ValueError(kind)


U_KINDS = ["wide", "low", "skew", "around_2_63"]


def batch(dtype, seed):
    r = np.random.default_rng(seed)
    parts = []
    kinds = U_KINDS if dtype == np.uint64 else F_KINDS
    for kind in kinds:
        for n in SIZES:
            if dtype == np.uint64:
                parts.append(u64_keys(kind, n, r))
            else:
                with np.errstate(over="ignore"):  # fp32: the huge kind rounds to infinities
                    parts.append(kind_keys(kind, n, r).astype(dtype))
    sizes = np.array([p.size for p in parts])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    return np.concatenate(parts), off


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.uint64])
@pytest.mark.parametrize("payload", [False, True])
def test_base_case_paths(dtype, payload):
    keys, off = batch(dtype, 5 + int(payload))
    pay = np.arange(keys.size, dtype=np.uint32) if payload else None
    print(f"base case dtype={np.dtype(dtype).name} payload={payload} segments={off.size - 1} total={keys.size}",
          flush=True)
    kd, od = dev(keys), dev(off)
    pd = None if pay is None else dev(pay)
    ipls.sort_segmented_(kd, od, pd)
    torch.cuda.synchronize()
    want, wpay, ost = oracle.sort_segmented(keys, off, pay, oracle.params())
    assert ost["max_level"] == 0  # every segment went straight to the base case
    assert same_bits(host(kd, keys.dtype), want)
    if payload:
        assert np.array_equal(host(pd, np.uint32), wpay)


SAMPLE_KINDS = ["binades", "binades_pos", "lognormal_wide", "zeros", "inf", "nan", "tiny", "huge"]


@pytest.mark.parametrize("n", [60_000, 200_000, 400_000])
@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.uint64])
def test_sample_sorts_of_skewed_ranges(n, dtype):
    r = np.random.default_rng(n // 1000 + 7)
    cases = U_KINDS if dtype == np.uint64 else SAMPLE_KINDS
    for kind in cases:
        if dtype == np.uint64:
            keys = u64_keys(kind, n, r)
        else:
            with np.errstate(over="ignore"):
                keys = kind_keys(kind, n, r).astype(dtype)
        print(f"sample sort kind={kind} n={n} dtype={np.dtype(dtype).name}", flush=True)
        kd = dev(keys)
        st = ipls.sort_(kd, None, stats=True)
        torch.cuda.synchronize()
        want, _, ost = oracle.sort(keys, None, oracle.params())
        assert same_bits(host(kd, keys.dtype), want), kind
        assert (st["levels"], st["passes"], st["level1_max_load"]) == \
            (ost["max_level"], ost["passes"], ost["level1_max_load"]), (kind, st, ost)
