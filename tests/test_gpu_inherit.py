"""GPU parity of sample inheritance, through the C ABI, bit for bit against the oracle.

A child's line is fitted before the parent's scatter, which also writes each key's class under
it.  The child's counting pass then reads those bytes.  Each case is checked for:

* keys and payloads equal to the oracle's output;
* the count of inherited partitions equal to the oracle's count;
* passes and levels equal to the oracle's.

The cases cover two and three levels of inheritance, every dtype, both tile sizes, NaNs and
infinities, segmented batches, and the default parameters at a size where the 1% sample gives
children enough keys.
"""
import numpy as np
import pytest

import gen
import oracle
import paper_2208_06902_amd as ipls

torch = pytest.importorskip("torch")
from gpu_util import dev, host, same_bits  # noqa: E402

pytestmark = pytest.mark.gpu

SMALL = dict(num_buckets=16, base_case_max=4096, sample_divisor=10)  # two levels at 2*10^5 keys
DEEP = dict(num_buckets=16, base_case_max=256, sample_divisor=10)  # three or more levels


def oparams(kw):
    return oracle.params(K=kw.get("num_buckets", 256), T=kw.get("base_case_max", 4096),
                         divisor=kw.get("sample_divisor", 100), sample_min=kw.get("sample_min", 0),
                         sample_max=kw.get("sample_max", 0), inherit=1)


def check(keys, payload=None, **kw):
    print(f"inherit n={keys.size} dtype={keys.dtype} payload={payload is not None} params={kw}", flush=True)
    p = ipls.default_params(inherit=1, **kw)
    k = dev(keys)
    pl = None if payload is None else dev(payload)
    st = ipls.sort_(k, pl, params=p, stats=True)
    torch.cuda.synchronize()
    want, wpay, ost = oracle.sort(keys, payload, oparams(kw))
    assert same_bits(host(k, keys.dtype), want)
    if payload is not None:
        assert np.array_equal(host(pl, np.uint32), wpay)
    assert (st["passes"], st["levels"], st["inherited"], st["closed"]) == \
        (ost["passes"], ost["max_level"], ost["inherited"], ost["closed"]), (st, ost)
    return st


@pytest.mark.parametrize("dist", ["normal", "lognormal", "mixgauss", "exponential", "uniform01"])
def test_two_levels(dist):
    st = check(gen.make(dist, 200_000, 4), **SMALL)
    assert st["inherited"] > 0


@pytest.mark.parametrize("dist", ["normal", "lognormal2", "uniform_int", "root_dups", "two_dups"])
def test_three_levels_with_payload(dist):
    k = gen.make(dist, 400_000, 8)
    st = check(k, gen.index_payload(k.size), **DEEP)
    if dist in ("normal", "lognormal2"):
        assert st["levels"] >= 3 and st["inherited"] > 16


@pytest.mark.parametrize("dt", [np.float32, np.uint64])
def test_other_dtypes(dt):
    k = gen.as_dtype(gen.make("normal", 300_000, 9), {np.float32: ipls.F32, np.uint64: ipls.U64}[dt])
    check(k, gen.index_payload(k.size), **DEEP)


@pytest.mark.parametrize("pay", [False, True])
def test_small_tiles(pay):
    # 2048-key tiles: the 4-wave variants of the counting and class-byte scatter kernels
    k = gen.make("normal", 400_000, 15)
    st = check(k, gen.index_payload(k.size) if pay else None, tile_keys=2048, **DEEP)
    assert st["inherited"] > 16


def test_specials_and_ragged_sizes():
    r = np.random.default_rng(11)
    k = r.standard_normal(250_003)
    k[r.integers(0, k.size, 300)] = np.nan
    k[r.integers(0, k.size, 300)] = -np.nan
    k[r.integers(0, k.size, 200)] = np.inf
    k[r.integers(0, k.size, 200)] = -np.inf
    k[r.integers(0, k.size, 500)] = -0.0
    check(k, gen.index_payload(k.size), **DEEP)
    check(k.astype(np.float32), None, **DEEP)


def test_single_value_children_and_spikes():
    r = np.random.default_rng(12)
    check(np.where(r.random(200_000) < 0.5, 1.0, 2.0), None, **SMALL)
    k = r.standard_normal(300_000)
    k[: 100_000] = 0.25
    r.shuffle(k)
    check(k, gen.index_payload(k.size), **DEEP)


def test_segmented_batch():
    sizes = gen.segment_sizes_lognormal(300, 13, median=20_000, lo=2, hi=600_000)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = np.concatenate([gen.make(("normal", "lognormal", "uniform_int")[i % 3], int(s), 50 + i)
                           for i, s in enumerate(sizes)])
    pay = gen.index_payload(keys.size)
    print(f"inherit segmented nseg={sizes.size} total={keys.size}", flush=True)
    kd, pd, od = dev(keys), dev(pay), dev(off)
    st = ipls.sort_segmented_(kd, od, pd, params=ipls.default_params(inherit=1, **DEEP), stats=True)
    torch.cuda.synchronize()
    want, wpay, ost = oracle.sort_segmented(keys, off, pay, oparams(DEEP))
    assert same_bits(host(kd, keys.dtype), want)
    assert np.array_equal(host(pd, np.uint32), wpay)
    assert st["inherited"] == ost["inherited"] > 0


def test_default_parameters_at_2e7():
    # the 1% sample (2*10^5 keys) gives the first level's children about 780 sample keys each
    st = check(gen.make("normal", 20_000_000, 14))
    assert st["inherited"] > 100


def test_invalid_combinations_rejected():
    k = dev(gen.normal(10_000, 1))
    for kw in (dict(model=1), dict(model=2), dict(model=3), dict(equality=1), dict(inherit=2)):
        p = ipls.default_params(**{"inherit": 1, **kw})
        with pytest.raises(ipls.IplsError):
            ipls.sort_(k, None, params=p)
