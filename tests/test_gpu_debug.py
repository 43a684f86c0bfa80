"""GPU tests of the invariant checks that IPLS_DEBUG_CHECKS switches on: after every pass the
histogram sums to each item's key count, the pass kept each item's multiset of keys and payloads,
and every key lies in the bucket its model gives it; after the sort every segment is sorted and
holds its input's multiset.  Valid sorts pass them and give the oracle's output; a mismatch that
the host plants in the final comparison (IPLS_DEBUG_CHECKS=2, every kernel runs as usual) comes
back as IPLS_ERR_DEVICE, and the same context then sorts correctly with the checks off.
"""
import numpy as np
import pytest

import gen
import oracle
import paper_2208_06902_amd as ipls

torch = pytest.importorskip("torch")
from gpu_util import dev, host, same_bits  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [
    # (name, dist, n, dtype, payload, library params, oracle params)
    ("fmcd normal", "normal", 1_000_003, np.float64, False, {}, {}),
    ("zipf u64 payload equality", "zipf_u64", 300_001, np.uint64, True, {"equality": 1}, {"equality": 1}),
    ("f32 lognormal2 auto", "lognormal2", 200_003, np.float32, False, {"model": 1, "num_buckets": 128, "leaves": 64},
     {"model": 1, "K": 128, "leaves": 64}),
    ("two dups splitter tree", "two_dups", 300_007, np.float64, True, {"model": 3}, {"model": 3}),
    ("inherit deep", "exponential", 200_000, np.float64, False,
     {"inherit": 1, "num_buckets": 16, "base_case_max": 256, "sample_divisor": 10},
     {"inherit": 1, "K": 16, "T": 256, "divisor": 10}),
]


def _keys(dist, n, dtype):
    k = gen.make(dist, n, 17)
    return k if k.dtype == dtype else k.astype(dtype)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_checks_pass_on_valid_sorts(case, monkeypatch):
    name, dist, n, dtype, with_pay, lib_kw, or_kw = case
    monkeypatch.setenv("IPLS_DEBUG_CHECKS", "1")
    keys = _keys(dist, n, dtype)
    pay = gen.index_payload(keys.size) if with_pay else None
    print(f"debug checks: {name} n={keys.size}", flush=True)
    kd = dev(keys)
    pd = None if pay is None else dev(pay)
    ipls.sort_(kd, pd, params=ipls.default_params(**lib_kw) if lib_kw else None)
    torch.cuda.synchronize()
    want, wpay, _ = oracle.sort(keys, pay, oracle.params(**or_kw))
    assert same_bits(host(kd, keys.dtype), want)
    if pay is not None:
        assert np.array_equal(host(pd, np.uint32), wpay)


def test_checks_pass_on_a_segmented_batch(monkeypatch):
    monkeypatch.setenv("IPLS_DEBUG_CHECKS", "1")
    r = np.random.default_rng(41)
    sizes = r.integers(1, 30_000, 300)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = gen.make("mixgauss", int(off[-1]), 42)
    print(f"debug checks: segmented nseg={sizes.size} total={keys.size}", flush=True)
    kd = dev(keys)
    ipls.sort_segmented_(kd, dev(off))
    torch.cuda.synchronize()
    want, _, _ = oracle.sort_segmented(keys, off, None, oracle.params())
    assert same_bits(host(kd, keys.dtype), want)


def test_planted_mismatch_is_reported_then_the_context_sorts(monkeypatch):
    keys = gen.make("lognormal", 500_000, 43)
    print("debug checks: planted mismatch", flush=True)
    monkeypatch.setenv("IPLS_DEBUG_CHECKS", "2")
    kd = dev(keys)
    with pytest.raises(ipls.IplsError) as e:
        ipls.sort_(kd)
    torch.cuda.synchronize()
    assert "IPLS_ERR_DEVICE" in str(e.value)
    monkeypatch.setenv("IPLS_DEBUG_CHECKS", "0")
    kd = dev(keys)
    ipls.sort_(kd)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort(keys, None, oracle.params())
    assert same_bits(host(kd, keys.dtype), want)
