"""Parity at the full workload sizes, in the launch configuration the benchmark times.

* 10^8 fp64 keys of each of the five distributions: the whole output against the oracle, bit
  for bit, with the benchmark's parameters (K 256, T 4096, sample capped at 4096 keys).
* 10^8 normal fp64 keys with sample inheritance (a 131072-key first sample): the whole output and
  the count of inherited partitions against the oracle.
* 2*10^8 Zipf(1.1) uint64 keys with their uint32 index as payload: the whole output, keys and
  payload, against the oracle (stable order is unique).
* 10^9 uniform uint64 keys: too large for the oracle in a test, so checked by properties that
  hold at any size: the output is non-decreasing and is the same multiset as the input
  (compared with an independent device sort of the input).

The two uint64 inputs are drawn on the GPU (gen.device); the oracle gets a host copy of the
same bytes.
"""
import numpy as np
import pytest

import gen
import gen.device as gdev
import oracle
import paper_2208_06902_amd as ipls

torch = pytest.importorskip("torch")
from gpu_util import same_bits  # noqa: E402

pytestmark = pytest.mark.gpu

BENCH = dict(num_buckets=256, base_case_max=4096, sample_max=4096)
FULL_DISTS = [("normal", 2), ("lognormal", 3), ("exponential", 4), ("mixgauss", 5), ("uniform_int", 6)]


def _sort_on_device(keys, payload=None, **kw):
    kd = torch.from_numpy(keys.view(np.int64) if keys.dtype == np.uint64 else keys).to("cuda:0")
    if keys.dtype == np.uint64:
        kd = kd.view(torch.uint64)
    pd = None if payload is None else torch.from_numpy(payload.view(np.int32)).to("cuda:0")
    st = ipls.sort_(kd, pd, params=ipls.default_params(**kw), stats=True)
    torch.cuda.synchronize()
    return kd, pd, st


@pytest.mark.parametrize("dist,seed", FULL_DISTS)
def test_1e8_fp64_against_oracle(dist, seed):
    n = 100_000_000
    print(f"full size {dist} n={n} seed={seed}", flush=True)
    keys = gen.make(dist, n, seed)
    kd, _, st = _sort_on_device(keys, **BENCH)
    got = kd.cpu().numpy()
    del kd
    want, _, ost = oracle.sort(keys, None, oracle.params(sample_max=4096))
    assert same_bits(got, want)
    assert (st["passes"], st["levels"]) == (ost["passes"], ost["max_level"])


def test_1e8_fp64_sample_inheritance_against_oracle():
    # a 131072-key first sample gives the 256 children about 512 sample keys each: they inherit
    n = 100_000_000
    print(f"full size normal n={n} with sample inheritance", flush=True)
    keys = gen.make("normal", n, 2)
    kd, _, st = _sort_on_device(keys, num_buckets=256, base_case_max=4096, sample_max=131072, inherit=1)
    got = kd.cpu().numpy()
    del kd
    want, _, ost = oracle.sort(keys, None, oracle.params(sample_max=131072, inherit=1))
    assert same_bits(got, want)
    assert (st["passes"], st["levels"]) == (ost["passes"], ost["max_level"])
    assert st["inherited"] == ost["inherited"] > 100


@pytest.mark.parametrize("equality", [0, 1])
def test_2e8_zipf_u64_payload_against_oracle(equality):
    n = 200_000_000
    print(f"full size zipf u64 + payload n={n} equality={equality}", flush=True)
    kd = gdev.zipf_u64(n, 8)
    keys = kd.cpu().numpy().view(np.uint64)
    pay = gen.index_payload(n)
    kd = kd.view(torch.uint64)
    pd = torch.from_numpy(pay.view(np.int32)).to("cuda:0")
    st = ipls.sort_(kd, pd, params=ipls.default_params(equality=equality, **BENCH), stats=True)
    torch.cuda.synchronize()
    got = kd.view(torch.int64).cpu().numpy().view(np.uint64)
    gpay = pd.cpu().numpy().view(np.uint32)
    del kd, pd
    want, wpay, ost = oracle.sort(keys, pay, oracle.params(sample_max=4096, equality=equality))
    assert np.array_equal(got, want)
    assert np.array_equal(gpay, wpay)
    assert st["closed"] == ost["closed"] and st["passes"] == ost["passes"]


def test_1e9_u64_sorted_permutation():
    n = 1_000_000_000
    print(f"full size u64 uniform n={n}", flush=True)
    src = gdev.u64_uniform(n, 7)
    kd = src.clone().view(torch.uint64)
    st = ipls.sort_(kd, None, params=ipls.default_params(**BENCH), stats=True)
    torch.cuda.synchronize()
    # uint64 order is the signed order of the values with the top bit flipped
    flip = torch.tensor(-(2**63), dtype=torch.int64, device="cuda:0")
    got = torch.bitwise_xor(kd.view(torch.int64), flip)
    del kd
    assert bool((got[1:] >= got[:-1]).all())
    ref = torch.sort(torch.bitwise_xor(src, flip)).values
    del src
    assert torch.equal(ref, got)
    assert st["levels"] >= 3
