"""Hypothesis property tests of the oracle on tiny inputs: the output is the stable sort by IEEE
totalOrder (a brute-force definition), for any small parameters, with or without the options."""
import struct

import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402


def total_order_key(v: float):
    bits = struct.unpack("<Q", struct.pack("<d", v))[0]
    return bits ^ 0xFFFFFFFFFFFFFFFF if bits >> 63 else bits | (1 << 63)


floats = st.floats(allow_nan=True, allow_infinity=True, width=64)
small_ints = st.integers(min_value=-4, max_value=4).map(float)


@settings(max_examples=300, deadline=None)
@given(keys=st.lists(st.one_of(floats, small_ints), min_size=0, max_size=300),
       K=st.sampled_from([4, 5, 16, 64]), T=st.sampled_from([1, 2, 8, 40]),
       model=st.sampled_from([0, 1, 3]), equality=st.sampled_from([0, 1]), seed=st.integers(0, 2**32))
def test_oracle_is_the_stable_total_order_sort(keys, K, T, model, equality, seed):
    k = np.array(keys, np.float64)
    pay = np.arange(k.size, dtype=np.uint32)
    p = oracle.params(K=K, T=T, sample_min=min(2 * K, T) or 1, seed=seed, model=model, leaves=4,
                      equality=equality)
    out, opay, _ = oracle.sort(k, pay, p)
    idx = sorted(range(k.size), key=lambda i: (total_order_key(float(k[i])), i))
    assert np.array_equal(opay, np.array(idx, np.uint32))
    assert np.array_equal(out.view(np.uint64), k[idx].view(np.uint64))


@settings(max_examples=200, deadline=None)
@given(keys=st.lists(st.integers(min_value=0, max_value=2**64 - 1), min_size=0, max_size=300),
       K=st.sampled_from([4, 16, 256]), T=st.sampled_from([1, 16, 64]), equality=st.sampled_from([0, 1]))
def test_oracle_sorts_u64(keys, K, T, equality):
    k = np.array(keys, np.uint64)
    out, _, _ = oracle.sort(k, None, oracle.params(K=K, T=T, sample_min=min(2 * K, T), equality=equality))
    assert np.array_equal(out, np.sort(k))


@settings(max_examples=200, deadline=None)
@given(keys=st.lists(st.one_of(floats, small_ints), min_size=0, max_size=400),
       K=st.sampled_from([4, 5, 8]), T=st.sampled_from([1, 4, 16]), seed=st.integers(0, 2**32))
def test_oracle_with_inheritance_is_the_stable_total_order_sort(keys, K, T, seed):
    # a half-size sample gives children restricted samples of several keys even on tiny inputs
    k = np.array(keys, np.float64)
    pay = np.arange(k.size, dtype=np.uint32)
    p = oracle.params(K=K, T=T, divisor=2, sample_min=min(3, T) or 1, seed=seed, inherit=1)
    out, opay, _ = oracle.sort(k, pay, p)
    idx = sorted(range(k.size), key=lambda i: (total_order_key(float(k[i])), i))
    assert np.array_equal(opay, np.array(idx, np.uint32))
    assert np.array_equal(out.view(np.uint64), k[idx].view(np.uint64))


def test_tiny_inputs_do_inherit():
    # the property test above reaches the inheritance path
    k = np.random.default_rng(1).standard_normal(400)
    _, _, st_ = oracle.sort(k, None, oracle.params(K=4, T=4, divisor=2, sample_min=3, inherit=1))
    assert st_["inherited"] > 10
