"""Pins of the oracle's splitter-tree classifier (model = 3): the comparison-based classifier of
IPS4o that the paper measures its learned models against.

Splitters are re-derived from the sample by their definition (quantiles x[floor(i S / K)]),
buckets against numpy's searchsorted, progress on the cases that break a strict or a non-strict
rule, and full sorts against numpy and Python's stable sort.
"""
import struct

import numpy as np
import pytest

import gen
import oracle


def ords_f64(a):
    u = np.ascontiguousarray(a, np.float64).view(np.uint64)
    neg = (u >> np.uint64(63)) == 1
    return np.where(neg, ~u, u | np.uint64(1 << 63))


def tree_params(**kw):
    return oracle.params(model=3, **kw)


@pytest.mark.parametrize("dist", ["normal", "exponential", "uniform_int", "two_dups"])
@pytest.mark.parametrize("K", [4, 37, 256])
def test_splitters_are_sample_quantiles_and_buckets_match_searchsorted(dist, K):
    keys = gen.make(dist, 60_000, 3)
    p = tree_params(K=K, T=256)
    m, _, _ = oracle.fit_bucket(keys, p)
    assert m.kind == oracle.MODEL_TREE
    S = oracle.sample_size(keys.size, p)
    pos = oracle.sample_positions(keys.size, 0, S, p.seed).astype(np.int64)
    o = np.sort(ords_f64(keys[pos]))
    split = np.array([o[(i * S) // K] for i in range(1, K)], np.uint64)
    assert np.array_equal(np.array(m.split[:K - 1], np.uint64), split)
    strict = bool(split[0] < o[-1])
    assert m.tree_strict == int(strict)
    b = oracle.classify_model(keys, m)
    want = np.searchsorted(split, ords_f64(keys), side="left" if strict else "right")
    assert np.array_equal(b, want.astype(np.uint32))


def test_every_splitter_at_the_max_uses_the_non_strict_rule():
    # a few 1.0 reach the sample, too few for a splitter: every splitter is 5.0, the maximum
    k = np.array([1.0] * 1500 + [5.0] * 98_500)
    np.random.default_rng(2).shuffle(k)
    p = tree_params(K=16, T=100)
    m, _, _ = oracle.fit_bucket(k, p)
    assert m.kind == oracle.MODEL_TREE
    b = oracle.classify_model(k, m)
    assert m.tree_strict == 0 and set(b[k == 5.0]) == {15} and set(b[k == 1.0]) == {0}
    out, _, _ = oracle.sort(k, None, p)
    assert np.array_equal(out, np.sort(k))


def test_every_splitter_at_the_min_keeps_the_strict_rule():
    k = np.array([1.0] * 98_500 + [5.0] * 1500)
    np.random.default_rng(3).shuffle(k)
    p = tree_params(K=16, T=100)
    m, _, _ = oracle.fit_bucket(k, p)
    assert m.kind == oracle.MODEL_TREE
    b = oracle.classify_model(k, m)
    assert m.tree_strict == 1 and set(b[k == 1.0]) == {0} and set(b[k == 5.0]) == {15}
    out, _, _ = oracle.sort(k, None, p)
    assert np.array_equal(out, np.sort(k))


def total_order_key(v: float):
    bits = struct.unpack("<Q", struct.pack("<d", v))[0]
    return bits ^ 0xFFFFFFFFFFFFFFFF if bits >> 63 else bits | (1 << 63)


@pytest.mark.parametrize("dist", ["normal", "lognormal2", "root_dups", "zipf_u64", "uniform_int"])
def test_sorts_with_the_splitter_tree(dist):
    k = gen.make(dist, 100_000, 7)
    pay = gen.index_payload(k.size)
    out, opay, st = oracle.sort(k, pay, tree_params(K=64, T=512))
    if k.dtype == np.uint64:
        idx = sorted(range(k.size), key=lambda i: (int(k[i]), i))
    else:
        idx = sorted(range(k.size), key=lambda i: (total_order_key(float(k[i])), i))
    assert np.array_equal(opay, np.array(idx, np.uint32))
    assert np.array_equal(out.view(np.uint64), k[idx].view(np.uint64))
    assert st["passes"] >= 1
