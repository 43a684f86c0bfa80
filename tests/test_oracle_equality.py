"""Pins of the oracle's equality buckets (IPS4o's, applied to the linear model).

The paper gives no numbers for them; the pins are their definition written out independently
(heavy runs of the sorted sample found by brute force, FMCD re-called on the reduced sample),
the order and exclusivity properties the bucket mapping must have, full sorts against numpy and
Python's stable sort, and the gain on duplicate-heavy inputs.
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


def brute_heavy(keys, p):
    """Heavy values by definition: runs of the sorted sample longer than S/K, the first
    min(16, (K-4)/2) in ascending order."""
    n = keys.size
    S = oracle.sample_size(n, p)
    pos = oracle.sample_positions(n, 0, S, p.seed).astype(np.int64)
    o = np.sort(ords_f64(keys[pos]))
    vals, counts = np.unique(o, return_counts=True)
    emax = min(16, (p.num_buckets - 4) // 2)
    heavy = [int(v) for v, c in zip(vals, counts) if int(c) * p.num_buckets > S][:emax]
    return S, o, heavy


def dup_heavy_keys(n, seed, nvals=6, frac=0.6):
    r = np.random.default_rng(seed)
    k = r.standard_normal(n)
    hot = r.choice(np.round(r.standard_normal(nvals), 3), n)
    m = r.random(n) < frac
    k[m] = hot[m]
    return k


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("K", [16, 64, 256])
def test_heavy_values_and_reduced_fit_match_their_definition(seed, K):
    keys = dup_heavy_keys(40_000, seed)
    p = oracle.params(K=K, T=256, equality=1)
    m, _, _ = oracle.fit_bucket(keys, p)
    S, o, heavy = brute_heavy(keys, p)
    assert m.neq == len(heavy) > 0
    assert [int(m.heavy[e]) for e in range(m.neq)] == heavy
    assert m.Km == K - 2 * m.neq
    # the linear part is FMCD on the sample without the heavy runs
    keep = ~np.isin(o, np.array(heavy, np.uint64))
    xr = np.sort(keys[oracle.sample_positions(keys.size, 0, S, p.seed).astype(np.int64)])[keep]
    a, b, D = oracle.fmcd(xr, m.Km)
    assert (m.const0, m.a, m.b, m.D) == (0, a, b, D)


def test_equality_off_or_no_heavy_values_changes_nothing():
    keys = gen.normal(50_000, 4)
    m0, _, _ = oracle.fit_bucket(keys, oracle.params(T=256))
    m1, _, _ = oracle.fit_bucket(keys, oracle.params(T=256, equality=1))
    assert m1.neq == 0 and (m0.kind, m0.a, m0.b, m0.D) == (m1.kind, m1.a, m1.b, m1.D)


@pytest.mark.parametrize("seed", [5, 6])
def test_bucket_mapping_is_ordered_and_heavy_buckets_are_exclusive(seed):
    keys = dup_heavy_keys(30_000, seed, nvals=9)
    K = 64
    p = oracle.params(K=K, T=256, equality=1)
    m, _, _ = oracle.fit_bucket(keys, p)
    assert m.neq > 0
    b = oracle.classify_model(keys, m).astype(np.int64)
    assert b.max() < K
    order = np.argsort(ords_f64(keys), kind="stable")
    assert np.all(np.diff(b[order]) >= 0)  # buckets follow key order
    o = ords_f64(keys)
    for e in range(m.neq):
        h = np.uint64(m.heavy[e])
        hb = np.unique(b[o == h])
        assert hb.size == 1
        assert np.all(o[b == hb[0]] == h)  # the heavy value's bucket holds it alone


def test_two_values_become_two_closed_buckets():
    k = np.array([1.5] * 30_000 + [-2.0] * 20_000)
    np.random.default_rng(1).shuffle(k)
    p = oracle.params(K=16, T=100, equality=1)
    m, _, _ = oracle.fit_bucket(k, p)
    assert m.neq == 2 and m.const0 == 1
    out, _, st = oracle.sort(k, None, p)
    assert np.array_equal(out, np.sort(k))
    assert st["passes"] == 1 and st["closed"] == 2  # both equality buckets close at level 2


def test_single_value_sample_keeps_the_degenerate_rule():
    k = np.full(10_000, 7.0)
    k[:3] = [1.0, 2.0, 3.0]  # too rare to reach the sample as a run of its own
    m, _, _ = oracle.fit_bucket(k, oracle.params(K=16, T=100, equality=1))
    assert m.neq in (0, 1)
    out, _, _ = oracle.sort(k, None, oracle.params(K=16, T=100, equality=1))
    assert np.array_equal(out, np.sort(k))


def total_order_key(v: float):
    bits = struct.unpack("<Q", struct.pack("<d", v))[0]
    return bits ^ 0xFFFFFFFFFFFFFFFF if bits >> 63 else bits | (1 << 63)


@pytest.mark.parametrize("dist", ["uniform_int", "root_dups", "two_dups", "normal", "zipf_u64"])
def test_sorts_with_equality_buckets(dist):
    k = gen.make(dist, 120_000, 9)
    pay = gen.index_payload(k.size)
    p = oracle.params(K=64, T=512, equality=1)
    out, opay, _ = oracle.sort(k, pay, p)
    if k.dtype == np.uint64:
        idx = sorted(range(k.size), key=lambda i: (int(k[i]), i))
    else:
        idx = sorted(range(k.size), key=lambda i: (total_order_key(float(k[i])), i))
    assert np.array_equal(opay, np.array(idx, np.uint32))
    assert np.array_equal(out.view(np.uint64), k[idx].view(np.uint64))


def test_equality_buckets_cut_passes_on_zipf():
    z = gen.zipf_u64(400_000, 3)
    _, _, off = oracle.sort(z, None, oracle.params())
    _, _, on = oracle.sort(z, None, oracle.params(equality=1))
    assert on["keys_partitioned"] < 0.8 * off["keys_partitioned"]
    assert on["max_level"] <= off["max_level"]
