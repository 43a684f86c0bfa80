"""Pins of the oracle's sample inheritance.

The paper samples every bucket afresh.  With inheritance a child bucket may reuse the parent's
sorted sample restricted to it.  The pins are:

* the rule, restated here in numpy from separately pinned parts: FMCD, the classifier and the
  sample.  A child of the first level inherits when it is partitioned itself, its restricted
  sample holds at least max(3, sample_min or 2K) keys, and FMCD on it is usable.  The oracle's
  count of inherited partitions must equal the count the rule gives.
* that restricted samples are contiguous ranges of the parent's sorted sample.  This holds because
  the line is monotone in the key order.
* full sorts against numpy and Python's stable sort, over two and three levels of inheritance.
"""
import struct

import numpy as np
import pytest

import gen
import oracle


def rule_count(keys, p):
    """Inherited partitions at level 2 by the rule, for inputs whose level-2 buckets all go to the
    base case."""
    K, T = p.num_buckets, p.base_case_max
    m, _, _ = oracle.fit_bucket(keys, p)
    assert m.kind == oracle.MODEL_LINEAR
    S = oracle.sample_size(keys.size, p)
    x = oracle.sorted_sample(keys, S, p.seed)
    cls_s = oracle.classify_model(x, m).astype(np.int64)
    assert np.all(np.diff(cls_s) >= 0)  # restricted samples are contiguous ranges
    counts = np.bincount(oracle.classify_model(keys, m).astype(np.int64), minlength=K)
    thr = max(3, p.sample_min or 2 * K)
    n_inh = 0
    for c in range(K):
        r = x[cls_s == c]
        ok = counts[c] > T and r.size >= thr and np.isfinite(r[0]) and np.isfinite(r[-1])
        if ok:
            f = oracle.fmcd(r, K)
            ok = f is not None and f[0] > 0 and np.isfinite(f[0]) and np.isfinite(f[1])
        n_inh += int(ok)
        # the sample the oracle hands child c is exactly this restriction (or none)
        got = oracle.child_sample(keys, c, p)
        if ok:
            assert np.array_equal(got, oracle.ord_keys(r.astype(keys.dtype))), c
        else:
            assert got.size == 0, c
    return n_inh, counts


CASES = ["normal", "lognormal", "mixgauss", "exponential", "uniform01"]


@pytest.mark.parametrize("dist", CASES)
def test_inherited_count_follows_the_rule(dist):
    keys = gen.make(dist, 200_000, 4)
    p = oracle.params(K=16, T=4096, divisor=10, inherit=1)
    want, _ = rule_count(keys, p)
    out, _, st = oracle.sort(keys, None, p)
    assert np.array_equal(out, np.sort(keys))
    assert st["max_level"] == 2, st  # every level-2 bucket went to the base case
    assert st["inherited"] == want > 0, (st, want)


def test_single_value_children_draw_a_fresh_sample():
    # two values: the first level splits them, each child's restricted sample is one value, FMCD on
    # it is unusable, so each child samples afresh and is closed as homogeneous
    keys = np.where(np.random.default_rng(3).random(200_000) < 0.5, 1.0, 2.0)
    p = oracle.params(K=16, T=4096, divisor=10, inherit=1)
    want, counts = rule_count(keys, p)
    out, _, st = oracle.sort(keys, None, p)
    assert np.array_equal(out, np.sort(keys))
    assert want == 0 and (counts > 4096).sum() == 2
    assert st["inherited"] == 0 and st["closed"] == 2 and st["max_level"] == 1


def test_threshold_above_every_restricted_sample_means_no_inheritance():
    keys = gen.normal(200_000, 5)
    p = oracle.params(K=16, T=4096, divisor=10, sample_min=4096, inherit=1)
    out, _, st = oracle.sort(keys, None, p)
    assert np.array_equal(out, np.sort(keys)) and st["inherited"] == 0


def test_inheritance_off_matches_fresh_samples_and_the_rule_off():
    keys = gen.normal(200_000, 6)
    _, _, off = oracle.sort(keys, None, oracle.params(K=16, T=4096, divisor=10))
    assert off["inherited"] == 0
    want, _ = rule_count(keys, oracle.params(K=16, T=4096, divisor=10, inherit=1))
    _, _, on = oracle.sort(keys, None, oracle.params(K=16, T=4096, divisor=10, inherit=1))
    assert on["inherited"] == want > 0
    assert on["max_level"] == off["max_level"] == 2


def total_order_key(v: float):
    bits = struct.unpack("<Q", struct.pack("<d", v))[0]
    return bits ^ 0xFFFFFFFFFFFFFFFF if bits >> 63 else bits | (1 << 63)


@pytest.mark.parametrize("dist", ["normal", "uniform_int", "root_dups", "lognormal2", "zipf_u64"])
def test_three_levels_sort_stably(dist):
    k = gen.make(dist, 400_000, 8)
    pay = gen.index_payload(k.size)
    p = oracle.params(K=16, T=256, divisor=10, inherit=1)
    out, opay, st = oracle.sort(k, pay, p)
    if k.dtype == np.uint64:
        idx = np.argsort(k, kind="stable")
    else:
        idx = np.array(sorted(range(k.size), key=lambda i: (total_order_key(float(k[i])), i)))
    assert np.array_equal(opay, idx.astype(np.uint32))
    assert np.array_equal(out.view(np.uint64), k[idx].view(np.uint64))
    if dist in ("normal", "lognormal2"):
        assert st["max_level"] >= 3 and st["inherited"] > 16  # inherited at two levels


def test_segments_inherit_independently():
    sizes = [150_000, 3, 90_000, 0, 120_000]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = np.concatenate([gen.make("normal", s, 30 + i) for i, s in enumerate(sizes)])
    p = oracle.params(K=16, T=4096, divisor=10, inherit=1)
    out, _, st = oracle.sort_segmented(keys, off, None, p)
    total = 0
    for i in range(len(sizes)):
        seg = keys[off[i]:off[i + 1]]
        assert np.array_equal(out[off[i]:off[i + 1]], np.sort(seg))
        if seg.size:
            _, _, one = oracle.sort(seg, None, p)
            total += one["inherited"]
    assert st["inherited"] == total > 0


@pytest.mark.parametrize("kw", [dict(model=1), dict(model=2), dict(model=3), dict(equality=1)])
def test_inheritance_needs_the_plain_line(kw):
    with pytest.raises(ValueError):
        oracle.sort(gen.normal(1000, 1), None, oracle.params(inherit=1, **kw))
