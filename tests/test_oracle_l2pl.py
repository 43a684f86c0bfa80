"""Pins of the oracle's two-level piecewise-linear CDF model (no GPU).

The paper fixes only the model's form (a two-level RMI whose leaves predict K times the eCDF,
trained by mean-squared error); it prints no numbers for it.  These tests pin the oracle to the
mathematics instead: the loss against its definition evaluated by numpy, the gradient against
central finite differences, the trained leaves against each leaf's closed-form least-squares
line, and the envelope and classifier against monotonicity.
"""
from fractions import Fraction

import numpy as np
import pytest

import gen
import oracle


def sample_of(dist, S, seed):
    return np.sort(gen.make(dist, S, seed))


def geometry(x, K, M):
    a, b, D = oracle.fmcd(x, M)
    first, c, h, m2 = oracle.l2pl_geometry(x, M, a, b)
    return first.astype(np.int64), c, h


@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20", "normal"])
def test_leaves_are_contiguous_and_cover_sample(dist):
    x = sample_of(dist, 20000, 1)
    a, b, D = oracle.fmcd(x, 256)
    first, c, h, m2 = oracle.l2pl_geometry(x, 256, a, b)
    first = first.astype(np.int64)
    assert first[0] == 0 and first[-1] == x.size and np.all(np.diff(first) >= 0)
    leaf = oracle.classify_linear(x, a, b, 256)
    for l in range(256):
        xs = x[first[l]:first[l + 1]]
        assert np.all(leaf[first[l]:first[l + 1]] == l)
        if xs.size:
            # centre = mean, scale = largest distance to it, m2 = mean of u^2
            assert c[l] == pytest.approx(xs.mean(), rel=1e-12, abs=1e-300)
            assert h[l] == (np.abs(xs - c[l]).max() or 1.0)
            assert m2[l] == pytest.approx(np.mean(((xs - c[l]) / h[l]) ** 2), rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20"])
def test_loss_matches_its_definition(dist):
    K, M = 256, 256
    x = sample_of(dist, 8000, 2)
    first, c, h = geometry(x, K, M)
    ab = np.random.default_rng(0).standard_normal(2 * M)
    g, loss = oracle.l2pl_grad(x, K, M, first, c, h, ab)
    y = K * (np.arange(x.size) + 0.5) / x.size
    for l in range(M):
        j0, j1 = first[l], first[l + 1]
        if j1 == j0:
            assert loss[l] == 0.0 and g[2 * l] == 0.0 and g[2 * l + 1] == 0.0
            continue
        u = (x[j0:j1] - c[l]) / h[l]
        r = ab[2 * l] * u + ab[2 * l + 1] - y[j0:j1]
        assert loss[l] == pytest.approx(np.mean(r * r), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20", "exponential"])
def test_gradient_matches_finite_differences(dist):
    K, M = 256, 256
    x = sample_of(dist, 6000, 3)
    first, c, h = geometry(x, K, M)
    ab = np.random.default_rng(1).standard_normal(2 * M) * 3
    g, _ = oracle.l2pl_grad(x, K, M, first, c, h, ab)
    eps = 1e-5
    for k in range(2 * M):
        e = np.zeros(2 * M)
        e[k] = eps
        _, lp = oracle.l2pl_grad(x, K, M, first, c, h, ab + e)
        _, lm = oracle.l2pl_grad(x, K, M, first, c, h, ab - e)
        fd = (lp[k // 2] - lm[k // 2]) / (2 * eps)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-6)


@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20", "uniform01"])
def test_training_converges_to_leaf_least_squares(dist):
    K, M = 256, 256
    x = sample_of(dist, 30000, 4)
    first, c, h = geometry(x, K, M)
    out = oracle.l2pl_train(x, K, M, 200)
    assert out is not None
    root, leaf, ab = out
    y = K * (np.arange(x.size) + 0.5) / x.size
    checked = 0
    for l in range(M):
        j0, j1 = first[l], first[l + 1]
        if j1 - j0 < 3 or x[j1 - 1] == x[j0]:
            continue
        u = (x[j0:j1] - c[l]) / h[l]
        A = np.stack([u, np.ones_like(u)], 1)
        (alpha, beta), *_ = np.linalg.lstsq(A, y[j0:j1], rcond=None)
        if alpha < 0:  # the trained slope is clipped at zero
            continue
        assert ab[2 * l] == pytest.approx(alpha, rel=1e-5, abs=1e-6)
        assert ab[2 * l + 1] == pytest.approx(beta, rel=1e-6, abs=1e-6)
        checked += 1
    assert checked > 100


@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20", "uniform_int"])
def test_envelope_is_monotone_and_classifier_is_monotone(dist):
    K, M = 256, 256
    x = sample_of(dist, 20000, 5)
    root, leaf, ab = oracle.l2pl_train(x, K, M, 32)
    A, B, LO, HI = leaf[0::4], leaf[1::4], leaf[2::4], leaf[3::4]
    assert LO[0] == 0.0 and np.all(LO[1:] == HI[:-1]) and np.all(HI >= LO) and np.all(A >= 0)
    assert np.all(HI <= K)
    keys = np.sort(gen.make(dist, 50000, 6))
    m = oracle.Model(kind=oracle.MODEL_L2PL, K=K)
    buckets = oracle.classify_model(keys, m, root, leaf, M)
    assert np.all(np.diff(buckets.astype(np.int64)) >= 0)


@pytest.mark.parametrize("model", [1, 2])
@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20", "normal", "uniform_int"])
def test_sort_with_learned_model_equals_numpy(model, dist):
    k = gen.make(dist, 60000, 7)
    out, _, st = oracle.sort(k, None, oracle.params(K=64, T=256, model=model))
    assert np.array_equal(out, np.sort(k))
    if model == 2:
        assert st["l2pl_used"] >= 1


@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20"])
def test_learned_model_lowers_max_load_on_skew(dist):
    # the gain the two-level model is meant to bring: a lower maximum bucket load than FMCD
    k = gen.make(dist, 10**6, 8)
    m, root, leaf = oracle.fit_bucket(k, oracle.params(model=1))
    assert m.kind == oracle.MODEL_L2PL
    assert m.max_load_l2pl < m.max_load_linear
    full = np.bincount(oracle.classify_model(k, m, root, leaf, 256), minlength=256).max()
    lin = oracle.Model(kind=oracle.MODEL_LINEAR, K=256, a=m.a, b=m.b)
    full_lin = np.bincount(oracle.classify_model(k, lin), minlength=256).max()
    assert full < full_lin


def fma_exact(a, x, b):
    """fma(a, x, b): the exact a*x + b rounded once (Fraction -> float rounds to nearest even)."""
    return float(Fraction(a) * Fraction(x) + Fraction(b))


@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20", "normal"])
def test_exported_leaf_line_is_the_trained_line(dist):
    # A leaf is trained as t = alpha u + beta in its centred coordinate u = (x - c)/h and exported
    # for classification as t = fma(A, x, B).  The export must be that same line in x: for every
    # sample key of every non-empty leaf, fma(A, x, B) agrees with the exact alpha (x - c)/h + beta
    # up to the rounding of A = alpha/h, of A c and B = beta - A c, and of the fma itself, each at
    # most half an ulp: |error| <= 2^-52 (|A x| + 3 |A c| + |beta| + |t|).  A B that dropped the
    # 1/h, or a line in the wrong coordinate, misses by whole buckets.
    K, M = 256, 256
    x = sample_of(dist, 12000, 9)
    root, leaf, ab = oracle.l2pl_train(x, K, M, 4)
    first, c, h, _ = oracle.l2pl_geometry(x, M, root[0], root[1])
    first = first.astype(np.int64)
    eps = Fraction(1, 2**52)
    checked = 0
    for l in range(M):
        j0, j1 = first[l], first[l + 1]
        if j1 == j0:
            continue
        A, B = leaf[4 * l], leaf[4 * l + 1]
        alpha, beta = Fraction(ab[2 * l]), Fraction(ab[2 * l + 1])
        cl, hl = Fraction(c[l]), Fraction(h[l])
        for j in range(j0, j1, max(1, (j1 - j0) // 4)):
            xj = Fraction(x[j])
            exact = alpha * (xj - cl) / hl + beta
            got = Fraction(fma_exact(A, x[j], B))
            bound = eps * (abs(Fraction(A) * xj) + 3 * abs(Fraction(A) * cl) + abs(beta) + abs(exact))
            assert abs(got - exact) <= bound, (l, j, float(got), float(exact))
            checked += 1
    assert checked > 200


@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20", "exponential"])
def test_auto_policy_tries_the_learned_model_only_where_fmcd_can_overflow(dist):
    # FMCD's conflict degree D bounds a bucket's sample keys, so its buckets hold about D n / S of
    # the n keys at most.  The auto policy trains the two-level model only when that exceeds the
    # base-case threshold T (D n > T S); elsewhere the item keeps its line untrained.  D comes from
    # the exhaustive search of the FMCD definition on the item's sample, not from the oracle's fit.
    import test_oracle_pins as pins
    K, n = 64, 20000
    keys = gen.make(dist, n, 12)
    p0 = oracle.params(K=K, model=1)
    S = oracle.sample_size(n, p0)
    x = np.sort(keys[oracle.sample_positions(n, 0, S, p0.seed).astype(np.int64)])
    D, _, _ = pins.fmcd_brute(list(x), K)
    t_try, t_keep = max(1, D * n // S - 1), D * n // S + 1
    assert D * n > t_try * S and D * n <= t_keep * S
    m, _, _ = oracle.fit_bucket(keys, oracle.params(K=K, T=t_keep, model=1))
    assert m.D == D and m.kind == oracle.MODEL_LINEAR and m.max_load_l2pl == 0 and m.max_load_linear == 0
    m, _, _ = oracle.fit_bucket(keys, oracle.params(K=K, T=t_try, model=1))
    assert m.D == D and m.max_load_l2pl > 0
    assert (m.kind == oracle.MODEL_L2PL) == (m.max_load_l2pl < m.max_load_linear)
    # the forced two-level policy ignores the gate
    m, _, _ = oracle.fit_bucket(keys, oracle.params(K=K, T=t_keep, model=2))
    assert m.max_load_l2pl > 0
