"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test checks the oracle against something other than itself: the Worked Example's printed
layouts, brute force over tiny inputs, closed forms, exact rational arithmetic, IEEE 754
totalOrder written out from its definition, Python's stable sort, and a published test vector.
"""
import json
import math
import os
import struct
from fractions import Fraction

import numpy as np
import pytest

import gen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load_worked():
    with open(os.path.join(GOLD, "worked_example.json")) as f:
        return json.load(f)


# ---------------------------------------------------------------- Worked Example (Proposed Algorithm)

def test_worked_example_buckets_match_paper_colours():
    w = load_worked()
    keys = np.array(w["input"], np.float64)
    got = oracle.classify_linear(keys, w["a"], w["b"], w["k"])
    colour_of = dict(zip(w["buffered_layout"], w["buffered_colours"]))
    want = [w["colour_bucket"][colour_of[k]] for k in w["input"]]
    assert got.tolist() == want
    # the text's own example: key 28 -> floor(2.65) = 2
    i = w["input"].index(w["text_example"]["key"])
    assert got[i] == w["text_example"]["bucket"]
    assert np.bincount(got, minlength=4).tolist() == [7, 2, 4, 7]


def test_worked_example_contiguous_layout_is_stable_distribution():
    w = load_worked()
    keys = np.array(w["input"], np.float64)
    b = oracle.classify_linear(keys, w["a"], w["b"], w["k"])
    assert oracle.stable_layout(keys, b, w["k"]).tolist() == w["contiguous_layout"]
    assert [w["colour_bucket"][c] for c in w["contiguous_colours"]] == sorted(b.tolist())


def test_worked_example_buffered_layout():
    w = load_worked()
    keys = np.array(w["input"], np.float64)
    b = oracle.classify_linear(keys, w["a"], w["b"], w["k"])
    assert oracle.buffered_layout(keys, b, w["k"], w["buffer_size"]).tolist() == w["buffered_layout"]


def test_worked_example_final_output():
    w = load_worked()
    keys = np.array(w["input"], np.float64)
    p = oracle.params(K=w["k"], T=w["base_case_below"] - 1, sample_min=8)
    out, _, st = oracle.sort(keys, None, p)
    assert out.tolist() == w["sorted"]
    assert st["passes"] >= 1


def test_worked_example_boundary_keys_fp64():
    # t = fma(0.15, x, -1.55) in fp64 for the keys nearest a bucket boundary, pinned by exact
    # rational arithmetic: the rounded t must be within half an ulp of the exact product-sum
    a, b = 0.15, -1.55
    for x in (10.0, 11.0, 22.0, 25.0):
        exact = Fraction(a) * Fraction(x) + Fraction(b)
        t = math.fma(a, x, b) if hasattr(math, "fma") else float(exact)
        assert abs(Fraction(t) - exact) <= Fraction(math.ulp(t)) / 2
    got = oracle.classify_linear(np.array([10.0, 11.0, 22.0, 25.0]), a, b, 4)
    # 0.15 and -1.55 are not exact in binary: 10 -> t just below 0, 22 -> just below 1.75
    assert got.tolist() == [0, 0, 1, 2]


# ---------------------------------------------------------------- FMCD (Linear Models section)

def fmcd_brute(x, K):
    """Smallest D >= 1 whose every (D+1)-key window spans at least u(D) = (x[S-1-D]-x[D])/(K-2),
    searched exhaustively; D stops at floor(S/3), past which the previous spread is kept."""
    S = len(x)
    u = lambda D: (x[S - 1 - D] - x[D]) / (K - 2)
    for D in range(1, S // 3 + 1):
        uD = u(D)
        if all(x[i + D] - x[i] >= uD for i in range(S - D)):
            return D, uD, False
    return S // 3 + 1, u(S // 3), True


@pytest.mark.parametrize("trial", range(40))
def test_fmcd_matches_brute_force_min_D(trial):
    r = np.random.default_rng(1000 + trial)
    for _ in range(50):
        S = int(r.integers(3, 60))
        K = int(r.integers(4, 20))
        kind = r.integers(0, 3)
        if kind == 0:
            x = np.sort(r.random(S))
        elif kind == 1:
            x = np.sort(r.integers(0, 8, S).astype(np.float64))
        else:
            x = np.sort(r.standard_normal(S) ** 3)
        a, b, D = oracle.fmcd(x, K)
        Db, ub, capped = fmcd_brute(x.tolist(), K)
        assert D == Db, (x.tolist(), K)
        if ub > 0:
            assert a == 1.0 / ub


def windows_span(x, D, K):
    """The conflict-degree condition for D, vectorised: every (D+1)-key window spans u(D)."""
    S = x.size
    u = (x[S - 1 - D] - x[D]) / (K - 2)
    return bool(np.all(x[D:] - x[:S - D] >= u))


@pytest.mark.parametrize("dist,S,K", [("normal", 200_000, 256), ("lognormal2", 100_000, 256),
                                      ("mixgauss", 50_000, 37), ("uniform_int", 30_000, 256),
                                      ("exponential", 4096, 256), ("uniform01", 1_000_000, 256)])
def test_fmcd_D_is_minimal_at_sample_sizes(dist, S, K):
    # at the sample sizes the sort uses: the condition holds at the returned D and fails at D - 1
    # (checked directly, without relying on the search the oracle uses); capped: fails at S//3
    x = np.sort(gen.make(dist, S, 3))
    a, b, D = oracle.fmcd(x, K)
    if D > S // 3:
        assert D == S // 3 + 1 and not windows_span(x, S // 3, K)
        return
    assert windows_span(x, D, K)
    assert D == 1 or not windows_span(x, D - 1, K)
    assert a == 1.0 / ((x[S - 1 - D] - x[D]) / (K - 2))


def test_fmcd_condition_is_monotone_in_D():
    # the reason a bisection over D finds the smallest D: once the condition holds, it holds for
    # every larger D (checked exhaustively on small samples with heavy duplication)
    r = np.random.default_rng(77)
    for _ in range(300):
        S = int(r.integers(3, 120))
        K = int(r.integers(4, 30))
        x = np.sort(np.round(r.standard_normal(S) * r.choice([1, 4, 40])))
        seen = False
        for D in range(1, S // 3 + 1):
            ok = windows_span(x, D, K)
            assert ok or not seen
            seen = seen or ok


@pytest.mark.parametrize("N,K", [(20, 4), (100, 10), (1000, 258), (37, 6), (513, 256), (4097, 256)])
def test_fmcd_arithmetic_progression_closed_form(N, K):
    # x_j = j: every D-window spans exactly D, u(D) = (N-1-2D)/(K-2), so the first D that works
    # is the smallest D with D*K >= N-1, i.e. D = max(1, ceil((N-1)/K)).
    x = np.arange(N, dtype=np.float64)
    a, b, D = oracle.fmcd(x, K)
    assert D == max(1, -(-(N - 1) // K))
    u = Fraction(N - 1 - 2 * D, K - 2)
    assert abs(Fraction(a) - 1 / u) <= Fraction(math.ulp(a))
    b_exact = (K - (1 / u) * (N - 1)) / 2  # x[S-1-D] + x[D] = N-1
    # K - a (N-1) cancels: the rounding error is a few ulps of K, not of b
    assert abs(Fraction(b) - b_exact) <= 4 * Fraction(math.ulp(float(K)))


def test_fmcd_worked_example_vector():
    # sorted Worked Example keys, K = 4: D = 6, u = (33 - 13)/2 = 10, a = 1/10; exact b = -3/10
    x = np.sort(np.array(load_worked()["input"], np.float64))
    a, b, D = oracle.fmcd(x, 4)
    assert D == 6 and fmcd_brute(x.tolist(), 4)[0] == 6
    assert a == 0.1
    # b = (4 - 0.1 * 46) / 2 cancels against K = 4: within an ulp of 4 of the exact -3/10
    assert abs(Fraction(b) - Fraction(-3, 10)) <= Fraction(math.ulp(4.0))
    # fp64 rounding puts x[D] = 13 just below t = 1, hence bucket 0 and counts [7, 2, 4, 7]
    buckets = oracle.classify_linear(np.array(load_worked()["input"], np.float64), a, b, 4)
    assert np.bincount(buckets, minlength=4).tolist() == [7, 2, 4, 7]


def test_fmcd_small_vector_uncapped():
    # every 3-window of this sample spans 1 >= u(3) = (2 - 1)/2, and 3*3 <= 10: uncapped
    x = np.array([0, 0, 0, 1, 1, 1, 2, 2, 2, 3], np.float64)
    a, b, D = oracle.fmcd(x, 4)
    Db, ub, capped = fmcd_brute(x.tolist(), 4)
    assert not capped and D == Db == 3 and a == 1.0 / ub
    assert (a, b, D) == (2.0, -1.0, 3)


def test_fmcd_capped_case():
    # a run of five equal keys defeats every window width up to floor(10/3) = 3: the search gives
    # up with D = 4, keeps u(3) = (x[6] - x[3]) / 2 = 1, and centres with x[5] + x[4] = 1
    x = np.array([0, 0, 0, 0, 0, 1, 2, 3, 4, 5], np.float64)
    a, b, D = oracle.fmcd(x, 4)
    Db, ub, capped = fmcd_brute(x.tolist(), 4)
    assert capped and D == Db == 4 and ub == 1.0
    assert (a, b) == (1.0, 1.5)


@pytest.mark.parametrize("x", [[5.0] * 10, [1.0] * 4 + [2.0] * 12 + [3.0] * 4, [1.0] * 30 + [2.0] * 70])
def test_fmcd_degenerate_spread(x):
    a, b, D = oracle.fmcd(np.array(x), 4)
    assert math.isinf(a) and (math.isnan(b) or math.isinf(b))


def test_fmcd_progress_points():
    # uncapped: x[D] maps to t ~ 1 and x[S-1-D] to t ~ K-1 (the offset's definition)
    r = np.random.default_rng(7)
    for _ in range(200):
        S = int(r.integers(50, 400))
        K = int(r.integers(4, 64))
        x = np.sort(r.random(S))
        a, b, D = oracle.fmcd(x, K)
        if 3 * D > S:
            continue
        assert abs(a * x[D] + b - 1.0) < 1e-9 * K
        assert abs(a * x[S - 1 - D] + b - (K - 1)) < 1e-9 * K


def test_fmcd_conflict_degree_bound():
    # distinct sample keys, uncapped D: no bucket of the fitted model holds more than D+1 samples
    r = np.random.default_rng(11)
    seen = 0
    for _ in range(400):
        S = int(r.integers(20, 500))
        K = int(r.integers(4, 40))
        x = np.unique(r.random(S) * r.choice([1.0, 1e3, 1e-3]))
        if x.size < 3:
            continue
        a, b, D = oracle.fmcd(x, K)
        if 3 * D > x.size:
            continue
        load = np.bincount(oracle.classify_linear(x, a, b, K), minlength=K).max()
        assert load <= D + 1
        seen += 1
    assert seen > 300


# ---------------------------------------------------------------- key map (IEEE 754 totalOrder)

def test_ord_total_order_f64():
    f = np.finfo(np.float64)
    neg_nan = struct.unpack("<d", struct.pack("<Q", 0xFFF8000000000000))[0]
    pos_nan = struct.unpack("<d", struct.pack("<Q", 0x7FF8000000000000))[0]
    ordered = [neg_nan, -np.inf, -f.max, -1.0, -f.tiny, -5e-324, -0.0, 0.0, 5e-324, f.tiny, 1.0, f.max, np.inf,
               pos_nan]
    o = oracle.ord_keys(np.array(ordered, np.float64))
    assert all(int(o[i]) < int(o[i + 1]) for i in range(len(o) - 1))


def test_ord_total_order_f32():
    f = np.finfo(np.float32)
    ordered = [-np.inf, -f.max, -1.0, -f.tiny, -0.0, 0.0, f.tiny, 1.0, f.max, np.inf]
    o = oracle.ord_keys(np.array(ordered, np.float32))
    assert all(int(o[i]) < int(o[i + 1]) for i in range(len(o) - 1))
    assert int(o.max()) < 2**32


def test_ord_and_val_u64():
    u = np.array([0, 1, 2**53, 2**53 + 1, 2**53 + 3, 2**63, 2**64 - 1], np.uint64)
    assert oracle.ord_keys(u).tolist() == u.tolist()
    v = oracle.val_keys(u)
    # u64 -> f64 rounds to nearest, ties to even (exact rational check)
    for x, y in zip(u.tolist(), v.tolist()):
        err = abs(Fraction(y) - x)
        assert err <= Fraction(math.ulp(y)) / 2
    assert v[3] == 2.0**53 and v[4] == 2.0**53 + 4 and v[6] == 2.0**64


def test_ord_matches_numeric_order_random():
    x = np.random.default_rng(3).standard_normal(5000) * 1e10
    o = oracle.ord_keys(x)
    assert np.array_equal(np.argsort(o, kind="stable"), np.argsort(x, kind="stable"))


# ---------------------------------------------------------------- sample

def test_splitmix64_published_vector():
    # SplitMix64 from state 0: the first outputs are mix64(gamma), mix64(2 gamma)
    g = 0x9E3779B97F4A7C15
    assert oracle.mix64(g) == 0xE220A8397B1DCDAF
    assert oracle.mix64((2 * g) % 2**64) == 0x6E789E6AA1B965F4


@pytest.mark.parametrize("n", [4097, 10**4, 10**6, 10**8, 3 * 10**9])
def test_sample_size_policy(n):
    p = oracle.params()
    S = oracle.sample_size(n, p)
    assert S == min(n, max(512, -(-n // 100)))


def test_log2_against_exact_bounds():
    # 24 fractional bits, truncated: log2(n) - 2^-23 < L <= log2(n) + tiny, and exact at powers of two
    import math
    r = np.random.default_rng(11)
    ns = [1, 2, 3, 5, 4095, 4096, 4097, 10**6, 10**8, 10**9, 2**53 - 1, 2**53 + 1, 2**64 - 1]
    ns += [int(v) for v in r.integers(1, 2**62, 2000)]
    for n in ns:
        L = oracle.log2(n)
        exact = math.log2(n) if n < 2**53 else math.log2(n >> 11) + 11
        assert exact - 2**-22 < L <= exact + 1e-12, (n, L, exact)
    for e in range(64):
        assert oracle.log2(2**e) == e


@pytest.mark.parametrize("n,S", [(10**6, 1019), (10**8, 1360), (10**9, 1530)])
def test_paper_sample_size_vectors(n, S):
    # alpha*K - 1 with alpha = 0.2 log2(n) and K = 256, rounded (Proposed Algorithm chapter)
    assert oracle.sample_size(n, oracle.params(sample_policy=1)) == S


def test_paper_sample_size_rounding_and_bounds():
    import math
    for K in (4, 16, 256):
        p = oracle.params(K=K, sample_policy=1)
        for n in list(range(1, 3000)) + [10**k + 7 for k in range(4, 12)]:
            t = 0.2 * math.log2(n) * K - 1
            if abs(t - math.floor(t) - 0.5) < 1e-4:
                continue  # within the 24-bit logarithm's error of a rounding tie
            want = max(0, math.floor(t + 0.5)) if t - math.floor(t) != 0.5 else math.floor(t)
            want = min(want, (n + 1) // 2, n)
            assert oracle.sample_size(n, p) == want, (K, n)
    assert oracle.sample_size(10**8, oracle.params(sample_policy=1, sample_min=2000)) == 2000
    assert oracle.sample_size(10**8, oracle.params(sample_policy=1, sample_max=1000)) == 1000


@pytest.mark.parametrize("n,S,lo", [(5000, 512, 0), (10**6, 10**4, 123456), (997, 997, 5), (10**5, 1000, 7)])
def test_sample_positions_one_per_stratum(n, S, lo):
    pos = oracle.sample_positions(n, lo, S, 42)
    j = np.arange(S, dtype=object)
    start = np.array([(int(k) * n) // S for k in range(S)], np.int64)
    end = np.array([((int(k) + 1) * n) // S for k in range(S)], np.int64)
    assert np.all(pos.astype(np.int64) >= start) and np.all(pos.astype(np.int64) < end)
    assert np.array_equal(pos, oracle.sample_positions(n, lo, S, 42))
    if S < n:
        assert not np.array_equal(pos, oracle.sample_positions(n, lo, S, 43))


def test_sorted_sample_is_sorted_sample():
    k = gen.normal(20000, 5)
    S = 512
    x = oracle.sorted_sample(k, S, 9)
    pos = oracle.sample_positions(k.size, 0, S, 9)
    assert np.array_equal(x, np.sort(k[pos.astype(np.int64)]))


# ---------------------------------------------------------------- full sort vs brute force

def total_order_key(v: float):
    bits = struct.unpack("<Q", struct.pack("<d", v))[0]
    return bits ^ 0xFFFFFFFFFFFFFFFF if bits >> 63 else bits | (1 << 63)


CASES = [
    ("uniform01", 20000, dict()),
    ("normal", 30000, dict()),
    ("exponential", 30000, dict(K=16, T=64)),
    ("mixgauss", 30000, dict(K=8, T=32)),
    ("uniform_int", 30000, dict(K=32, T=100)),
    ("lognormal", 30000, dict(K=4, T=16)),
    ("chi_squared", 20000, dict(K=64, T=256)),
    ("root_dups", 20000, dict(K=16, T=50)),
    ("two_dups", 20000, dict(K=16, T=50)),
    ("lognormal2", 20000, dict(K=32, T=64)),
]


@pytest.mark.parametrize("dist,n,kw", CASES)
def test_sort_equals_numpy_sort(dist, n, kw):
    k = gen.make(dist, n, 17)
    out, _, st = oracle.sort(k, None, oracle.params(**kw))
    assert np.array_equal(out, np.sort(k))
    assert st["passes"] >= 1


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.uint64])
def test_sort_payload_is_stable(dtype):
    r = np.random.default_rng(5)
    if dtype == np.uint64:
        k = r.integers(0, 50, 6000).astype(np.uint64) * np.uint64(2**40)
    else:
        k = r.integers(-30, 30, 6000).astype(dtype) * dtype(0.5)
        k[::7] = -0.0
    pay = np.arange(k.size, dtype=np.uint32)
    out, pout, _ = oracle.sort(k, pay, oracle.params(K=8, T=40))
    if dtype == np.float64:
        want = sorted(range(k.size), key=lambda i: total_order_key(float(k[i])))
    else:
        o = oracle.ord_keys(k)  # order of a stable sort by ord, through Python's stable sorted()
        want = sorted(range(k.size), key=lambda i: int(o[i]))
    assert pout.tolist() == want
    assert np.array_equal(out.view(np.uint8), k[np.array(want)].view(np.uint8))


def test_sort_signed_zero_and_specials():
    k = np.concatenate([gen.special_f64(), np.zeros(50), -np.zeros(50), gen.normal(500, 1)])
    np.random.default_rng(0).shuffle(k)
    out, _, _ = oracle.sort(k, None, oracle.params(K=4, T=8))
    want = sorted(k.tolist(), key=total_order_key)
    assert [total_order_key(v) for v in out.tolist()] == [total_order_key(v) for v in want]


def test_all_equal_bucket_is_closed():
    k = np.full(10000, 3.25)
    pay = np.arange(10000, dtype=np.uint32)
    out, pout, st = oracle.sort(k, pay, oracle.params(K=16, T=100))
    assert st["closed"] == 1 and st["passes"] == 0
    assert np.array_equal(pout, pay)


def test_two_valued_and_u64_collisions_split_by_digit():
    # 50/50: the fit is capped but its spread is positive, so FMCD itself splits 7 from 9
    k = np.array([7.0, 9.0] * 5000)
    out, _, st = oracle.sort(k, None, oracle.params(K=16, T=100))
    assert np.array_equal(out, np.sort(k)) and st["passes"] == 1 and st["closed"] == 2
    # 95/5: once D passes the few 9s, u(D) = 0: degenerate fit, split by the digit of ord - min
    k = np.array([7.0] * 9500 + [9.0] * 500)
    np.random.default_rng(1).shuffle(k)
    out, _, st = oracle.sort(k, None, oracle.params(K=16, T=100))
    assert np.array_equal(out, np.sort(k)) and st["fallback"] == 1 and st["closed"] == 2
    # u64 keys above 2^53 that collapse to one fp64 value: the fit is degenerate, the digit splits
    u = (np.uint64(2**60) + np.random.default_rng(2).integers(0, 200, 20000).astype(np.uint64))
    out, _, st = oracle.sort(u, None, oracle.params(K=16, T=64))
    assert np.array_equal(out, np.sort(u)) and st["fallback"] >= 1


def msd_case(kind):
    r = np.random.default_rng(31)
    if kind == "u64_collide":
        # u64 keys above 2^53 that collapse to a single fp64 value
        return (np.uint64(2**60) + r.integers(0, 100, 20000).astype(np.uint64))
    if kind == "two_valued":
        k = np.array([7.0] * 9500 + [9.0] * 500)
        r.shuffle(k)
        return k
    # fp32, 95/5 two-valued: the sample's spread collapses as for fp64
    k = np.array([1.5] * 9500 + [2.75] * 500, np.float32)
    r.shuffle(k)
    return k


@pytest.mark.parametrize("kind", ["u64_collide", "two_valued", "f32_two_valued"])
@pytest.mark.parametrize("K", [16, 256])
def test_msd_digit_uses_the_top_log2K_bits(kind, K):
    # IPS2Ra's most-significant-digit split (IPS4o section): the digit is the top floor(log2 K)
    # bits of ord - min over the bucket's range, so the smallest key gets digit 0, the largest a
    # digit in [K/2, K-1] (its top bit is set), and no digit reaches K; a range below K/2 is split
    # by the offset itself.  A digit one bit narrower puts the largest key below K/2; one bit
    # wider overflows K.
    k = msd_case(kind)
    out, _, counts, m = oracle.partition(k, None, oracle.params(K=K, T=64))
    assert m.kind == oracle.MODEL_MSD
    assert int(counts.sum()) == k.size and counts.size == K
    nz = np.nonzero(counts)[0]
    assert nz[0] == 0
    ok = oracle.ord_keys(k)
    R = int(ok.max() - ok.min())
    if R >= K // 2:
        assert K // 2 <= nz[-1] <= K - 1
    else:
        # a range narrower than the digit: the digit is the offset itself, one bucket per value
        assert nz[-1] == R
        assert np.array_equal(counts, np.bincount((ok - ok.min()).astype(np.int64), minlength=K))
    # the largest key is in the last non-empty bucket, the smallest in bucket 0
    o = oracle.ord_keys(out)
    end = np.cumsum(counts.astype(np.int64))
    last = o[end[nz[-1]] - int(counts[nz[-1]]):end[nz[-1]]]
    assert oracle.ord_keys(k).max() in last and oracle.ord_keys(k).min() in o[:int(counts[0])]


def test_u64_and_f32_sorts():
    u = gen.u64_uniform(50000, 3)
    out, _, _ = oracle.sort(u, None, oracle.params(K=32, T=128))
    assert np.array_equal(out, np.sort(u))
    f = gen.normal(50000, 4).astype(np.float32)
    out, _, _ = oracle.sort(f, None, oracle.params(K=32, T=128))
    assert np.array_equal(out, np.sort(f))
    z = gen.zipf_u64(50000, 8)
    pay = np.arange(z.size, dtype=np.uint32)
    out, pout, st = oracle.sort(z, pay, oracle.params(K=64, T=256))
    assert np.array_equal(pout, np.argsort(z, kind="stable").astype(np.uint32))
    assert st["closed"] >= 1


def test_partition_invariants():
    k = gen.exponential(100000, 6)
    out, _, counts, m = oracle.partition(k, None, oracle.params())
    assert int(counts.sum()) == k.size and m.kind == oracle.MODEL_LINEAR
    # every bucket's keys precede the next bucket's keys; the layout is the stable one
    b = oracle.classify_model(k, m)
    assert np.array_equal(out, oracle.stable_layout(k, b, 256))
    edges = np.cumsum(counts.astype(np.int64))
    for c in range(255):
        lo, hi = (edges[c - 1] if c else 0), edges[c]
        if hi > lo and edges[c + 1] > hi:
            assert out[lo:hi].max() <= out[hi:edges[c + 1]].min()


def test_segmented_equals_per_segment():
    r = np.random.default_rng(9)
    sizes = gen.segment_sizes_lognormal(40, 1, median=2000, hi=50000)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = np.concatenate([gen.make(gen.CONFIG1_DISTS[i % 6], int(s), i) for i, s in enumerate(sizes)])
    out, _, _ = oracle.sort_segmented(keys, off, None, oracle.params(K=32, T=256))
    for s in range(len(sizes)):
        a, b = int(off[s]), int(off[s + 1])
        assert np.array_equal(out[a:b], np.sort(keys[a:b]))


def _bucket_rule(n, K, T):
    # the smallest power of two k >= 8n/T, kept within [min(K, 64), K]
    need = -(-8 * n // T)
    k = 1
    while k < need and k < K:
        k *= 2
    return min(max(k, min(K, 64)), K)


@pytest.mark.parametrize("K,T", [(256, 4096), (256, 256), (128, 4096), (48, 1024), (200, 4096)])
def test_bucket_policy_count(K, T):
    # a bucket of n keys is partitioned into the rule's number of buckets with the plain FMCD line;
    # every other configuration, and bucket_policy 0, keeps K
    for n in (T + 1, 2 * T, 8 * T - 1, 8 * T, 8 * T + 1, 32 * T, 32 * T + 1, 10**8):
        p = oracle.params(K=K, T=T)
        assert oracle.bucket_count(n, p) == _bucket_rule(n, K, T), (n, K, T)
        for other in (dict(bucket_policy=0), dict(model=1), dict(model=3), dict(equality=1), dict(inherit=1)):
            assert oracle.bucket_count(n, oracle.params(K=K, T=T, **other)) == K, (n, other)


@pytest.mark.parametrize("n", [5000, 20000, 150000])
def test_bucket_policy_fit_uses_the_bucket_count(n):
    # the fitted line maps onto the bucket's own count, and its sample's 2K minimum follows it
    keys = gen.make("exponential", n, 3)
    p = oracle.params()
    m, _, _ = oracle.fit_bucket(keys, p)
    Ki = _bucket_rule(n, 256, 4096)
    assert m.K == Ki
    assert m.S == min(n, max(2 * Ki, -(-n // 100)))
    out, _, _ = oracle.sort(keys, None, p)
    assert np.array_equal(out, np.sort(keys))
    m0, _, _ = oracle.fit_bucket(keys, oracle.params(bucket_policy=0))
    assert m0.K == 256
