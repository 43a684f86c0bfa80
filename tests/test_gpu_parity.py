"""GPU parity: the HIP library, called through its C ABI, against the CPU oracle, bit for bit.

Sizes are small enough for the oracle to finish in seconds yet span many tiles, several levels
and ragged tails.  Every case prints its name before it touches the GPU.
"""
import numpy as np
import pytest

import gen
import oracle
import paper_2208_06902_amd as ipls

torch = pytest.importorskip("torch")
from gpu_util import dev, host, same_bits  # noqa: E402

pytestmark = pytest.mark.gpu


def gpu_sort(keys, payload=None, **kw):
    p = ipls.default_params(**kw) if kw else None
    k = dev(keys)
    pl = None if payload is None else dev(payload)
    st = ipls.sort_(k, pl, params=p, stats=True)
    torch.cuda.synchronize()
    return host(k, keys.dtype), (None if pl is None else host(pl, np.uint32)), st


def oracle_params(**kw):
    m = dict(K=kw.get("num_buckets", 256), T=kw.get("base_case_max", 4096), divisor=kw.get("sample_divisor", 100),
             sample_min=kw.get("sample_min", 0), sample_max=kw.get("sample_max", 0),
             model=kw.get("model", 0), leaves=kw.get("leaves", 256), train_iters=kw.get("train_iters", 4),
             sample_policy=kw.get("sample_policy", 0), equality=kw.get("equality", 0),
             bucket_policy=kw.get("bucket_policy", 1))
    return oracle.params(**m)


def check_sort(keys, payload=None, **kw):
    print(f"case n={keys.size} dtype={keys.dtype} payload={payload is not None} params={kw}", flush=True)
    got, gpay, st = gpu_sort(keys, payload, **kw)
    want, wpay, ost = oracle.sort(keys, payload, oracle_params(**kw))
    assert same_bits(got, want)
    if payload is not None:
        assert np.array_equal(gpay, wpay)
    assert st["passes"] == ost["passes"], (st, ost)
    assert st["levels"] == ost["max_level"], (st, ost)
    assert st["level1_max_load"] == ost["level1_max_load"], (st, ost)
    return st


DISTS = ["uniform01", "normal", "lognormal", "exponential", "mixgauss", "uniform_int", "chi_squared", "root_dups",
         "two_dups", "lognormal2", "mixgauss20"]


@pytest.mark.parametrize("dist", DISTS)
def test_sort_f64_default_params(dist):
    check_sort(gen.make(dist, 300_001, 21))


@pytest.mark.parametrize("dist", ["normal", "exponential", "uniform_int", "two_dups"])
@pytest.mark.parametrize("kw", [dict(num_buckets=16, base_case_max=64), dict(num_buckets=64, base_case_max=200),
                                dict(num_buckets=4, base_case_max=8, sample_min=8),
                                dict(num_buckets=256, base_case_max=1000, sample_divisor=7),
                                dict(tile_keys=2048), dict(tile_keys=2048, num_buckets=64, base_case_max=1024),
                                dict(bucket_policy=0), dict(bucket_policy=0, num_buckets=64, base_case_max=200),
                                dict(num_buckets=200, base_case_max=1000)])
def test_sort_f64_params(dist, kw):
    check_sort(gen.make(dist, 50_000, 5), **kw)


@pytest.mark.parametrize("dist", ["normal", "exponential", "two_dups", "zipf_u64"])
@pytest.mark.parametrize("kw", [dict(sample_policy=1), dict(sample_policy=1, num_buckets=16, base_case_max=64),
                                dict(sample_policy=1, num_buckets=64, base_case_max=32, sample_min=20)])
def test_sort_paper_sample_policy(dist, kw):
    k = gen.make(dist, 250_000, 17)
    check_sort(k, gen.index_payload(k.size), **kw)


@pytest.mark.parametrize("dist", ["zipf_u64", "root_dups", "two_dups", "uniform_int", "normal", "mixgauss"])
@pytest.mark.parametrize("kw", [dict(equality=1), dict(equality=1, num_buckets=16, base_case_max=64),
                                dict(equality=1, num_buckets=64, base_case_max=300, tile_keys=2048)])
def test_sort_equality_buckets(dist, kw):
    k = gen.make(dist, 220_000, 23)
    check_sort(k, gen.index_payload(k.size), **kw)


def test_equality_buckets_f32_and_heavy_specials():
    r = np.random.default_rng(5)
    k = r.standard_normal(150_000).astype(np.float32)
    k[::3] = np.float32(0.5)
    k[1::7] = -np.float32(0.0)
    k[2::11] = np.float32(np.inf)
    check_sort(k, gen.index_payload(k.size), equality=1, num_buckets=32, base_case_max=128)
    u = np.concatenate([gen.u64_uniform(50_000, 3), np.full(40_000, 2**63, np.uint64), np.full(30_000, 7, np.uint64)])
    r.shuffle(u)
    check_sort(u, None, equality=1, num_buckets=64, base_case_max=256)


@pytest.mark.parametrize("dist", ["normal", "lognormal2", "zipf_u64", "root_dups", "uniform_int"])
@pytest.mark.parametrize("kw", [dict(model=3), dict(model=3, num_buckets=37, base_case_max=200),
                                dict(model=3, num_buckets=64, base_case_max=1000, tile_keys=2048)])
def test_sort_splitter_tree(dist, kw):
    k = gen.make(dist, 200_000, 29)
    check_sort(k, gen.index_payload(k.size), **kw)


def test_splitter_tree_f32_specials():
    r = np.random.default_rng(8)
    k = r.standard_normal(120_000).astype(np.float32)
    k[::5] = np.float32(np.nan)
    k[1::13] = -np.float32(0.0)
    check_sort(k, None, model=3, num_buckets=16, base_case_max=64)


def test_sort_u64_uniform_and_zipf_payload():
    check_sort(gen.u64_uniform(400_000, 7))
    z = gen.zipf_u64(300_000, 8)
    st = check_sort(z, gen.index_payload(z.size))
    assert st["levels"] >= 2


@pytest.mark.parametrize("dist", ["normal", "lognormal2", "uniform_int"])
def test_sort_f32_with_payload(dist):
    k = gen.make(dist, 200_000, 9).astype(np.float32)
    check_sort(k, gen.index_payload(k.size), num_buckets=64, base_case_max=512)
    check_sort(k, gen.index_payload(k.size), tile_keys=2048)


def test_payload_stability_heavy_duplicates():
    r = np.random.default_rng(3)
    k = r.integers(0, 40, 120_000).astype(np.float64)
    k[::5] = -0.0
    k[1::5] = 0.0
    check_sort(k, gen.index_payload(k.size), num_buckets=32, base_case_max=256)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4095, 4096, 4097, 8192 + 7, 65_537])
def test_sizes_around_tiles_and_base_case(n):
    k = gen.normal(n, 31)
    got, _, _ = gpu_sort(k)
    assert same_bits(got, oracle.sort(k)[0]) if n else got.size == 0


def test_back_to_back_sorts_of_changing_sizes():
    # each call's segment offsets [0, n] must be its own: sorts of changing sizes issued back to
    # back (some with payloads, some on a second stream), every result checked
    r = np.random.default_rng(77)
    side = torch.cuda.Stream()
    cases = []
    for c in range(40):
        n = int(r.integers(2, 300_000)) if c % 4 else int(r.integers(4097, 20_000))
        k = gen.make(["normal", "exponential", "uniform_int", "lognormal2"][c % 4], n, 500 + c)
        pay = gen.index_payload(n) if c % 3 == 0 else None
        cases.append((k, pay))
    print(f"back to back: {len(cases)} sorts", flush=True)
    outs = []
    for c, (k, pay) in enumerate(cases):
        kd = dev(k)
        pd = None if pay is None else dev(pay)
        if c % 5 == 4:
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                ipls.sort_(kd, pd)
            torch.cuda.current_stream().wait_stream(side)
        else:
            ipls.sort_(kd, pd)
        outs.append((kd, pd))
    torch.cuda.synchronize()
    for (k, pay), (kd, pd) in zip(cases, outs):
        order = np.argsort(k, kind="stable")
        assert same_bits(host(kd, k.dtype), k[order])
        if pay is not None:
            assert np.array_equal(host(pd, np.uint32), pay[order])


def test_all_equal_and_two_valued():
    k = np.full(100_000, 2.5)
    st = check_sort(k, gen.index_payload(k.size))
    assert st["passes"] == 0
    k = np.array([7.0] * 95_000 + [9.0] * 5_000)
    np.random.default_rng(1).shuffle(k)
    check_sort(k, gen.index_payload(k.size), num_buckets=16, base_case_max=100)


def test_special_values_and_nans():
    neg_nan = np.array([0xFFF8000000000001], np.uint64).view(np.float64)[0]
    pos_nan = np.array([0x7FF8000000000002], np.uint64).view(np.float64)[0]
    base = gen.normal(20_000, 2)
    k = np.concatenate([base, np.repeat(gen.special_f64(), 300), [neg_nan] * 50, [pos_nan] * 50])
    np.random.default_rng(4).shuffle(k)
    check_sort(k, gen.index_payload(k.size), num_buckets=32, base_case_max=128)
    u = np.concatenate([gen.u64_uniform(30_000, 1), np.array([0, 1, 2**53, 2**53 + 1, 2**64 - 1] * 100, np.uint64),
                        np.uint64(2**60) + np.arange(5000, dtype=np.uint64)])
    check_sort(u, None, num_buckets=16, base_case_max=64)


def test_worked_example():
    import json, os
    with open(os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")) as f:
        w = json.load(f)
    k = np.array(w["input"], np.float64)
    got, _, _ = gpu_sort(k, num_buckets=w["k"], base_case_max=w["base_case_below"] - 1, sample_min=8)
    assert got.tolist() == w["sorted"]


def test_config1_full_size():
    k = gen.uniform01(1_000_000, 1)
    check_sort(k)


# ---------------------------------------------------------------- intermediate states

@pytest.mark.parametrize("dist,dtype", [("normal", np.float64), ("exponential", np.float64),
                                        ("u64_uniform", np.uint64), ("lognormal2", np.float32),
                                        ("uniform_int", np.float64)])
def test_first_level_partition_parity(dist, dtype):
    k = gen.make(dist, 700_003, 13)
    k = k.astype(dtype) if dtype != np.uint64 else k
    pay = gen.index_payload(k.size)
    print(f"partition {dist} {dtype}", flush=True)
    kd, pd = dev(k), dev(pay)
    counts, (a, b, D, degen) = ipls.partition_(kd, pd)
    torch.cuda.synchronize()
    want, wpay, wcounts, m = oracle.partition(k, pay, oracle.params())
    assert (a, b, D) == (m.a, m.b, m.D) and degen == 0
    assert np.array_equal(host(counts, np.uint64), wcounts)
    assert same_bits(host(kd, k.dtype), want)
    assert np.array_equal(host(pd, np.uint32), wpay)


@pytest.mark.parametrize("dist,n,smax", [("normal", 700_003, 4096), ("lognormal2", 300_001, 1000),
                                         ("uniform_int", 250_000, 4096), ("two_dups", 90_001, 700),
                                         ("mixgauss", 6_000, 0)])
def test_first_level_partition_capped_samples(dist, n, smax):
    # samples of at most 4096 keys are gathered, sorted and fitted by one launch: the same line
    # and the same partition as the oracle's
    k = gen.make(dist, n, 29)
    pay = gen.index_payload(k.size)
    print(f"partition {dist} n={n} sample_max={smax}", flush=True)
    kd, pd = dev(k), dev(pay)
    counts, (a, b, D, degen) = ipls.partition_(kd, pd, ipls.default_params(sample_max=smax))
    torch.cuda.synchronize()
    want, wpay, wcounts, m = oracle.partition(k, pay, oracle.params(sample_max=smax))
    assert degen == 0 and m.degenerate == 0
    assert (a, b, D) == (m.a, m.b, m.D)
    assert np.array_equal(host(counts, np.uint64), wcounts)
    assert same_bits(host(kd, k.dtype), want)
    assert np.array_equal(host(pd, np.uint32), wpay)


@pytest.mark.parametrize("S", [3, 5, 100, 511, 8192, 16384, 16385, 20_000, 100_003, 1_000_000])
@pytest.mark.parametrize("K", [4, 37, 256])
def test_fmcd_fit_parity(S, K):
    x = np.sort(gen.lognormal(S, S + K))
    print(f"fit S={S} K={K}", flush=True)
    a, b, D, degen = ipls.fit_model(dev(x), K)
    want = oracle.fmcd(x, K)
    assert (a, b, D) == want
    usable = want[0] > 0 and np.isfinite(want[0]) and np.isfinite(want[1])
    assert degen == (0 if usable else 1)


def test_fmcd_fit_unsorted_and_degenerate():
    x = gen.normal(50_000, 3)
    a, b, D, _ = ipls.fit_model(dev(x), 256, sorted_=False)
    assert (a, b, D) == oracle.fmcd(np.sort(x), 256)
    _, _, _, degen = ipls.fit_model(dev(np.full(1000, 3.0)), 256)
    assert degen == 1
    u = np.sort(gen.u64_uniform(30_000, 2))
    assert ipls.fit_model(dev(u), 128)[:3] == oracle.fmcd(oracle.val_keys(u), 128)


def test_fmcd_fit_duplicate_heavy_samples():
    r = np.random.default_rng(8)
    for t in range(20):
        S = int(r.integers(3, 30_000))
        x = np.sort(r.integers(0, int(r.integers(2, 50)), S).astype(np.float64))
        got = ipls.fit_model(dev(x), 64)
        want = oracle.fmcd(x, 64)
        if got[3]:
            assert not (want[0] > 0 and np.isfinite(want[0]) and np.isfinite(want[1]))
        else:
            assert got[:3] == want


# ---------------------------------------------------------------- segmented

@pytest.mark.parametrize("nseg,seed", [(1, 1), (37, 2), (2000, 3)])
def test_segmented_matches_oracle(nseg, seed):
    sizes = gen.segment_sizes_lognormal(nseg, seed, median=3000, lo=0, hi=300_000)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = np.concatenate([gen.make(gen.CONFIG1_DISTS[i % 6], int(s), i) for i, s in enumerate(sizes)])
    pay = gen.index_payload(keys.size)
    print(f"segmented nseg={nseg} total={keys.size}", flush=True)
    kd, pd = dev(keys), dev(pay)
    ipls.sort_segmented_(kd, dev(off), pd)
    torch.cuda.synchronize()
    want, wpay, _ = oracle.sort_segmented(keys, off, pay, oracle.params())
    assert same_bits(host(kd, keys.dtype), want)
    assert np.array_equal(host(pd, np.uint32), wpay)


def test_segmented_many_items():
    # 5000 segments above T: a first level of 5000 items (several rounds of the plan kernel's
    # eight-items-a-thread scan), every sample of 2K keys (the 8 KB fit)
    r = np.random.default_rng(21)
    sizes = r.integers(4097, 9000, 5000)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = r.standard_normal(int(off[-1])) * r.choice([1e-3, 1.0, 1e3], int(off[-1]))
    pay = gen.index_payload(keys.size)
    print(f"segmented many items nseg={sizes.size} total={keys.size}", flush=True)
    kd, pd = dev(keys), dev(pay)
    st = ipls.sort_segmented_(kd, dev(off), pd, stats=True)
    torch.cuda.synchronize()
    want, wpay, ost = oracle.sort_segmented(keys, off, pay, oracle.params())
    assert same_bits(host(kd, keys.dtype), want)
    assert np.array_equal(host(pd, np.uint32), wpay)
    assert (st["passes"], st["levels"]) == (ost["passes"], ost["max_level"]), (st, ost)


def test_decreasing_segment_offsets_set_the_device_error_word():
    # the offsets check runs on the device (the library never reads the offsets on the host): a
    # segment whose end is below its start sets the error word, no kernel writes a key, the call
    # returns IPLS_ERR_DEVICE and ipls_stream_status reports it; the same context then sorts a
    # valid batch exactly as the oracle does
    import ctypes as C

    keys = gen.make("normal", 20_000, 33)
    off = np.array([0, 5000, 3000, 20_000], dtype=np.uint64)
    print(f"case decreasing offsets {off.tolist()}", flush=True)
    kd, od = dev(keys), dev(off)
    stream = torch.cuda.current_stream()
    lib = ipls.load()
    rc = lib.ipls_sort_segmented(C.c_void_p(kd.data_ptr()), None, C.c_void_p(od.data_ptr()), off.size - 1,
                                 ipls.F64, None, None, C.c_void_p(stream.cuda_stream))
    torch.cuda.synchronize()
    assert rc == 5  # IPLS_ERR_DEVICE
    assert lib.ipls_stream_status(C.c_void_p(stream.cuda_stream)) == 5
    assert same_bits(host(kd, keys.dtype), keys)  # nothing was moved
    good = np.array([0, 3000, 5000, 20_000], dtype=np.uint64)
    od = dev(good)
    ipls.sort_segmented_(kd, od)
    torch.cuda.synchronize()
    assert lib.ipls_stream_status(C.c_void_p(stream.cuda_stream)) == 0
    want, _, _ = oracle.sort_segmented(keys, good, None, oracle_params())
    assert same_bits(host(kd, keys.dtype), want)
