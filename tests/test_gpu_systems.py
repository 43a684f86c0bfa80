"""The batched and served forms on the GPU.

* Autotuner: the parameters it picks are valid and the segmented sort under them equals the
  oracle.
* Request server: requests of mixed sizes, dtypes and distributions, some with payloads, are
  admitted under a small HBM budget (so some must wait for memory), run concurrently on several
  lanes and in batches; every result is bit-identical to the same request sorted alone, and to
  the oracle.
"""
import numpy as np
import pytest

import gen
import oracle
import paper_2208_06902_amd as ipls

torch = pytest.importorskip("torch")
from gpu_util import dev, host, same_bits  # noqa: E402

pytestmark = pytest.mark.gpu

NP_DT = {ipls.F64: np.float64, ipls.F32: np.float32, ipls.U64: np.uint64}


def oracle_params_of(p):
    return oracle.params(K=p.num_buckets, T=p.base_case_max, divisor=p.sample_divisor, sample_min=p.sample_min,
                         sample_max=p.sample_max, seed=p.seed, model=p.model, leaves=p.leaves,
                         train_iters=p.train_iters, sample_policy=p.sample_policy)


def test_autotuned_segmented_sort_matches_oracle():
    sizes = gen.segment_sizes_lognormal(3000, 4, median=4096, lo=64, hi=2_000_000)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = np.concatenate([gen.make(gen.CONFIG1_DISTS[i % 6], int(s), 100 + i) for i, s in enumerate(sizes)])
    print(f"autotune nseg={sizes.size} total={keys.size}", flush=True)
    kd, od = dev(keys), dev(off)
    p, rep = ipls.autotune_segmented(kd, od)
    torch.cuda.synchronize()
    print("tuned", p.num_buckets, p.base_case_max, p.tile_keys, rep, flush=True)
    assert p.num_buckets in (64, 128, 256) and p.base_case_max in (1024, 2048, 4096)
    assert p.tile_keys in (0, 2048, 4096)
    assert rep["trials"] >= 4 and rep["best_ms"] <= rep["default_ms"]
    assert same_bits(host(kd, keys.dtype), keys)  # the tuner works on a private copy
    ipls.sort_segmented_(kd, od, params=p)
    torch.cuda.synchronize()
    want, _, _ = oracle.sort_segmented(keys, off, None, oracle_params_of(p))
    assert same_bits(host(kd, keys.dtype), want)


def _request_inputs(count, seed, max_n):
    r = np.random.default_rng(seed)
    dists = ["lognormal2", "mixgauss20", "normal", "exponential", "uniform_int"]
    reqs = []
    for i in range(count):
        n = int(round(10 ** r.uniform(3, np.log10(max_n))))
        u = r.random()
        dt = ipls.F64 if u < 0.5 else (ipls.U64 if u < 0.8 else ipls.F32)
        x = gen.as_dtype(gen.make(dists[i % len(dists)], n, 1000 + i), dt)
        pay = gen.index_payload(n) if i % 3 == 0 else None
        reqs.append((dt, x, pay))
    return reqs


def _fill(view, a):
    if a.dtype == np.uint64:
        view.view(torch.int64).copy_(torch.from_numpy(a.view(np.int64)))
    elif a.dtype == np.uint32:
        view.copy_(torch.from_numpy(a.view(np.int32)))
    else:
        view.copy_(torch.from_numpy(a))


def _read(view, like):
    if like == np.uint64:
        return view.view(torch.int64).cpu().numpy().view(np.uint64)
    if like == np.uint32:
        return view.cpu().numpy().view(np.uint32)
    return view.cpu().numpy()


def _serve_all(srv, reqs):
    """Admit, fill and submit every request (waiting for memory when the budget is full)."""
    out = {}
    pending = []  # (req_id, index) in submission order

    def drain_one():
        rid, i = pending.pop(0)
        info = srv.wait(rid)
        out[i] = (_read(views[rid][0], reqs[i][1].dtype),
                  None if views[rid][1] is None else _read(views[rid][1], np.uint32), info)
        srv.release(rid)

    views = {}
    waited = 0
    for i, (dt, x, pay) in enumerate(reqs):
        while True:
            got = srv.reserve(x.size, dt, pay is not None)
            if got is not None:
                break
            waited += 1
            drain_one()
        rid, kv, pv = got
        _fill(kv, x)
        if pay is not None:
            _fill(pv, pay)
        srv.submit(rid)
        views[rid] = (kv, pv)
        pending.append((rid, i))
    while pending:
        drain_one()
    return out, waited


@pytest.mark.parametrize("model", [0, 1])
def test_server_results_equal_alone_and_oracle(model):
    reqs = _request_inputs(48, 5 + model, 2_000_000)
    total = sum(x.size * x.itemsize * 2 + (0 if p is None else 8 * p.size) for _, x, p in reqs)
    params = ipls.default_params(model=model)
    cfg = ipls.server_config(params, lanes=3, batch_max_keys=1 << 16, batch_keys=1 << 20)
    # a budget of a third of the total: some requests must wait for memory
    budget = max(total // 3, 64 << 20)
    print(f"server model={model} requests={len(reqs)} total_bytes={total} budget={budget}", flush=True)
    arena = torch.empty(budget, dtype=torch.uint8, device="cuda:0")
    with ipls.Server(arena, cfg) as srv:
        out, waited = _serve_all(srv, reqs)
        st = srv.stats()
    print("server stats", st, "waited", waited, flush=True)
    assert st["completed"] == len(reqs) and st["batches_run"] >= 1 and st["singles_run"] >= 1
    assert waited > 0 and st["rejected"] > 0
    for i, (dt, x, pay) in enumerate(reqs):
        got, gpay, info = out[i]
        assert info["status"] == 0 and info["t_done"] >= info["t_start"] >= info["t_submit"]
        # alone: the same request through the plain entry point
        kd = dev(x)
        pd = None if pay is None else dev(pay)
        ipls.sort_(kd, pd, params=params)
        torch.cuda.synchronize()
        assert same_bits(got, host(kd, x.dtype)), i
        if pay is not None:
            assert np.array_equal(gpay, host(pd, np.uint32)), i
        want, wpay, _ = oracle.sort(x, pay, oracle_params_of(params))
        assert same_bits(got, want), i
        if pay is not None:
            assert np.array_equal(gpay, wpay), i


def test_server_wait_before_the_rest_of_a_batch_is_submitted():
    # reserve three small requests (one batch), submit only the first, wait on it: the lane takes
    # the submitted slot alone; the others run once submitted, and every result is its own sort
    cfg = ipls.server_config(ipls.default_params(), lanes=1, batch_max_keys=1 << 16, batch_keys=1 << 18)
    xs = [gen.make("normal", n, 70 + i) for i, n in enumerate((5000, 3000, 7000))]
    arena = torch.empty(64 << 20, dtype=torch.uint8, device="cuda:0")
    print("server partial batch", [x.size for x in xs], flush=True)
    with ipls.Server(arena, cfg) as srv:
        got = [srv.reserve(x.size, ipls.F64) for x in xs]
        for (rid, kv, _), x in zip(got, xs):
            _fill(kv, x)
        srv.submit(got[0][0])
        i0 = srv.wait(got[0][0])
        assert i0["status"] == 0 and i0["batch_size"] == 1
        srv.submit(got[2][0])
        srv.submit(got[1][0])
        i1, i2 = srv.wait(got[1][0]), srv.wait(got[2][0])
        assert i1["status"] == 0 and i2["status"] == 0
        for (rid, kv, _), x in zip(got, xs):
            want, _, _ = oracle.sort(x, None, oracle.params())
            assert same_bits(_read(kv, np.float64), want)
            srv.release(rid)
