"""GPU parity of the two-level piecewise-linear CDF model against the CPU oracle (bit for bit),
its use inside the sort, and what it gains over FMCD on skewed inputs."""
import numpy as np
import pytest

import gen
import oracle
import paper_2208_06902_amd as ipls

torch = pytest.importorskip("torch")
from gpu_util import dev, host, same_bits  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dist,S,K,M", [("lognormal2", 20000, 256, 256), ("mixgauss20", 4096, 256, 256),
                                        ("normal", 50000, 64, 128), ("exponential", 3000, 256, 32),
                                        ("uniform_int", 20000, 256, 256)])
def test_l2pl_train_matches_oracle(dist, S, K, M):
    x = np.sort(gen.make(dist, S, 3))
    print(f"l2pl train {dist} S={S} K={K} M={M}", flush=True)
    root, leaf, ab = ipls.l2pl_train(dev(x), K, M, 32)
    torch.cuda.synchronize()
    want = oracle.l2pl_train(x, K, M, 32)
    assert want is not None
    assert same_bits(host(root, np.float64), want[0])
    assert same_bits(host(leaf, np.float64), want[1])
    assert same_bits(host(ab, np.float64), want[2])


@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20", "exponential"])
def test_l2pl_gradient_matches_oracle(dist):
    K, M = 256, 256
    x = np.sort(gen.make(dist, 8000, 4))
    ab = np.random.default_rng(5).standard_normal(2 * M) * 4
    g, loss = ipls.l2pl_grad(dev(x), K, M, dev(ab))
    torch.cuda.synchronize()
    a, b, _ = oracle.fmcd(x, M)
    first, c, h, m2 = oracle.l2pl_geometry(x, M, a, b)
    og, ol = oracle.l2pl_grad(x, K, M, first, c, h, ab)
    assert same_bits(host(g, np.float64), og)
    assert same_bits(host(loss, np.float64), ol)


def test_l2pl_degenerate_root_is_reported():
    x = np.full(5000, 2.0)
    with pytest.raises(ipls.IplsError):
        ipls.l2pl_train(dev(x), 256, 256, 8)


def _sort_both(keys, **kw):
    p = ipls.default_params(**kw)
    k = dev(keys)
    st = ipls.sort_(k, None, params=p, stats=True)
    torch.cuda.synchronize()
    op = oracle.params(K=p.num_buckets, T=p.base_case_max, model=p.model, leaves=p.leaves,
                       train_iters=p.train_iters, sample_max=p.sample_max)
    want, _, ost = oracle.sort(keys, None, op)
    return host(k, keys.dtype), st, want, ost


@pytest.mark.parametrize("model", [ipls.MODEL_AUTO, ipls.MODEL_L2PL])
@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20", "normal", "uniform_int", "exponential"])
def test_sort_with_learned_model_matches_oracle(model, dist):
    keys = gen.make(dist, 400_001, 6)
    print(f"sort learned model={model} {dist}", flush=True)
    got, st, want, ost = _sort_both(keys, model=model)
    assert same_bits(got, want)
    assert (st["passes"], st["levels"], st["l2pl_used"]) == (ost["passes"], ost["max_level"], ost["l2pl_used"])


def test_learned_model_with_payload_and_f32():
    k = gen.make("lognormal2", 300_000, 7).astype(np.float32)
    pay = gen.index_payload(k.size)
    kd, pd = dev(k), dev(pay)
    ipls.sort_(kd, pd, params=ipls.default_params(model=ipls.MODEL_AUTO, num_buckets=128, leaves=64))
    torch.cuda.synchronize()
    want, wpay, _ = oracle.sort(k, pay, oracle.params(K=128, model=1, leaves=64))
    assert same_bits(host(kd, np.float32), want) and np.array_equal(host(pd, np.uint32), wpay)


@pytest.mark.parametrize("dist", ["lognormal2", "mixgauss20"])
def test_learned_model_gain(dist):
    """The two-level model lowers the first level's largest bucket (the conflict degree that bounds
    the recursion) and needs no more levels than FMCD alone, on the skewed inputs of the served
    workload."""
    keys = gen.make(dist, 4_000_000, 9)
    res = {}
    for model in (ipls.MODEL_FMCD, ipls.MODEL_AUTO):
        got, st, want, ost = _sort_both(keys, model=model)
        assert same_bits(got, want)
        res[model] = st
    fm, l2 = res[ipls.MODEL_FMCD], res[ipls.MODEL_AUTO]
    print(f"{dist}: FMCD {fm} | two-level {l2}", flush=True)
    assert l2["l2pl_used"] >= 1
    assert l2["level1_max_load"] < fm["level1_max_load"]
    assert l2["levels"] <= fm["levels"]
