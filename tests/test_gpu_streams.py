"""Stream ordering of the sort on a caller's stream, and the per-level profile records.

The top-level sort runs its base case on a second stream of the engine context.  The caller's
stream must still see the finished result: work queued on it after the call, with no host
synchronisation in between, reads the sorted keys.  Several sorts of different sizes go back to
back on one non-default stream; a torch reduction on that stream checks each result, and only
then does the host synchronise.
"""
import numpy as np
import pytest

import gen
import paper_2208_06902_amd as ipls

torch = pytest.importorskip("torch")
from gpu_util import dev  # noqa: E402

pytestmark = pytest.mark.gpu


def test_results_ordered_on_the_callers_stream():
    s1 = torch.cuda.Stream()
    sizes = [5_000_000, 300_000, 2_000_000, 70_001, 9_000_000]
    checks, wants = [], []
    with torch.cuda.stream(s1):
        for q, n in enumerate(sizes):
            keys = gen.make(("normal", "lognormal", "uniform_int", "exponential", "mixgauss")[q], n, 60 + q)
            print(f"stream case {q}: n={n}", flush=True)
            kd = torch.from_numpy(keys).to("cuda:0", non_blocking=False)
            ipls.sort_(kd, None, stream=s1)
            # queued on s1 right after the call: sortedness and a checksum of the bits
            ok = (kd[1:] >= kd[:-1]).all()
            chk = kd.view(torch.int64).sum()
            checks.append((ok, chk))
            wants.append(int(np.sort(keys).view(np.int64).sum(dtype=np.int64)))
    s1.synchronize()
    for (ok, chk), want in zip(checks, wants):
        assert bool(ok.item())
        assert int(chk.item()) == want


def test_segmented_many_small_and_large_on_a_stream():
    # many segments go straight to the base case at the first level, beside the large segments'
    # partition
    s1 = torch.cuda.Stream()
    r = np.random.default_rng(3)
    sizes = np.where(r.random(3000) < 0.97, r.integers(2, 4096, 3000), r.integers(50_000, 400_000, 3000))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = r.standard_normal(int(off[-1]))
    print(f"segmented stream case: nseg={sizes.size} total={keys.size}", flush=True)
    with torch.cuda.stream(s1):
        kd = torch.from_numpy(keys).to("cuda:0")
        od = torch.from_numpy(off.view(np.int64)).to("cuda:0").view(torch.uint64)
        ipls.sort_segmented_(kd, od, stream=s1)
        got = kd.to("cpu", non_blocking=False)
    s1.synchronize()
    want = np.concatenate([np.sort(keys[off[i]:off[i + 1]]) for i in range(sizes.size)])
    assert np.array_equal(got.numpy().view(np.uint64), want.view(np.uint64))


def test_profile_records_per_level_add_up_to_the_totals():
    # the per-level figures of each profiled kernel sum to its totals; the counting and scatter
    # bytes of a level are w and 2w per key of the level's items
    k = gen.make("normal", 2_000_000, 41)
    print("profile per level: 2e6 normal", flush=True)
    kd = dev(k)
    ipls.profile_enable(True)
    st = ipls.sort_(kd, None, ipls.default_params(sample_max=4096), stats=True)
    torch.cuda.synchronize()
    for kern in (ipls.KERNEL_SCATTER, ipls.KERNEL_CLASSIFY, ipls.KERNEL_BASE):
        n, ms, by = ipls.profile_read(kern)
        per = [ipls.profile_read_level(kern, lv) for lv in range(16)]
        assert n == sum(p[0] for p in per) and n > 0
        assert abs(by - sum(p[2] for p in per)) <= 1e-6 * by
        assert abs(ms - sum(p[1] for p in per)) <= 1e-6 * max(ms, 1e-9)
    n0, _, b0 = ipls.profile_read_level(ipls.KERNEL_SCATTER, 0)
    c0 = ipls.profile_read_level(ipls.KERNEL_CLASSIFY, 0)[2]
    assert n0 == 1 and b0 == 2 * 8 * k.size and c0 == 8 * k.size
    assert ipls.profile_read_level(ipls.KERNEL_SCATTER, st["levels"])[0] == 0
    ipls.profile_enable(False)
