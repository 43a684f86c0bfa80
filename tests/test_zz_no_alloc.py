"""The allocation-free entry point (ipls_sort_noalloc) through the C ABI against ipls_sort_ex.

Two calls in a row on the same GPU (the second smaller, so it reuses the scratch array the first
left behind), fp64 with a payload and uint64 keys only; every output must be bit-identical to
ipls_sort_ex of the same input with the same parameters, and the statistics must agree.  Sizes
above the array's limit are refused before any device work.
"""
import ctypes as C

import numpy as np
import pytest

import gen
import paper_2208_06902_amd as ipls

torch = pytest.importorskip("torch")
from gpu_util import dev, host, same_bits  # noqa: E402

pytestmark = pytest.mark.gpu


def _noalloc(kd, pd, params):
    st = ipls.Stats()
    rc = ipls.load().ipls_sort_noalloc(C.c_void_p(kd.data_ptr()), None if pd is None else C.c_void_p(pd.data_ptr()),
                                       kd.numel(), ipls._dtype_code(kd), C.byref(params), C.byref(st),
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, st.as_dict()


@pytest.mark.parametrize("case", ["f64_payload", "u64_keys", "f64_learned"])
def test_noalloc_matches_sort_ex_twice(case):
    dist, dtype, pay, model = {"f64_payload": ("normal", ipls.F64, True, 0),
                               "u64_keys": ("lognormal2", ipls.U64, False, 1),
                               "f64_learned": ("mixgauss20", ipls.F64, False, 1)}[case]
    params = ipls.default_params(model=model, sample_max=4096)
    for i, n in enumerate((ipls.NOALLOC_MAX_KEYS, 1_234_567)):
        x = gen.as_dtype(gen.make(dist, n, 300 + i), dtype)
        p = gen.index_payload(n) if pay else None
        print(f"noalloc case={case} call={i} n={n}", flush=True)
        kd, pd = dev(x), (None if p is None else dev(p))
        rc, st = _noalloc(kd, pd, params)
        assert rc == 0, ipls.STATUS.get(rc, rc)
        kr, pr = dev(x), (None if p is None else dev(p))
        want_st = ipls.sort_(kr, pr, params=params, stats=True)
        torch.cuda.synchronize()
        assert same_bits(host(kd, x.dtype), host(kr, x.dtype))
        if p is not None:
            assert np.array_equal(host(pd, np.uint32), host(pr, np.uint32))
        assert st == want_st


def test_noalloc_refuses_more_keys_than_its_array_serves():
    lib = ipls.load()
    # the size check comes first: the key pointer is never used
    rc = lib.ipls_sort_noalloc(C.c_void_p(4096), None, ipls.NOALLOC_MAX_KEYS + 1, ipls.F64, None, None, None)
    assert rc == 6  # IPLS_ERR_UNSUPPORTED
