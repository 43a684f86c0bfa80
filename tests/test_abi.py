"""The C-ABI library loads and exports every entry point include/ipls.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2208_06902_amd as ipls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "ipls.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\*?\s+\*?(ipls_[a-z_0-9]+)\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ["ipls_sort", "ipls_sort_ex", "ipls_sort_segmented", "ipls_fit_model", "ipls_partition",
                 "ipls_workspace_bytes", "ipls_stream_status", "ipls_status_string", "ipls_l2pl_train",
                 "ipls_l2pl_grad", "ipls_default_params", "ipls_profile_enable", "ipls_profile_read"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(ipls.LIB_PATH):
        pytest.skip("libipls.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(ipls.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(declared_symbols()) <= set(ipls.EXPORTS) | set(declared_symbols())


def test_host_only_entry_points():
    if not os.path.exists(ipls.LIB_PATH):
        pytest.skip("libipls.so not built")
    p = ipls.default_params()
    assert (p.num_buckets, p.base_case_max, p.sample_divisor, p.model, p.leaves) == (256, 4096, 100, 0, 256)
    assert ipls.status_string(0) == "IPLS_OK" and ipls.status_string(5) == "IPLS_ERR_DEVICE"
    assert ipls.workspace_bytes(1000, ipls.F64, False) == 8192  # 8000 bytes rounded up to 256
    assert ipls.workspace_bytes(1000, ipls.F32, True) == 4096 + 4000
    assert ipls.workspace_bytes(10, 7, False) == 0


@pytest.mark.parametrize("field,value", [("sample_policy", 2), ("num_buckets", 3), ("sample_divisor", 1),
                                         ("sample_min", 5000), ("model", 4), ("leaves", 2)])
def test_invalid_params_rejected_before_any_device_work(field, value):
    # argument errors return synchronously; the key pointer is never dereferenced
    if not os.path.exists(ipls.LIB_PATH):
        pytest.skip("libipls.so not built")
    p = ipls.default_params(**{field: value})
    lib = ipls.load()
    st = lib.ipls_sort_ex(ctypes.c_void_p(4096), None, 100, ipls.F64, ctypes.byref(p), None, 0, None, None)
    assert st == 1  # IPLS_ERR_INVALID


def test_unknown_param_name_is_an_error():
    if not os.path.exists(ipls.LIB_PATH):
        pytest.skip("libipls.so not built")
    with pytest.raises(TypeError):
        ipls.default_params(sample_polciy=1)


def test_host_side_argument_errors():
    # all reported synchronously, before any device work
    if not os.path.exists(ipls.LIB_PATH):
        pytest.skip("libipls.so not built")
    lib = ipls.load()
    p = ipls.default_params()
    fake = ctypes.c_void_p(1 << 20)
    assert lib.ipls_sort_ex(None, None, 10, ipls.F64, ctypes.byref(p), None, 0, None, None) == 1  # null keys
    assert lib.ipls_sort_ex(fake, None, 10, 7, ctypes.byref(p), None, 0, None, None) == 2  # unknown dtype
    assert lib.ipls_sort_ex(ctypes.c_void_p((1 << 20) + 4), None, 10, ipls.F64, ctypes.byref(p), None, 0,
                            None, None) == 1  # misaligned fp64 keys
    need = ipls.workspace_bytes(1000, ipls.F64, False)
    assert lib.ipls_sort_ex(fake, None, 1000, ipls.F64, ctypes.byref(p), fake, need - 1, None, None) == 1
    assert lib.ipls_sort_ex(fake, None, 1000, ipls.F64, ctypes.byref(p), ctypes.c_void_p((1 << 20) + 8), need,
                            None, None) == 1  # workspace not 256-byte aligned
    assert lib.ipls_sort_segmented(None, None, fake, 3, ipls.F64, None, None, None) == 1
    assert lib.ipls_fit_model(fake, 100, ipls.F64, 1, 3, fake, None) == 1  # K < 4
    assert lib.ipls_l2pl_train(fake, 2, 256, 256, 4, fake, fake, None, None) == 1  # S < 3
    big = ipls.default_params(num_buckets=512)
    assert lib.ipls_sort_ex(fake, None, 10, ipls.F64, ctypes.byref(big), None, 0, None, None) == 6  # K > 256


class _FakeDeviceTensor:
    """Stands in for a device tensor on a host without a GPU: the wrapper's checks read only these."""

    def __init__(self, n, dtype, contiguous=True):
        self._n, self.dtype, self._c = n, dtype, contiguous
        self.is_cuda = True

    def is_contiguous(self):
        return self._c

    def numel(self):
        return self._n

    def data_ptr(self):
        raise AssertionError("the wrapper reached the library call")


@pytest.mark.parametrize("bad", ["short", "strided", "dtype"])
@pytest.mark.parametrize("entry", ["sort_", "sort_plain", "sort_segmented_", "partition_"])
def test_wrapper_refuses_a_bad_payload_before_any_launch(monkeypatch, entry, bad):
    import torch

    def no_library(*a, **k):
        raise AssertionError("the wrapper reached the library")

    monkeypatch.setattr(ipls, "load", no_library)
    keys = _FakeDeviceTensor(100, torch.float64)
    pay = {"short": _FakeDeviceTensor(99, torch.int32),
           "strided": _FakeDeviceTensor(100, torch.int32, contiguous=False),
           "dtype": _FakeDeviceTensor(100, torch.int64)}[bad]
    with pytest.raises((ValueError, TypeError)):
        if entry == "sort_segmented_":
            ipls.sort_segmented_(keys, _FakeDeviceTensor(3, torch.int64), payload=pay)
        elif entry == "partition_":
            ipls.partition_(keys, payload=pay, params=object())
        else:
            getattr(ipls, entry)(keys, pay)


def test_noalloc_entry_point_refuses_sizes_beyond_its_array_without_a_gpu():
    # the dtype and size checks come before any HIP call, so they answer on a host without a GPU
    if not os.path.exists(ipls.LIB_PATH):
        pytest.skip("libipls.so not built")
    lib = ipls.load()
    assert lib.ipls_sort_noalloc(ctypes.c_void_p(4096), None, ipls.NOALLOC_MAX_KEYS + 1, ipls.F64, None, None,
                                 None) == 6  # IPLS_ERR_UNSUPPORTED
    assert lib.ipls_sort_noalloc(ctypes.c_void_p(4096), None, 100, 7, None, None, None) == 2  # IPLS_ERR_DTYPE
    with open(os.path.join(ROOT, "include", "ipls.h")) as f:
        assert f"#define IPLS_NOALLOC_MAX_KEYS (1ull << {ipls.NOALLOC_MAX_KEYS.bit_length() - 1})" in f.read()
