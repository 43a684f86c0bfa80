"""Python binding of libipls.so, the MI355X (gfx950) IPLS sort library.

Argument marshalling only: every step of the sort runs in the library's HIP kernels.  Tensors
are torch CUDA(HIP) tensors; their device pointers and the current stream are passed through
the C ABI declared in include/ipls.h.  Importing this module does not need a GPU; calling a
sort without the built library raises an error (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libipls.so")

F64, F32, U64 = 0, 1, 2
MODEL_FMCD, MODEL_AUTO, MODEL_L2PL = 0, 1, 2
KERNEL_SCATTER, KERNEL_CLASSIFY, KERNEL_BASE = 0, 1, 2

STATUS = {0: "IPLS_OK", 1: "IPLS_ERR_INVALID", 2: "IPLS_ERR_DTYPE", 3: "IPLS_ERR_OOM", 4: "IPLS_ERR_HIP",
          5: "IPLS_ERR_DEVICE", 6: "IPLS_ERR_UNSUPPORTED"}

EXPORTS = ["ipls_default_params", "ipls_sort", "ipls_sort_ex", "ipls_sort_noalloc", "ipls_sort_segmented", "ipls_fit_model",
           "ipls_partition", "ipls_l2pl_train", "ipls_l2pl_grad", "ipls_workspace_bytes", "ipls_stream_status",
           "ipls_status_string", "ipls_profile_enable", "ipls_profile_read", "ipls_profile_read_level", "ipls_autotune_segmented",
           "ipls_server_default_config", "ipls_server_create", "ipls_server_reserve", "ipls_server_submit",
           "ipls_server_wait", "ipls_server_poll", "ipls_server_release", "ipls_server_stats_get",
           "ipls_server_destroy"]


class IplsError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("num_buckets", C.c_uint32), ("base_case_max", C.c_uint32), ("sample_divisor", C.c_uint32),
                ("sample_min", C.c_uint32), ("sample_max", C.c_uint64), ("seed", C.c_uint64),
                ("model", C.c_uint32), ("leaves", C.c_uint32), ("train_iters", C.c_uint32),
                ("tile_keys", C.c_uint32), ("sample_policy", C.c_uint32),
                ("equality", C.c_uint32), ("inherit", C.c_uint32), ("bucket_policy", C.c_uint32)]


class LinearModel(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("D", C.c_uint64), ("K", C.c_uint32),
                ("degenerate", C.c_uint32)]


class Stats(C.Structure):
    _fields_ = [("levels", C.c_uint32), ("sample_depth", C.c_uint32), ("passes", C.c_uint64),
                ("closed", C.c_uint64), ("fallback", C.c_uint64), ("l2pl_used", C.c_uint64),
                ("base_buckets", C.c_uint64), ("level1_max_load", C.c_uint64), ("keys_partitioned", C.c_uint64),
                ("inherited", C.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class TuneReport(C.Structure):
    _fields_ = [("trials", C.c_uint32), ("window_segments", C.c_uint32), ("window_keys", C.c_uint64),
                ("default_ms", C.c_double), ("best_ms", C.c_double)]


class ServerConfig(C.Structure):
    _fields_ = [("lanes", C.c_uint32), ("batch_max_requests", C.c_uint32), ("batch_max_keys", C.c_uint64),
                ("batch_keys", C.c_uint64), ("params", Params)]


class ServerDone(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("n", C.c_uint64), ("status", C.c_int), ("batch_size", C.c_uint32),
                ("t_reserve", C.c_double), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in ("admitted", "completed", "rejected", "singles_run", "batches_run",
                                          "keys_sorted", "arena_bytes", "bytes_in_use", "peak_bytes_in_use",
                                          "queue_depth", "max_queue_depth")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load the built library (raises if it is missing: build it with build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libipls.so not built at {path}; run python -m paper_2208_06902_amd.build")
    # torch brings its own HIP runtime; load it first so that the library binds to the same one
    # (the library loaded first would bind the system's runtime, and torch would then share it)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    P, sz, u32, u64, i32, dbl = C.c_void_p, C.c_size_t, C.c_uint32, C.c_uint64, C.c_int, C.c_double
    sig = {
        "ipls_default_params": (None, [C.POINTER(Params)]),
        "ipls_sort": (i32, [P, P, sz, i32, P]),
        "ipls_sort_ex": (i32, [P, P, sz, i32, C.POINTER(Params), P, sz, C.POINTER(Stats), P]),
        "ipls_sort_noalloc": (i32, [P, P, sz, i32, C.POINTER(Params), C.POINTER(Stats), P]),
        "ipls_sort_segmented": (i32, [P, P, P, sz, i32, C.POINTER(Params), C.POINTER(Stats), P]),
        "ipls_fit_model": (i32, [P, sz, i32, i32, u32, P, P]),
        "ipls_partition": (i32, [P, P, sz, i32, C.POINTER(Params), P, P, P]),
        "ipls_l2pl_train": (i32, [P, sz, u32, u32, u32, P, P, P, P]),
        "ipls_l2pl_grad": (i32, [P, sz, u32, u32, P, P, P, P]),
        "ipls_workspace_bytes": (sz, [sz, i32, i32, C.POINTER(Params)]),
        "ipls_stream_status": (i32, [P]),
        "ipls_status_string": (C.c_char_p, [i32]),
        "ipls_profile_enable": (None, [i32]),
        "ipls_profile_read": (None, [i32, C.POINTER(u64), C.POINTER(dbl), C.POINTER(dbl)]),
        "ipls_profile_read_level": (None, [i32, i32, C.POINTER(u64), C.POINTER(dbl), C.POINTER(dbl)]),
        "ipls_autotune_segmented": (i32, [P, P, sz, i32, i32, C.POINTER(Params), C.POINTER(Params),
                                          C.POINTER(TuneReport), P]),
        "ipls_server_default_config": (None, [C.POINTER(ServerConfig)]),
        "ipls_server_create": (i32, [P, sz, C.POINTER(ServerConfig), C.POINTER(P)]),
        "ipls_server_reserve": (i32, [P, sz, i32, i32, C.POINTER(u64), C.POINTER(P), C.POINTER(P)]),
        "ipls_server_submit": (i32, [P, u64, P]),
        "ipls_server_wait": (i32, [P, u64, C.POINTER(ServerDone)]),
        "ipls_server_poll": (i32, [P, C.POINTER(ServerDone), sz, C.POINTER(sz)]),
        "ipls_server_release": (i32, [P, u64]),
        "ipls_server_stats_get": (i32, [P, C.POINTER(ServerStats)]),
        "ipls_server_destroy": (i32, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def default_params(**kw) -> Params:
    p = Params()
    load().ipls_default_params(C.byref(p))
    names = {f for f, _ in Params._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown ipls_params field {k!r}")
        setattr(p, k, v)
    return p


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.uint64:
        return U64
    raise TypeError(f"unsupported key dtype {t.dtype}")


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(st: int, where: str):
    if st != 0:
        raise IplsError(st, where)


def _check_tensor(t, name):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")


def _check_payload(payload, keys):
    """A payload is a contiguous 32-bit device tensor with one element per key: the library can
    only check its pointer's alignment, so a shorter or strided tensor is refused here."""
    import torch
    if payload is None:
        return
    _check_tensor(payload, "payload")
    if payload.dtype != torch.int32 and payload.dtype != torch.uint32:
        raise TypeError("payload must be 32-bit")
    if payload.numel() != keys.numel():
        raise ValueError("payload and keys differ in length")


def sort_(keys, payload=None, params: Params | None = None, workspace=None, stream=None, stats: bool = False):
    """Sort `keys` (and `payload`, stably) in place on the GPU.  Returns stats if asked."""
    _check_tensor(keys, "keys")
    _check_payload(payload, keys)
    st = Stats()
    ws, wsb = (None, 0) if workspace is None else (_ptr(workspace), workspace.numel() * workspace.element_size())
    rc = load().ipls_sort_ex(_ptr(keys), _ptr(payload), keys.numel(), _dtype_code(keys),
                             C.byref(params) if params is not None else None, ws, wsb, C.byref(st), _stream(stream))
    _check(rc, "ipls_sort_ex")
    return st.as_dict() if stats else None


NOALLOC_MAX_KEYS = 1 << 22  # IPLS_NOALLOC_MAX_KEYS


def sort_noalloc_(keys, payload=None, params: Params | None = None, stream=None, stats: bool = False):
    """ipls_sort_noalloc: as sort_ without a workspace, with every buffer carved from the library's
    static device scratch array (no allocation); at most NOALLOC_MAX_KEYS keys."""
    _check_tensor(keys, "keys")
    _check_payload(payload, keys)
    st = Stats()
    rc = load().ipls_sort_noalloc(_ptr(keys), _ptr(payload), keys.numel(), _dtype_code(keys),
                                  C.byref(params) if params is not None else None, C.byref(st), _stream(stream))
    _check(rc, "ipls_sort_noalloc")
    return st.as_dict() if stats else None


def sort_plain(keys, payload=None, stream=None):
    """ipls_sort: default parameters."""
    _check_tensor(keys, "keys")
    _check_payload(payload, keys)
    rc = load().ipls_sort(_ptr(keys), _ptr(payload), keys.numel(), _dtype_code(keys), _stream(stream))
    _check(rc, "ipls_sort")


def sort_segmented_(keys, offsets, payload=None, params: Params | None = None, stream=None, stats: bool = False):
    """Sort every segment [offsets[s], offsets[s+1]) of `keys` independently, in place."""
    import torch
    _check_tensor(keys, "keys")
    _check_tensor(offsets, "offsets")
    if offsets.dtype not in (torch.int64, torch.uint64):
        raise TypeError("offsets must be 64-bit")
    if offsets.numel() < 1:
        raise ValueError("offsets needs at least one element (nseg + 1)")
    _check_payload(payload, keys)
    st = Stats()
    rc = load().ipls_sort_segmented(_ptr(keys), _ptr(payload), _ptr(offsets), offsets.numel() - 1,
                                    _dtype_code(keys), C.byref(params) if params is not None else None,
                                    C.byref(st), _stream(stream))
    _check(rc, "ipls_sort_segmented")
    return st.as_dict() if stats else None


def fit_model(sample, K: int, sorted_: bool = True, stream=None):
    """FMCD fit of a device sample: (a, b, D, degenerate)."""
    import torch
    _check_tensor(sample, "sample")
    out = torch.zeros(C.sizeof(LinearModel), dtype=torch.uint8, device=sample.device)
    rc = load().ipls_fit_model(_ptr(sample), sample.numel(), _dtype_code(sample), int(sorted_), K, _ptr(out),
                               _stream(stream))
    _check(rc, "ipls_fit_model")
    m = LinearModel.from_buffer_copy(bytes(out.cpu().numpy()))
    return m.a, m.b, int(m.D), int(m.degenerate)


def partition_(keys, payload=None, params: Params | None = None, stream=None):
    """One distribution pass in place: returns (counts tensor (K, uint64), (a, b, D, degenerate))."""
    import torch
    _check_tensor(keys, "keys")
    _check_payload(payload, keys)
    p = params if params is not None else default_params()
    counts = torch.zeros(p.num_buckets, dtype=torch.uint64, device=keys.device)
    mbuf = torch.zeros(C.sizeof(LinearModel), dtype=torch.uint8, device=keys.device)
    rc = load().ipls_partition(_ptr(keys), _ptr(payload), keys.numel(), _dtype_code(keys), C.byref(p),
                               _ptr(counts), _ptr(mbuf), _stream(stream))
    _check(rc, "ipls_partition")
    m = LinearModel.from_buffer_copy(bytes(mbuf.cpu().numpy()))
    return counts, (m.a, m.b, int(m.D), int(m.degenerate))


def l2pl_train(x, K: int, M: int, iters: int, stream=None):
    """Train the two-level model on a sorted fp64 device sample: (root (2), leaf (4M), ab (2M))."""
    import torch
    _check_tensor(x, "x")
    root = torch.zeros(2, dtype=torch.float64, device=x.device)
    leaf = torch.zeros(4 * M, dtype=torch.float64, device=x.device)
    ab = torch.zeros(2 * M, dtype=torch.float64, device=x.device)
    rc = load().ipls_l2pl_train(_ptr(x), x.numel(), K, M, iters, _ptr(root), _ptr(leaf), _ptr(ab), _stream(stream))
    _check(rc, "ipls_l2pl_train")
    return root, leaf, ab


def l2pl_grad(x, K: int, M: int, ab, stream=None):
    """Per-leaf MSE gradient (2M) and loss (M) of the two-level model at ab (2M)."""
    import torch
    _check_tensor(x, "x")
    g = torch.zeros(2 * M, dtype=torch.float64, device=x.device)
    loss = torch.zeros(M, dtype=torch.float64, device=x.device)
    rc = load().ipls_l2pl_grad(_ptr(x), x.numel(), K, M, _ptr(ab), _ptr(g), _ptr(loss), _stream(stream))
    _check(rc, "ipls_l2pl_grad")
    return g, loss


def workspace_bytes(n: int, dtype: int, has_payload: bool, params: Params | None = None) -> int:
    return int(load().ipls_workspace_bytes(n, dtype, int(has_payload), C.byref(params) if params else None))


def profile_enable(on=True):
    """on: True (every kernel), False (off) or a bit mask of kernel ids (1 << KERNEL_SCATTER, ...)."""
    mask = (7 if on else 0) if isinstance(on, bool) else int(on)
    load().ipls_profile_enable(mask)


def profile_read(kernel: int):
    n, ms, by = C.c_uint64(), C.c_double(), C.c_double()
    load().ipls_profile_read(kernel, C.byref(n), C.byref(ms), C.byref(by))
    return int(n.value), float(ms.value), float(by.value)


def profile_read_level(kernel: int, level: int):
    """(launches, ms, bytes) of one kernel id's launches at one recursion level."""
    n, ms, by = C.c_uint64(), C.c_double(), C.c_double()
    load().ipls_profile_read_level(kernel, level, C.byref(n), C.byref(ms), C.byref(by))
    return int(n.value), float(ms.value), float(by.value)


def status_string(st: int) -> str:
    return load().ipls_status_string(st).decode()


def autotune_segmented(keys, offsets, has_payload: bool = False, base: Params | None = None, stream=None):
    """Pick K, T and the tile size for segmented sorts shaped like this batch: (Params, report)."""
    _check_tensor(keys, "keys")
    _check_tensor(offsets, "offsets")
    out, rep = Params(), TuneReport()
    rc = load().ipls_autotune_segmented(_ptr(keys), _ptr(offsets), offsets.numel() - 1, _dtype_code(keys),
                                        int(has_payload), C.byref(base) if base is not None else None,
                                        C.byref(out), C.byref(rep), _stream(stream))
    _check(rc, "ipls_autotune_segmented")
    return out, {f: getattr(rep, f) for f, _ in rep._fields_}


def server_config(params: Params | None = None, **kw) -> ServerConfig:
    c = ServerConfig()
    load().ipls_server_default_config(C.byref(c))
    if params is not None:
        c.params = params
    names = {f for f, _ in ServerConfig._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown ipls_server_config field {k!r}")
        setattr(c, k, v)
    return c


_TORCH_DT = {F64: "float64", F32: "float32", U64: "uint64"}
_WIDTH = {F64: 8, F32: 4, U64: 8}


class Server:
    """Request server over a device arena (a torch uint8 tensor that is the HBM budget).

    reserve() returns (req_id, keys_view, payload_view) -- tensors aliasing the request's slot in
    the arena, or None when the budget is full right now.  Fill the views (on any stream), then
    submit(); wait() or poll() for completion; read the views; release().
    """

    def __init__(self, arena, config: ServerConfig | None = None):
        import torch
        _check_tensor(arena, "arena")
        if arena.dtype != torch.uint8:
            raise TypeError("arena must be a uint8 tensor")
        self.arena = arena
        self._h = C.c_void_p()
        rc = load().ipls_server_create(_ptr(arena), arena.numel(), C.byref(config) if config else None,
                                       C.byref(self._h))
        _check(rc, "ipls_server_create")

    def reserve(self, n: int, dtype: int, payload: bool = False):
        import torch
        rid, kp, pp = C.c_uint64(), C.c_void_p(), C.c_void_p()
        rc = load().ipls_server_reserve(self._h, n, dtype, int(payload), C.byref(rid), C.byref(kp), C.byref(pp))
        if rc == 3:
            return None
        _check(rc, "ipls_server_reserve")
        base = self.arena.data_ptr()
        ko = kp.value - base
        w = _WIDTH[dtype]
        if dtype == U64:
            kv = self.arena[ko:ko + n * w].view(torch.int64).view(torch.uint64)
        else:
            kv = self.arena[ko:ko + n * w].view(getattr(torch, _TORCH_DT[dtype]))
        pv = None
        if payload:
            po = pp.value - base
            pv = self.arena[po:po + n * 4].view(torch.int32)
        return int(rid.value), kv, pv

    def submit(self, req_id: int, stream=None):
        _check(load().ipls_server_submit(self._h, req_id, _stream(stream)), "ipls_server_submit")

    def wait(self, req_id: int) -> dict:
        d = ServerDone()
        rc = load().ipls_server_wait(self._h, req_id, C.byref(d))
        _check(rc, "ipls_server_wait")
        return d.as_dict()

    def poll(self, max_items: int = 256) -> list:
        arr = (ServerDone * max_items)()
        cnt = C.c_size_t()
        _check(load().ipls_server_poll(self._h, arr, max_items, C.byref(cnt)), "ipls_server_poll")
        return [arr[i].as_dict() for i in range(cnt.value)]

    def release(self, req_id: int):
        _check(load().ipls_server_release(self._h, req_id), "ipls_server_release")

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().ipls_server_stats_get(self._h, C.byref(st)), "ipls_server_stats_get")
        return st.as_dict()

    def close(self):
        if self._h:
            load().ipls_server_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
