"""Sparse-HRIR rendering on MI355X (gfx950): Python binding of libhrir.so.

Every call below marshals arguments into the C ABI declared in
``include/hrir.h``; all rendering arithmetic runs in the library's HIP
kernels.  Device buffers are torch tensors on the current HIP device
(PyTorch provides device memory and streams only).  If ``libhrir.so`` has not
been built, importing this package raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_uint32, c_uint64, c_void_p

import numpy as np

# torch first: libhrir.so then binds to the HIP runtime torch already loaded
# (same soname), so device pointers and streams from torch are valid in it.
# Loading the library first would bring in a second HIP runtime.
import torch  # noqa: F401  (load order matters)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhrir.so")

HRIR_OK, HRIR_EINVAL, HRIR_ENOMEM, HRIR_ENOTPD, HRIR_EAGAIN, HRIR_EDEVICE = 0, -1, -2, -3, -4, -5
HRIR_REFIT_NNLS = 1
HRIR_FACTORIZE_DEVICE = 2
SPCONV_PERSISTENT, SPCONV_GRAPH, SPCONV_UNFUSED, SPCONV_LDS_GATHER, SPCONV_REGWIN, SPCONV_WG256 = 1, 2, 4, 8, 16, 32

_ERRNAMES = {-1: "EINVAL", -2: "ENOMEM", -3: "ENOTPD", -4: "EAGAIN", -5: "EDEVICE"}


class HrirError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class SpconvJob(ctypes.Structure):
    _fields_ = [("src", c_int32), ("filt", c_int32), ("out_off", c_int64)]


class BlockJob(ctypes.Structure):
    _fields_ = [("stream_id", c_int32), ("n", c_int32), ("filt_l", c_int32), ("filt_r", c_int32),
                ("flags", c_int32), ("pad", c_int32), ("in_off", c_int64), ("out_off", c_int64)]


BLOCK_FLUSH = 1

# numpy layout of block_job (40 bytes), for building job tables without a
# Python loop
BLOCK_JOB_DTYPE = np.dtype([("stream_id", "<i4"), ("n", "<i4"), ("filt_l", "<i4"), ("filt_r", "<i4"),
                            ("flags", "<i4"), ("pad", "<i4"), ("in_off", "<i8"), ("out_off", "<i8")])
assert BLOCK_JOB_DTYPE.itemsize == ctypes.sizeof(BlockJob)


STREAM_DIRECT_LAUNCH = 1
STREAM_ZERO_COPY = 2
STREAM_SLEEPING_COMPLETION = 4
STREAM_RESULT_TAIL = 1


class HrirResult(ctypes.Structure):
    _fields_ = [("tag", c_uint64), ("stream_id", c_int32), ("n", c_int32), ("out", POINTER(c_float)),
                ("t_submit_ns", c_int64), ("t_launch_ns", c_int64), ("t_done_ns", c_int64), ("flags", c_int32),
                ("pad", c_int32)]


assert ctypes.sizeof(HrirResult) == 56


class StreamLoad(ctypes.Structure):
    _fields_ = [("n_streams", c_int32), ("block_min", c_int32), ("block_max", c_int32), ("n_filters", c_int32),
                ("rate_hz", c_double), ("duration_s", c_double), ("seed", c_uint64), ("max_blocks", c_int64),
                ("signal", POINTER(c_float)), ("signal_len", c_int64), ("submit_threads", c_int32), ("pad", c_int32)]


class StreamLoadStats(ctypes.Structure):
    _fields_ = [("blocks", c_int64), ("out_samples", c_int64), ("eagain", c_int64), ("launches", c_int64),
                ("offered_hz", c_double), ("achieved_hz", c_double), ("out_samples_per_s", c_double),
                ("submit_s", c_double), ("wall_s", c_double), ("mean_batch", c_double), ("p50_ms", c_double),
                ("p99_ms", c_double), ("max_ms", c_double), ("p50_server_ms", c_double),
                ("p99_server_ms", c_double), ("p99_admit_ms", c_double), ("max_admit_ms", c_double),
                ("p99_collect_ms", c_double), ("max_collect_ms", c_double), ("max_wait_ms", c_double),
                ("max_launch_ms", c_double), ("p99_gen_lag_ms", c_double), ("max_gen_lag_ms", c_double)]


def _preload_torch_fft():
    """Load torch's hipFFT first (same soname as ROCm's), so the library's
    FFT leg runs on the FFT stack that matches torch's HIP runtime."""
    libdir = os.path.join(os.path.dirname(torch.__file__), "lib")
    for name in ("librocfft.so", "libhipfft.so"):
        path = os.path.join(libdir, name)
        if os.path.exists(path):
            ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with `python paper_1502_03162_amd/build.py`")
    _preload_torch_fft()
    lib = ctypes.CDLL(LIB_PATH)
    P_d, P_f, P_i32, P_i64 = POINTER(c_double), POINTER(c_float), POINTER(c_int32), POINTER(c_int64)
    sig = {
        "hrir_last_error": (c_char_p, []),
        "hrir_factorize": (c_int, [P_d, c_int32, c_int32, c_int32, c_int32, c_uint64, P_d, c_double, c_int32,
                                   c_uint32, P_d, P_d, P_i32, P_f, P_i32, P_d, P_d]),
        "spconv_plan": (c_int, [P_f, c_int32, P_i32, P_f, c_int32, c_int32, c_int32, POINTER(c_void_p)]),
        "spconv_plan_destroy": (None, [c_void_p]),
        "spconv_plan_multi": (c_int, [P_f, c_int32, c_int32, P_i32, P_i32, P_f, c_int32, c_int32, c_int32,
                                      POINTER(c_void_p)]),
        "spconv_batch_create": (c_int, [c_void_p, P_i64, P_i64, c_int32, POINTER(SpconvJob), c_int32, c_int32,
                                        c_int32, c_int32, POINTER(c_void_p)]),
        "spconv_batch_render": (c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p]),
        "spconv_batch_info": (c_int, [c_void_p, P_i64]),
        "spconv_batch_destroy": (None, [c_void_p]),
        "spconv_render": (c_int, [c_void_p, c_void_p, c_int64, P_i64, P_i64, c_int32, POINTER(SpconvJob), c_int32,
                                  c_void_p, c_int64, c_void_p]),
        "spconv_render_noalloc": (c_int, [c_void_p, c_void_p, c_int64, P_i64, P_i64, c_int32, POINTER(SpconvJob),
                                          c_int32, c_void_p, c_int64, c_void_p]),
        "dense_plan": (c_int, [P_f, c_int32, c_int32, POINTER(c_void_p)]),
        "dense_plan_destroy": (None, [c_void_p]),
        "dense_batch_create": (c_int, [c_void_p, P_i64, P_i64, c_int32, POINTER(SpconvJob), c_int32,
                                       POINTER(c_void_p)]),
        "dense_batch_render": (c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p]),
        "dense_batch_destroy": (None, [c_void_p]),
        "fftola_create": (c_int, [P_f, c_int32, c_int32, c_int32, P_i64, P_i64, c_int32, POINTER(SpconvJob), c_int32,
                                  POINTER(c_void_p)]),
        "fftola_render": (c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p]),
        "fftola_info": (c_int, [c_void_p, P_i64]),
        "fftola_destroy": (None, [c_void_p]),
        "spconv_plan_shape": (c_int, [c_void_p, P_i32]),
        "spconv_plan_device": (c_int, [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p), P_i32]),
        "block_streams_create": (c_int, [c_void_p, c_int32, POINTER(c_void_p)]),
        "block_streams_reset": (c_int, [c_void_p, P_i32, c_int32, c_void_p]),
        "block_render": (c_int, [c_void_p, c_void_p, c_int64, POINTER(BlockJob), c_int32, c_void_p, c_int64, c_void_p]),
        "block_streams_destroy": (None, [c_void_p]),
        "spconv_autotune": (c_int, [c_void_p, c_void_p, c_int64, P_i64, P_i64, c_int32, POINTER(SpconvJob), c_int32,
                                    c_void_p, c_int64, c_void_p, c_char_p, c_int32, P_i32, P_i32, P_i32, P_d]),
        "stream_open": (c_int, [c_void_p, c_int32, c_int64, c_int32, POINTER(c_void_p)]),
        "stream_submit": (c_int, [c_void_p, c_int32, P_f, c_int32, c_int32, c_int32, c_uint64]),
        "stream_end": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_uint64]),
        "stream_poll": (c_int, [c_void_p, POINTER(HrirResult), c_int32, c_int32]),
        "stream_info": (c_int, [c_void_p, P_i64]),
        "stream_close": (None, [c_void_p]),
        "stream_loadgen": (c_int, [c_void_p, POINTER(StreamLoad), POINTER(StreamLoadStats)]),
        "hrir_sparsify": (c_int, [P_d, c_int32, c_int32, P_d, c_int32, c_int32, P_d, P_d, c_int32, c_double, c_int32,
                                  P_i32, P_f, P_i32, P_d, P_d]),
        "hrir_tune_sigma": (c_int, [P_d, c_int32, c_int32, P_d, c_int32, P_d, c_int32, c_double, c_int32, c_double,
                                    P_d, P_d]),
        "hrir_sparsify_device": (c_int, [P_d, c_int32, c_int32, P_d, c_int32, c_int32, P_d, P_d, c_int32, c_double,
                                         c_int32, P_i32, P_f, P_i32, P_d, P_d]),
        "hrir_tune_sigma_device": (c_int, [P_d, c_int32, c_int32, P_d, c_int32, P_d, c_int32, c_double, c_int32,
                                           c_double, P_d, P_d]),
        "spconv_plan_topk": (c_int, [c_void_p, c_int32, c_void_p, c_int32, c_int64, c_int32, c_void_p]),
        "spconv_plan_read": (c_int, [c_void_p, c_int32, c_int32, P_i32, P_f]),
        "moving_create": (c_int, [c_void_p, c_int32, c_int64, c_int32, c_int32, c_int32, POINTER(c_void_p)]),
        "moving_render": (c_int, [c_void_p, c_void_p, c_int64, P_i32, c_void_p, c_int64, c_int64, c_void_p]),
        "moving_info": (c_int, [c_void_p, P_i64]),
        "moving_destroy": (None, [c_void_p]),
        "surrogate_select": (c_int, [P_d, P_d, c_int32, P_d, P_d, P_d, c_int32, P_d, P_d, c_int32, c_double, P_i32]),
        "mlp_create": (c_int, [P_i32, c_int32, c_int32, POINTER(c_void_p)]),
        "mlp_num_params": (c_int64, [c_void_p]),
        "mlp_set_params": (c_int, [c_void_p, P_f, c_int64]),
        "mlp_get_params": (c_int, [c_void_p, P_f, c_int64]),
        "mlp_forward": (c_int, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
        "mlp_grads": (c_int, [c_void_p, c_void_p, c_void_p, c_int32, P_f, P_d, c_void_p]),
        "mlp_train": (c_int, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_float, P_d, c_void_p]),
        "mlp_destroy": (None, [c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("hrir_last_error", "hrir_factorize", "spconv_plan", "spconv_plan_multi", "spconv_plan_destroy", "spconv_batch_create",
            "spconv_batch_render", "spconv_batch_info", "spconv_batch_destroy", "spconv_render", "spconv_render_noalloc", "dense_plan",
            "dense_plan_destroy", "dense_batch_create", "dense_batch_render", "dense_batch_destroy", "fftola_create",
            "fftola_render", "fftola_info", "fftola_destroy", "spconv_plan_shape", "spconv_autotune",
            "spconv_plan_device", "block_streams_create", "block_streams_reset", "block_render",
            "block_streams_destroy", "stream_open", "stream_submit", "stream_end", "stream_poll", "stream_info",
            "stream_close", "stream_loadgen", "hrir_sparsify", "hrir_tune_sigma", "hrir_sparsify_device",
            "hrir_tune_sigma_device",
            "spconv_plan_topk", "spconv_plan_read", "moving_create", "moving_render", "moving_info",
            "moving_destroy", "surrogate_select", "mlp_create", "mlp_num_params", "mlp_set_params", "mlp_get_params", "mlp_forward", "mlp_grads",
            "mlp_train", "mlp_destroy")


def lib() -> ctypes.CDLL:
    return _lib


def _check(rc: int):
    if rc != HRIR_OK:
        raise HrirError(rc, _lib.hrir_last_error().decode())


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(POINTER(ct))


def _dev_ptr(t, dtype=None) -> int:
    """Device address of a contiguous torch tensor on a HIP device."""
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    return t.data_ptr()


def _f32(t):
    import torch
    return c_void_p(_dev_ptr(t, torch.float32)), t.numel()


def _stream_handle(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


# ---------------------------------------------------------------------------
# Factorization (host, FP64)
# ---------------------------------------------------------------------------
def factorize(X, lf: int, iters: int, k: int, seed: int = 0, g0=None, lambda0: float = 0.0,
              refit: bool = True, want_cost: bool = True, device: bool = False) -> dict:
    """Toeplitz-constrained semi-NMF of an HRIR set X [n][m] (Alg. 1) and
    top-k sparsification; device=True runs the iterations on the GPU.
    Returns f, G (dense), p, g, nnz, err_db, cost."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, m = X.shape
    lg = max(m - lf + 1, 1)
    f = np.empty(max(lf, 1))
    G = np.empty((n, lg))
    p = np.empty((n, max(k, 1)), dtype=np.int32)
    g = np.empty((n, max(k, 1)), dtype=np.float32)
    nnz = np.empty(n, dtype=np.int32)
    err = np.empty(n)
    cost = np.empty(iters) if want_cost else None
    g0a = None if g0 is None else np.ascontiguousarray(g0, dtype=np.float64)
    _check(_lib.hrir_factorize(_ptr(X, c_double), n, m, lf, iters, c_uint64(seed),
                               None if g0a is None else _ptr(g0a, c_double), lambda0, k,
                               (HRIR_REFIT_NNLS if refit else 0) | (HRIR_FACTORIZE_DEVICE if device else 0),
                               _ptr(f, c_double), _ptr(G, c_double),
                               _ptr(p, c_int32), _ptr(g, c_float), _ptr(nnz, c_int32), _ptr(err, c_double),
                               None if cost is None else _ptr(cost, c_double)))
    return {"f": f, "G": G, "p": p, "g": g, "nnz": nnz, "err_db": err, "cost": cost}


HRIR_D_IDENTITY, HRIR_D_CONV, HRIR_D_WINDOW = 0, 1, 2
_TRANSFORMS = {"I": HRIR_D_IDENTITY, "C": HRIR_D_CONV, "W": HRIR_D_WINDOW}


def sparsify(X, f, k: int, transform: str = "I", sigma=None, lam=None, target_nnze: int = 0,
             threshold: float = 1e-4, device: bool = False) -> dict:
    """The paper's sparsifier (hrir_sparsify, or hrir_sparsify_device with
    device=True): per-row L1-NNLS with the resonance filter f fixed,
    transform 'I', 'C' or 'W' (sigma per row or a scalar), lam per row /
    scalar, or None to search lambda for target_nnze.  Returns p, g (k-slot
    tap table), nnze, lambda, err_db."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    n, m = X.shape
    sig = None if sigma is None else np.ascontiguousarray(np.broadcast_to(sigma, (n,)), dtype=np.float64)
    la = None if lam is None else np.ascontiguousarray(np.broadcast_to(lam, (n,)), dtype=np.float64)
    p = np.empty((n, max(k, 1)), dtype=np.int32)
    g = np.empty((n, max(k, 1)), dtype=np.float32)
    nnze = np.empty(n, dtype=np.int32)
    lam_out = np.empty(n)
    err = np.empty(n)
    fn = _lib.hrir_sparsify_device if device else _lib.hrir_sparsify
    _check(fn(_ptr(X, c_double), n, m, _ptr(f, c_double), f.size, _TRANSFORMS[transform],
                              None if sig is None else _ptr(sig, c_double), None if la is None else _ptr(la, c_double),
                              int(target_nnze), float(threshold), int(k), _ptr(p, c_int32), _ptr(g, c_float),
                              _ptr(nnze, c_int32), _ptr(lam_out, c_double), _ptr(err, c_double)))
    return {"p": p, "g": g, "nnze": nnze, "lambda": lam_out, "err_db": err}


def tune_sigma(X, f, grid, lam: float = 0.0, threshold: float = 1e-4, target_nnze: int = 0, device: bool = False):
    """Per-row window bandwidth from grid minimising spectral distortion
    (hrir_tune_sigma, or hrir_tune_sigma_device with device=True): each
    bandwidth's solution at lambda = lam, or, with target_nnze > 0, at the
    searched lambda that keeps at most target_nnze entries.  Returns
    (sigma, sd)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    gr = np.ascontiguousarray(grid, dtype=np.float64)
    n, m = X.shape
    sig = np.empty(n)
    sd = np.empty(n)
    fn = _lib.hrir_tune_sigma_device if device else _lib.hrir_tune_sigma
    _check(fn(_ptr(X, c_double), n, m, _ptr(f, c_double), f.size, _ptr(gr, c_double), gr.size, float(lam),
              int(target_nnze), float(threshold), _ptr(sig, c_double), _ptr(sd, c_double)))
    return sig, sd


# ---------------------------------------------------------------------------
# Rendering
# ---------------------------------------------------------------------------
class Plan:
    """Resonance filter(s) r and tap table (p, g) resident on the device.
    r is [lf], or [n_res][lf] with `regions` giving each filter's region
    (spconv_plan_multi)."""

    def __init__(self, r, p, g, lg: int, regions=None):
        r = np.ascontiguousarray(r, dtype=np.float32)
        p = np.ascontiguousarray(p, dtype=np.int32)
        g = np.ascontiguousarray(g, dtype=np.float32)
        if p.ndim != 2 or p.shape != g.shape:
            raise ValueError("p and g must be [n_filters][k] arrays of the same shape")
        r2 = r.reshape(1, -1) if r.ndim == 1 else r
        self.n_res = int(r2.shape[0])
        self.lf, self.lg = int(r2.shape[1]), int(lg)
        self.n_filters, self.k = p.shape
        rg = None if regions is None else np.ascontiguousarray(regions, dtype=np.int32)
        if rg is not None and rg.shape != (self.n_filters,):
            raise ValueError("regions must hold one region per filter")
        h = c_void_p()
        _check(_lib.spconv_plan_multi(_ptr(r2, c_float), self.n_res, self.lf, None if rg is None else _ptr(rg, c_int32),
                                      _ptr(p, c_int32), _ptr(g, c_float), p.shape[0], p.shape[1], lg, byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def out_len(self, src_len: int) -> int:
        return int(src_len) + self.lf + self.lg - 2

    def close(self):
        if getattr(self, "_h", None):
            _lib.spconv_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001  (interpreter shutdown: the library may already be gone)
            pass


def make_jobs(rows):
    """rows: iterable of (src, filt, out_off) -> (ctypes array, count)."""
    rows = list(rows)
    arr = (SpconvJob * max(len(rows), 1))()
    for i, (s, f, o) in enumerate(rows):
        arr[i].src, arr[i].filt, arr[i].out_off = int(s), int(f), int(o)
    return arr, len(rows)


def row_layout(plan: Plan, src_len, jobs_sf, align: int = 64):
    """Output offsets for jobs given as (src, filt) pairs: each row starts on
    an `align`-element boundary.  Returns (out_off int64[n_jobs], total)."""
    src_len = np.asarray(src_len, dtype=np.int64)
    off = np.zeros(len(jobs_sf), dtype=np.int64)
    pos = 0
    for i, (s, _f) in enumerate(jobs_sf):
        off[i] = pos
        pos += (plan.out_len(src_len[s]) + align - 1) // align * align
    return off, int(pos)


class Batch:
    """A prepared job list over a fixed set of sources (spconv_batch_*)."""

    def __init__(self, plan: Plan, src_off, src_len, jobs, tile: int = 0, group: int = 0, flags: int = 0):
        self.plan = plan
        self.src_off = np.ascontiguousarray(src_off, dtype=np.int64)
        self.src_len = np.ascontiguousarray(src_len, dtype=np.int64)
        jobs, n_jobs = make_jobs(jobs)
        self._jobs = jobs
        self.n_jobs = n_jobs
        h = c_void_p()
        _check(_lib.spconv_batch_create(plan.handle, _ptr(self.src_off, c_int64), _ptr(self.src_len, c_int64),
                                        self.src_len.size, jobs, n_jobs, tile, group, flags, byref(h)))
        self._h = h

    def info(self) -> dict:
        a = np.zeros(5, dtype=np.int64)
        _check(_lib.spconv_batch_info(self._h, _ptr(a, c_int64)))
        return {"tiles": int(a[0]), "tile": int(a[1]), "group": int(a[2]), "grid": int(a[3]),
                "kernel": ("quad", "register_window", "lds_gather", "unfused")[int(a[4])]}

    def render(self, src, out, stream=None):
        """Enqueue on `stream` (default: torch's current stream)."""
        sp, sn = _f32(src)
        op, on = _f32(out)
        _check(_lib.spconv_batch_render(self._h, sp, sn, op, on, c_void_p(_stream_handle(stream))))

    def close(self):
        if getattr(self, "_h", None):
            _lib.spconv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001  (interpreter shutdown: the library may already be gone)
            pass


def autotune(plan: Plan, src, src_off, src_len, jobs, out, cache_path=None, force_flags: int = 0,
             stream=None) -> dict:
    """Fastest (tile, group, flags) for this job list (spconv_autotune);
    overwrites `out`'s job rows while timing."""
    src_off = np.ascontiguousarray(src_off, dtype=np.int64)
    src_len = np.ascontiguousarray(src_len, dtype=np.int64)
    jobs, n = make_jobs(jobs)
    sp, sn = _f32(src)
    op, on = _f32(out)
    t, g, f = c_int32(), c_int32(), c_int32()
    ms = c_double()
    _check(_lib.spconv_autotune(plan.handle, sp, sn, _ptr(src_off, c_int64), _ptr(src_len, c_int64), src_len.size,
                                jobs, n, op, on, c_void_p(_stream_handle(stream)),
                                None if cache_path is None else os.fsencode(cache_path), force_flags, byref(t),
                                byref(g), byref(f), byref(ms)))
    return {"tile": t.value, "group": g.value, "flags": f.value, "ms": ms.value}


def render(plan: Plan, src, src_off, src_len, jobs, out, stream=None):
    """One-shot synchronous render (spconv_render)."""
    src_off = np.ascontiguousarray(src_off, dtype=np.int64)
    src_len = np.ascontiguousarray(src_len, dtype=np.int64)
    jobs, n = make_jobs(jobs)
    sp, sn = _f32(src)
    op, on = _f32(out)
    _check(_lib.spconv_render(plan.handle, sp, sn, _ptr(src_off, c_int64), _ptr(src_len, c_int64), src_len.size,
                              jobs, n, op, on, c_void_p(_stream_handle(stream))))


def render_noalloc(plan: Plan, src, src_off, src_len, jobs, out, stream=None):
    """One-shot synchronous render that allocates nothing
    (spconv_render_noalloc): same results as render()."""
    src_off = np.ascontiguousarray(src_off, dtype=np.int64)
    src_len = np.ascontiguousarray(src_len, dtype=np.int64)
    jobs, n = make_jobs(jobs)
    sp, sn = _f32(src)
    op, on = _f32(out)
    _check(_lib.spconv_render_noalloc(plan.handle, sp, sn, _ptr(src_off, c_int64), _ptr(src_len, c_int64),
                                      src_len.size, jobs, n, op, on, c_void_p(_stream_handle(stream))))


NOALLOC_MAX_JOBS = 16384
NOALLOC_MAX_TILES = 65536


# ---------------------------------------------------------------------------
# Dense direct render (comparison leg)
# ---------------------------------------------------------------------------
class DensePlan:
    """Full HRIRs h [n_filters][m] (m <= 200) resident on the device."""

    def __init__(self, h):
        h = np.ascontiguousarray(h, dtype=np.float32)
        if h.ndim != 2:
            raise ValueError("h must be [n_filters][m]")
        self.n_filters, self.m = h.shape
        hd = c_void_p()
        _check(_lib.dense_plan(_ptr(h, c_float), h.shape[0], h.shape[1], byref(hd)))
        self._h = hd

    @property
    def handle(self):
        return self._h

    def out_len(self, src_len: int) -> int:
        return int(src_len) + self.m - 1

    def close(self):
        if getattr(self, "_h", None):
            _lib.dense_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001  (interpreter shutdown: the library may already be gone)
            pass


class DenseBatch:
    def __init__(self, plan: DensePlan, src_off, src_len, jobs):
        self.plan = plan
        self.src_off = np.ascontiguousarray(src_off, dtype=np.int64)
        self.src_len = np.ascontiguousarray(src_len, dtype=np.int64)
        jobs, n = make_jobs(jobs)
        self._jobs = jobs
        hd = c_void_p()
        _check(_lib.dense_batch_create(plan.handle, _ptr(self.src_off, c_int64), _ptr(self.src_len, c_int64),
                                       self.src_len.size, jobs, n, byref(hd)))
        self._h = hd

    def render(self, src, out, stream=None):
        sp, sn = _f32(src)
        op, on = _f32(out)
        _check(_lib.dense_batch_render(self._h, sp, sn, op, on, c_void_p(_stream_handle(stream))))

    def close(self):
        if getattr(self, "_h", None):
            _lib.dense_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001  (interpreter shutdown: the library may already be gone)
            pass


# ---------------------------------------------------------------------------
# Partitioned FFT convolution, overlap-add (comparison leg)
# ---------------------------------------------------------------------------
class FftOla:
    """Overlap-add FFT convolution of a fixed job list (hipFFT transforms)."""

    def __init__(self, h, nfft: int, src_off, src_len, jobs):
        h = np.ascontiguousarray(h, dtype=np.float32)
        self.n_filters, self.m = h.shape
        self.src_off = np.ascontiguousarray(src_off, dtype=np.int64)
        self.src_len = np.ascontiguousarray(src_len, dtype=np.int64)
        jobs, n = make_jobs(jobs)
        self._jobs = jobs
        hd = c_void_p()
        _check(_lib.fftola_create(_ptr(h, c_float), h.shape[0], h.shape[1], nfft, _ptr(self.src_off, c_int64),
                                  _ptr(self.src_len, c_int64), self.src_len.size, jobs, n, byref(hd)))
        self._h = hd

    def out_len(self, src_len: int) -> int:
        return int(src_len) + self.m - 1

    def info(self) -> dict:
        a = np.zeros(4, dtype=np.int64)
        _check(_lib.fftola_info(self._h, _ptr(a, c_int64)))
        return {"nfft": int(a[0]), "block": int(a[1]), "source_blocks": int(a[2]), "job_blocks": int(a[3])}

    def render(self, src, out, stream=None):
        sp, sn = _f32(src)
        op, on = _f32(out)
        _check(_lib.fftola_render(self._h, sp, sn, op, on, c_void_p(_stream_handle(stream))))

    def close(self):
        if getattr(self, "_h", None):
            _lib.fftola_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001  (interpreter shutdown: the library may already be gone)
            pass


# ---------------------------------------------------------------------------
# Block rendering with device-resident stream history
# ---------------------------------------------------------------------------
class Streams:
    """Per-stream history slots for block rendering (block_streams_*)."""

    def __init__(self, plan: Plan, max_streams: int):
        self.plan = plan
        self.max_streams = max_streams
        self.tail = plan.lf + plan.lg - 2
        hd = c_void_p()
        _check(_lib.block_streams_create(plan.handle, max_streams, byref(hd)))
        self._h = hd
        self._jobs = (BlockJob * max_streams)()

    def reset(self, slots, stream=None):
        a = np.ascontiguousarray(slots, dtype=np.int32)
        _check(_lib.block_streams_reset(self._h, _ptr(a, c_int32), a.size, c_void_p(_stream_handle(stream))))

    def render(self, d_in, jobs, d_out, stream=None):
        """jobs: a numpy array of BLOCK_JOB_DTYPE, or an iterable of
        (stream_id, n, filt_l, filt_r, in_off, out_off, flush)."""
        if isinstance(jobs, np.ndarray):
            if jobs.dtype != BLOCK_JOB_DTYPE or not jobs.flags.c_contiguous:
                raise ValueError("job table must be a contiguous BLOCK_JOB_DTYPE array")
            table, n = jobs.ctypes.data_as(POINTER(BlockJob)), jobs.size
        else:
            n = 0
            for (sid, ln, fl, fr, io, oo, flush) in jobs:
                j = self._jobs[n]
                j.stream_id, j.n, j.filt_l, j.filt_r = int(sid), int(ln), int(fl), int(fr)
                j.flags, j.pad, j.in_off, j.out_off = BLOCK_FLUSH if flush else 0, 0, int(io), int(oo)
                n += 1
            table = self._jobs
        if d_in is None:
            ip, inn = c_void_p(0), 0
        else:
            ip, inn = _f32(d_in)
        op, on = _f32(d_out)
        _check(_lib.block_render(self._h, ip, inn, table, n, op, on, c_void_p(_stream_handle(stream))))

    def close(self):
        if getattr(self, "_h", None):
            _lib.block_streams_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001  (interpreter shutdown: the library may already be gone)
            pass


class Server:
    """Streaming request loop with continuous batching (stream_*).

    submit/end return False when the server refuses the block for lack of
    room (HRIR_EAGAIN): poll, then try again.  poll returns finished results
    as (tag, stream_id, out, t_submit_ns, t_launch_ns, t_done_ns, is_tail)
    with out a float32 array [2, n] (left, right) copied out of the server's
    buffer."""

    def __init__(self, plan: Plan, max_streams: int, hbm_budget: int = 0, flags: int = 0):
        self.plan = plan
        self.max_streams = max_streams
        self.tail = plan.lf + plan.lg - 2
        hd = c_void_p()
        _check(_lib.stream_open(plan.handle, max_streams, int(hbm_budget), flags, byref(hd)))
        self._h = hd
        self._res = (HrirResult * 4096)()

    def submit(self, stream_id: int, block, filt_l: int, filt_r: int, tag: int = 0) -> bool:
        a = np.ascontiguousarray(block, dtype=np.float32)
        rc = _lib.stream_submit(self._h, int(stream_id), _ptr(a, c_float), a.size, int(filt_l), int(filt_r), int(tag))
        if rc == HRIR_EAGAIN:
            return False
        _check(rc)
        return True

    def end(self, stream_id: int, filt_l: int, filt_r: int, tag: int = 0) -> bool:
        rc = _lib.stream_end(self._h, int(stream_id), int(filt_l), int(filt_r), int(tag))
        if rc == HRIR_EAGAIN:
            return False
        _check(rc)
        return True

    def poll(self, max_results: int = 4096, timeout_us: int = 0):
        n = _lib.stream_poll(self._h, self._res, min(int(max_results), len(self._res)), int(timeout_us))
        if n < 0:
            _check(n)
        out = []
        for i in range(n):
            r = self._res[i]
            if r.n > 0:
                y = np.ctypeslib.as_array(r.out, shape=(2 * r.n,)).reshape(2, r.n).copy()
            else:
                y = np.zeros((2, 0), dtype=np.float32)
            out.append((int(r.tag), int(r.stream_id), y, int(r.t_submit_ns), int(r.t_launch_ns), int(r.t_done_ns),
                        bool(r.flags & STREAM_RESULT_TAIL)))
        return out

    def info(self) -> dict:
        v = np.zeros(8, dtype=np.int64)
        _check(_lib.stream_info(self._h, _ptr(v, c_int64)))
        keys = ("launches", "results", "samples", "eagain", "max_batch", "generations", "gen_samples", "queued")
        return dict(zip(keys, (int(x) for x in v)))

    def loadgen(self, signal, n_streams: int, rate_hz: float, duration_s: float, block_min: int = 64,
                block_max: int = 1024, n_filters: int = 2, seed: int = 0, max_blocks: int = 1 << 22,
                submit_threads: int = 1) -> dict:
        """Runs the library's open-loop Poisson load generator (stream_loadgen)
        against this server; rate_hz <= 0 submits back to back."""
        sig = np.ascontiguousarray(signal, dtype=np.float32)
        cfg = StreamLoad(int(n_streams), int(block_min), int(block_max), int(n_filters), float(rate_hz),
                         float(duration_s), int(seed), int(max_blocks), _ptr(sig, c_float), sig.size,
                         int(submit_threads), 0)
        st = StreamLoadStats()
        _check(_lib.stream_loadgen(self._h, byref(cfg), byref(st)))
        return {name: getattr(st, name) for name, _ in StreamLoadStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.stream_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001  (interpreter shutdown: the library may already be gone)
            pass


class Mlp:
    """Direction-conditioned surrogate network (mlp_*): ReLU layers with the
    given sizes; parameters as a list of (W [k_in][k_out], b [k_out])."""

    def __init__(self, sizes, max_batch: int):
        self.sizes = [int(x) for x in sizes]
        sz = np.asarray(self.sizes, dtype=np.int32)
        hd = c_void_p()
        _check(_lib.mlp_create(_ptr(sz, c_int32), len(self.sizes) - 1, int(max_batch), byref(hd)))
        self._h = hd
        self.n_params = int(_lib.mlp_num_params(hd))

    def set_params(self, params):
        flat = np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()])
                               for W, b in params]).astype(np.float32)
        _check(_lib.mlp_set_params(self._h, _ptr(flat, c_float), flat.size))

    def _unflatten(self, flat):
        out, o = [], 0
        for k_in, k_out in zip(self.sizes[:-1], self.sizes[1:]):
            W = flat[o:o + k_in * k_out].reshape(k_in, k_out)
            o += k_in * k_out
            b = flat[o:o + k_out]
            o += k_out
            out.append((W, b))
        return out

    def get_params(self):
        flat = np.empty(self.n_params, dtype=np.float32)
        _check(_lib.mlp_get_params(self._h, _ptr(flat, c_float), flat.size))
        return self._unflatten(flat)

    def forward(self, x, y, stream=None):
        """x: device tensor [n][sizes[0]], y: device tensor [n][sizes[-1]] (float32)."""
        xp, _ = _f32(x)
        yp, _ = _f32(y)
        _check(_lib.mlp_forward(self._h, xp, int(x.shape[0]), yp, c_void_p(_stream_handle(stream))))

    def grads(self, x, t, stream=None):
        flat = np.empty(self.n_params, dtype=np.float32)
        loss = c_double()
        xp, _ = _f32(x)
        tp, _ = _f32(t)
        _check(_lib.mlp_grads(self._h, xp, tp, int(x.shape[0]), _ptr(flat, c_float), byref(loss),
                              c_void_p(_stream_handle(stream))))
        return loss.value, self._unflatten(flat)

    def train(self, x, t, steps: int, lr: float, stream=None) -> float:
        loss = c_double()
        xp, _ = _f32(x)
        tp, _ = _f32(t)
        _check(_lib.mlp_train(self._h, xp, tp, int(x.shape[0]), int(steps), float(lr), byref(loss),
                              c_void_p(_stream_handle(stream))))
        return loss.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001  (interpreter shutdown: the library may already be gone)
            pass


def surrogate_select(q_az, q_el, val_az, val_el, val_err_db, meas_az, meas_el, max_err_db: float = -30.0):
    """Per query: -1 (use the surrogate) or the index of the nearest measured
    direction (surrogate_select)."""
    d = lambda a: np.ascontiguousarray(a, dtype=np.float64)  # noqa: E731
    qa, qe, va, ve, vr, ma, me = (d(x) for x in (q_az, q_el, val_az, val_el, val_err_db, meas_az, meas_el))
    ch = np.empty(qa.size, dtype=np.int32)
    _check(_lib.surrogate_select(_ptr(qa, c_double), _ptr(qe, c_double), qa.size, _ptr(va, c_double),
                                 _ptr(ve, c_double), _ptr(vr, c_double), va.size, _ptr(ma, c_double),
                                 _ptr(me, c_double), ma.size, float(max_err_db), _ptr(ch, c_int32)))
    return ch


def plan_topk(plan: Plan, first_row: int, dense, width: int, stream=None):
    """spconv_plan_topk: rows of a device tensor [n_rows][row_stride] -> the
    plan's tap rows first_row.. (k largest finite positive entries among the
    first `width`)."""
    dp, _ = _f32(dense)
    _check(_lib.spconv_plan_topk(plan.handle, int(first_row), dp, int(dense.shape[0]), int(dense.stride(0)),
                                 int(width), c_void_p(_stream_handle(stream))))


def plan_read(plan: Plan, first_row: int, n_rows: int):
    """Plan rows back to the host: (p int32 [n][k], g float32 [n][k])."""
    p = np.empty((n_rows, plan.k), dtype=np.int32)
    g = np.empty((n_rows, plan.k), dtype=np.float32)
    _check(_lib.spconv_plan_read(plan.handle, int(first_row), int(n_rows), _ptr(p, c_int32), _ptr(g, c_float)))
    return p, g


class Moving:
    """Moving sources (moving_*): n_src equal-length sources whose direction
    changes every seg_len samples, with a linear crossfade of `fade` samples."""

    def __init__(self, plan: Plan, n_src: int, src_len: int, seg_len: int, fade: int, tile: int = 0):
        self.plan = plan
        hd = c_void_p()
        _check(_lib.moving_create(plan.handle, int(n_src), int(src_len), int(seg_len), int(fade), int(tile),
                                  byref(hd)))
        self._h = hd
        v = np.zeros(4, dtype=np.int64)
        _check(_lib.moving_info(hd, _ptr(v, c_int64)))
        self.n_seg, self.out_len, self.n_tiles, self.tile = (int(x) for x in v)
        self.n_src = n_src

    def render(self, src, seg_filt, out, out_stride: int, stream=None):
        sf = np.ascontiguousarray(seg_filt, dtype=np.int32)
        if sf.shape != (self.n_src, self.n_seg, 2):
            raise ValueError(f"seg_filt must be [{self.n_src}][{self.n_seg}][2]")
        sp, sn = _f32(src)
        op, on = _f32(out)
        _check(_lib.moving_render(self._h, sp, sn, _ptr(sf, c_int32), op, int(out_stride), on,
                                  c_void_p(_stream_handle(stream))))

    def close(self):
        if getattr(self, "_h", None):
            _lib.moving_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001  (interpreter shutdown: the library may already be gone)
            pass
