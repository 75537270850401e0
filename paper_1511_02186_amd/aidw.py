"""Thin ctypes binding over libaidw.so (include/aidw.h).

The functions below carry the C names and only marshal arguments: every step
of the interpolation runs in the library's HIP kernels.  Tensors are torch
tensors already resident on the GPU; the library is handed their device
pointers and torch's current HIP stream.  If libaidw.so has not been built,
loading fails with an error instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# AIDW_LIBRARY selects another build of the library (same ABI), e.g. one made
# with extra compile options; the in-tree build is the default.
LIB_PATH = os.environ.get("AIDW_LIBRARY") or os.path.join(HERE, "libaidw.so")

AIDW_OK = 0
AIDW_EINVAL = -1
AIDW_ENOMEM = -2
AIDW_EDEVICE = -3
AIDW_EAGAIN = -4
AIDW_ENOTFOUND = -5

AIDW_FP32_SCALED = 0
AIDW_FP64 = 1

AIDW_FLAG_ASYNC = 1
AIDW_FLAG_GRID_KNN = 2

AIDW_ACCESS_SCALAR = 0
AIDW_ACCESS_TILED = 1
AIDW_ACCESS_NAIVE = 2
AIDW_LAYOUT_SOA = 0
AIDW_LAYOUT_AOAS = 1
AIDW_KMAX = 32
AIDW_MAX_POINTS = (1 << 31) - (1 << 16)
AIDW_NOALLOC_SCRATCH_BYTES = 64 << 20


class aidw_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("default_precision", ctypes.c_int),
                ("hbm_budget_bytes", ctypes.c_size_t), ("tune_path", ctypes.c_char_p),
                ("deterministic", ctypes.c_int)]


class aidw_issue_costs(ctypes.Structure):
    _fields_ = [("fma_cycles", ctypes.c_double), ("exp_cycles", ctypes.c_double),
                ("exp_cycles_beside_fma", ctypes.c_double), ("clock_ghz", ctypes.c_double),
                ("compute_units", ctypes.c_int), ("sgpr_operand_cycles", ctypes.c_double),
                ("sgpr_beside_vgpr_cycles", ctypes.c_double)]


class aidw_problem(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("data_xy", ctypes.c_void_p),
        ("data_z", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("query_xy", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("k", ctypes.c_int),
        ("alpha_levels", ctypes.c_double * 5),
        ("R_min", ctypes.c_double),
        ("R_max", ctypes.c_double),
        ("area", ctypes.c_double),
        ("out", ctypes.c_void_p),
        ("r_obs", ctypes.c_void_p),
        ("alpha", ctypes.c_void_p),
        ("knn_idx", ctypes.c_void_p),
        ("flags", ctypes.c_uint),
    ]


class aidw_tuning(ctypes.Structure):
    _fields_ = [("q_per_lane", ctypes.c_int), ("max_waves_per_simd", ctypes.c_int),
                ("split_segments", ctypes.c_int), ("speculate", ctypes.c_int),
                ("query_order", ctypes.c_int)]


class aidw_server_options(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_size_t), ("streams", ctypes.c_int),
                ("tick_pair_evals", ctypes.c_double), ("max_wait_s", ctypes.c_double),
                ("segment_points", ctypes.c_int64)]


class aidw_job(ctypes.Structure):
    _fields_ = [
        ("dataset", ctypes.c_uint64),
        ("data_xy", ctypes.c_void_p),
        ("data_z", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("area", ctypes.c_double),
        ("query_xy", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("k", ctypes.c_int),
        ("alpha_levels", ctypes.c_double * 5),
        ("R_min", ctypes.c_double),
        ("R_max", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("out", ctypes.c_void_p),
        ("r_obs", ctypes.c_void_p),
        ("alpha", ctypes.c_void_p),
        ("knn_idx", ctypes.c_void_p),
    ]


class aidw_server_counters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("ticks", ctypes.c_uint64),
                ("pair_evals", ctypes.c_double), ("arena_in_use", ctypes.c_size_t),
                ("queued", ctypes.c_uint64), ("admitted", ctypes.c_uint64)]


class AidwError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (status_name(status), message))
        self.status = status


_lib = None

_SIGNATURES = {
    "aidw_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(aidw_options)]),
    "aidw_destroy": (None, [ctypes.c_void_p]),
    "aidw_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "aidw_interpolate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_void_p]),
    "aidw_interpolate_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_problem)]),
    "aidw_interpolate_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_problem)]),
    "aidw_query_order": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p]),
    "aidw_describe_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_problem),
                                            ctypes.c_char_p, ctypes.c_size_t]),
    "aidw_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_tuning)]),
    "aidw_idw": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_problem), ctypes.c_double]),
    "aidw_interpolate_variant": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_problem),
                                                ctypes.c_int, ctypes.c_int]),
    "aidw_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                 ctypes.c_double, ctypes.POINTER(aidw_tuning)]),
    "aidw_tune_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "aidw_tune_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "aidw_synchronize": (ctypes.c_int, [ctypes.c_void_p]),
    "aidw_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_problem), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "aidw_batch_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint]),
    "aidw_batch_destroy": (None, [ctypes.c_void_p]),
    "aidw_interpolate_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_problem),
                                              ctypes.c_int, ctypes.c_uint]),
    "aidw_dataset_register": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_uint64)]),
    "aidw_dataset_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "aidw_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_server_options),
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "aidw_server_destroy": (None, [ctypes.c_void_p]),
    "aidw_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_job),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "aidw_probe_issue_costs": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_issue_costs)]),
    "aidw_server_submit_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_job),
                                                ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]),
    "aidw_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_double)]),
    "aidw_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_double)]),
    "aidw_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_job),
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "aidw_submit_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_job), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "aidw_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_double)]),
    "aidw_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
    "aidw_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aidw_server_counters)]),
    "aidw_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "aidw_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "aidw_version": (ctypes.c_int, []),
}


def lib():
    """Load libaidw.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libaidw.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_name(status: int) -> str:
    return lib().aidw_status_string(int(status)).decode()


def last_error(h=None) -> str:
    """The calling thread's most recent error message: of any call, or of
    calls on handle h."""
    return lib().aidw_last_error(h).decode()


def check(status: int) -> int:
    if status != AIDW_OK:
        raise AidwError(status, last_error())
    return status


# ---- the C entry points, same names ---------------------------------------

def aidw_create(device: int = 0, default_precision: int = AIDW_FP32_SCALED,
                hbm_budget_bytes: int = 0, tune_path=None, deterministic: int = 0) -> int:
    h = ctypes.c_void_p()
    opt = aidw_options(device, default_precision, hbm_budget_bytes,
                       None if tune_path is None else os.fsencode(tune_path), int(deterministic))
    check(lib().aidw_create(ctypes.byref(h), ctypes.byref(opt)))
    return h.value


def aidw_destroy(h) -> None:
    lib().aidw_destroy(h)


def aidw_set_stream(h, stream_ptr: int) -> int:
    return lib().aidw_set_stream(h, stream_ptr)


def aidw_interpolate(h, data_xy_ptr, data_z_ptr, m, query_xy_ptr, n, k, alpha_levels, R_min,
                     R_max, area, out_ptr) -> int:
    lv = (ctypes.c_double * 5)(*[float(a) for a in alpha_levels])
    return lib().aidw_interpolate(h, data_xy_ptr, data_z_ptr, int(m), query_xy_ptr, int(n),
                                  int(k), lv, float(R_min), float(R_max), float(area), out_ptr)


def aidw_interpolate_ex(h, problem: aidw_problem) -> int:
    return lib().aidw_interpolate_ex(h, ctypes.byref(problem))


def aidw_interpolate_noalloc(h, problem: aidw_problem) -> int:
    return lib().aidw_interpolate_noalloc(h, ctypes.byref(problem))


def aidw_query_order(h, query_xy, n: int, order) -> int:
    """Tile order of n queries into order (device tensors or raw addresses)."""
    ptr = lambda t: t if t is None or isinstance(t, int) else t.data_ptr()
    return lib().aidw_query_order(h, ptr(query_xy), int(n), ptr(order))


def aidw_describe_launch(h, problem: aidw_problem) -> str:
    """The kernels aidw_interpolate_ex would launch for `problem` (raises on error)."""
    buf = ctypes.create_string_buffer(1024)
    check(lib().aidw_describe_launch(h, ctypes.byref(problem), buf, len(buf)))
    return buf.value.decode()


def aidw_idw(h, problem: aidw_problem, power: float) -> int:
    return lib().aidw_idw(h, ctypes.byref(problem), float(power))


def aidw_interpolate_variant(h, problem: aidw_problem, access: int, layout: int) -> int:
    return lib().aidw_interpolate_variant(h, ctypes.byref(problem), int(access), int(layout))


def aidw_tune(h, m, n, k, budget_s=10.0):
    t = aidw_tuning()
    check(lib().aidw_tune(h, int(m), int(n), int(k), float(budget_s), ctypes.byref(t)))
    return {"q_per_lane": t.q_per_lane, "max_waves_per_simd": t.max_waves_per_simd,
            "split_segments": t.split_segments, "speculate": t.speculate}


def aidw_tune_save(h, path) -> int:
    return lib().aidw_tune_save(h, str(path).encode())


def aidw_tune_load(h, path) -> int:
    return lib().aidw_tune_load(h, str(path).encode())


def aidw_set_tuning(h, q_per_lane: int = 0, max_waves_per_simd: int = 0,
                    split_segments: int = 0, speculate: int = 0, query_order: int = 0) -> int:
    if not (q_per_lane or max_waves_per_simd or split_segments or speculate or query_order):
        return lib().aidw_set_tuning(h, None)
    t = aidw_tuning(int(q_per_lane), int(max_waves_per_simd), int(split_segments), int(speculate),
                    int(query_order))
    return lib().aidw_set_tuning(h, ctypes.byref(t))


def _problem_array(problems):
    arr = (aidw_problem * len(problems))(*problems)
    return arr


def aidw_batch_create(h, problems) -> int:
    arr = _problem_array(problems)
    b = ctypes.c_void_p()
    check(lib().aidw_batch_create(h, arr, len(problems), ctypes.byref(b)))
    return b.value


def aidw_batch_launch(b, flags: int = 0) -> int:
    return lib().aidw_batch_launch(b, int(flags))


def aidw_batch_destroy(b) -> None:
    lib().aidw_batch_destroy(b)


def aidw_interpolate_batch(h, problems, flags: int = 0) -> int:
    arr = _problem_array(problems)
    return lib().aidw_interpolate_batch(h, arr, len(problems), int(flags))


def aidw_synchronize(h) -> int:
    return lib().aidw_synchronize(h)


def aidw_version() -> int:
    return lib().aidw_version()


def aidw_dataset_register(h, data_xy_ptr, data_z_ptr, m, area) -> int:
    i = ctypes.c_uint64()
    check(lib().aidw_dataset_register(h, data_xy_ptr, data_z_ptr, int(m), float(area),
                                      ctypes.byref(i)))
    return i.value


def aidw_dataset_release(h, dataset_id) -> int:
    return lib().aidw_dataset_release(h, int(dataset_id))


def aidw_server_create(h, arena_bytes=0, streams=0, tick_pair_evals=0.0, max_wait_s=0.0,
                       segment_points=0) -> int:
    opt = aidw_server_options(int(arena_bytes), int(streams), float(tick_pair_evals),
                              float(max_wait_s), int(segment_points))
    s = ctypes.c_void_p()
    check(lib().aidw_server_create(h, ctypes.byref(opt), ctypes.byref(s)))
    return s.value


def aidw_server_destroy(s) -> None:
    lib().aidw_server_destroy(s)


def aidw_server_submit(s, job: aidw_job) -> int:
    t = ctypes.c_uint64()
    check(lib().aidw_server_submit(s, ctypes.byref(job), ctypes.byref(t)))
    return t.value


def aidw_submit(h, job: aidw_job) -> int:
    """Submit to the handle's own serving loop; returns the ticket."""
    t = ctypes.c_uint64()
    check(lib().aidw_submit(h, ctypes.byref(job), ctypes.byref(t)))
    return t.value


def aidw_probe_issue_costs(h):
    """SIMD cycles per wave64 instruction on the handle's device (dict)."""
    c = aidw_issue_costs()
    check(lib().aidw_probe_issue_costs(h, ctypes.byref(c)))
    return {f: getattr(c, f) for f, _ in c._fields_}


def _tickets(fn, s, jobs):
    n = len(jobs)
    arr = (aidw_job * max(n, 1))(*jobs)
    tickets = (ctypes.c_uint64 * max(n, 1))()
    check(fn(s, arr, n, tickets))
    return [tickets[i] for i in range(n)]


def aidw_server_submit_batch(s, jobs):
    """Tickets of the jobs, submitted all or none (raises AidwError)."""
    return _tickets(lib().aidw_server_submit_batch, s, jobs)


def aidw_submit_batch(h, jobs):
    """The same on the handle's own serving loop."""
    return _tickets(lib().aidw_submit_batch, h, jobs)


def aidw_server_poll(s, ticket):
    """(status, job_status, latency_s); status AIDW_EAGAIN while pending."""
    js, lat = ctypes.c_int(), ctypes.c_double()
    st = lib().aidw_server_poll(s, int(ticket), ctypes.byref(js), ctypes.byref(lat))
    return st, js.value, lat.value


def aidw_poll(h, ticket):
    js, lat = ctypes.c_int(), ctypes.c_double()
    st = lib().aidw_poll(h, int(ticket), ctypes.byref(js), ctypes.byref(lat))
    return st, js.value, lat.value


def aidw_server_wait(s, ticket, timeout_s=-1.0):
    js, lat = ctypes.c_int(), ctypes.c_double()
    st = lib().aidw_server_wait(s, int(ticket), float(timeout_s), ctypes.byref(js),
                                ctypes.byref(lat))
    return st, js.value, lat.value


def aidw_wait(h, ticket, timeout_s=-1.0):
    js, lat = ctypes.c_int(), ctypes.c_double()
    st = lib().aidw_wait(h, int(ticket), float(timeout_s), ctypes.byref(js), ctypes.byref(lat))
    return st, js.value, lat.value


def aidw_server_stats(s):
    c = aidw_server_counters()
    st = lib().aidw_server_stats(s, ctypes.byref(c))
    return st, {f: getattr(c, f) for f, _ in c._fields_}


# ---- torch convenience layer ------------------------------------------------

class Context:
    """Owns one aidw handle bound to a device and torch's current stream."""

    def __init__(self, device: int = 0, default_precision: int = AIDW_FP32_SCALED,
                 hbm_budget_bytes: int = 0, tune_path=None, deterministic: int = 0):
        self.device = device
        self.h = aidw_create(device, default_precision, hbm_budget_bytes, tune_path,
                             deterministic)

    def close(self):
        if self.h:
            aidw_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, q_per_lane: int = 0, max_waves_per_simd: int = 0,
                   split_segments: int = 0, speculate: int = 0, query_order: int = 0):
        check(aidw_set_tuning(self.h, q_per_lane, max_waves_per_simd, split_segments, speculate,
                              query_order))

    def bind_current_stream(self):
        import torch

        check(aidw_set_stream(self.h, torch.cuda.current_stream(self.device).cuda_stream))

    def problem(self, data_xy, data_z, query_xy, k, out, alpha_levels=(1, 2, 3, 4, 5),
                R_min=0.0, R_max=2.0, area=None, r_obs=None, alpha=None, knn_idx=None,
                flags=0) -> aidw_problem:
        import torch

        if area is None:
            raise ValueError("area (A of Eq. 2) must be given")
        dt = data_xy.dtype
        prec = {torch.float32: AIDW_FP32_SCALED, torch.float64: AIDW_FP64}.get(dt)
        if prec is None:
            raise TypeError("point arrays must be float32 or float64, got %s" % dt)
        for t in (data_z, query_xy, out):
            if t.dtype != dt:
                raise TypeError("all point arrays and out must share one dtype")
        for t in (data_xy, data_z, query_xy, out, r_obs, alpha, knn_idx):
            if t is not None and (not t.is_cuda or not t.is_contiguous()):
                raise ValueError("tensors must be contiguous and on the GPU")
        m = data_z.numel()
        n = out.numel()
        if data_xy.numel() != 2 * m or query_xy.numel() != 2 * n:
            raise ValueError("data_xy must be [2, m] and query_xy [2, n]")
        p = aidw_problem()
        p.precision = prec
        p.data_xy = data_xy.data_ptr()
        p.data_z = data_z.data_ptr()
        p.m = m
        p.query_xy = query_xy.data_ptr()
        p.n = n
        p.k = int(k)
        p.alpha_levels = (ctypes.c_double * 5)(*[float(a) for a in alpha_levels])
        p.R_min, p.R_max, p.area = float(R_min), float(R_max), float(area)
        p.out = out.data_ptr()
        p.r_obs = r_obs.data_ptr() if r_obs is not None else None
        p.alpha = alpha.data_ptr() if alpha is not None else None
        p.knn_idx = knn_idx.data_ptr() if knn_idx is not None else None
        p.flags = int(flags)
        return p

    def interpolate(self, data_xy, data_z, query_xy, k, alpha_levels=(1, 2, 3, 4, 5),
                    R_min=0.0, R_max=2.0, area=None, diag=False, flags=0, out=None, knn=True):
        """AIDW of the queries over the data (torch tensors on the GPU).

        Returns `out`, or (out, r_obs, alpha, knn_idx) with diag=True; knn=False
        leaves knn_idx None (asking for the indices keeps m unsplit)."""
        import torch

        n = query_xy.shape[-1]
        dev = data_xy.device
        if out is None:
            out = torch.empty(n, dtype=data_xy.dtype, device=dev)
        want_knn = knn
        r_obs = alpha = knn = None
        if diag:
            r_obs = torch.empty(n, dtype=torch.float64, device=dev)
            alpha = torch.empty(n, dtype=torch.float64, device=dev)
            if want_knn:
                knn = torch.empty((n, int(k)), dtype=torch.int32, device=dev)
        self.bind_current_stream()
        p = self.problem(data_xy, data_z, query_xy, k, out, alpha_levels, R_min, R_max, area,
                         r_obs, alpha, knn, flags)
        check(aidw_interpolate_ex(self.h, p))
        if diag:
            return out, r_obs, alpha, knn
        return out


def make_job(query_xy, k, out, alpha_levels=(1, 2, 3, 4, 5), R_min=0.0, R_max=2.0,
             dataset=0, data_xy=None, data_z=None, area=None, r_obs=None, alpha=None,
             knn_idx=None):
    """aidw_job over torch tensors on the GPU: a registered dataset id, or
    data_xy/data_z/area.  float32 tensors give an FP32-scaled job, float64
    tensors an FP64 one."""
    import torch

    j = aidw_job()
    j.dataset = int(dataset)
    if not dataset:
        if data_xy is None or data_z is None or area is None:
            raise ValueError("give a dataset id or data_xy, data_z and area")
        j.data_xy = data_xy.data_ptr()
        j.data_z = data_z.data_ptr()
        j.m = data_z.numel()
        j.area = float(area)
    prec = {torch.float32: AIDW_FP32_SCALED, torch.float64: AIDW_FP64}.get(out.dtype)
    if prec is None:
        raise TypeError("out must be float32 or float64, got %s" % out.dtype)
    j.precision = prec
    j.query_xy = query_xy.data_ptr()
    j.n = out.numel()
    j.k = int(k)
    j.alpha_levels = (ctypes.c_double * 5)(*[float(a) for a in alpha_levels])
    j.R_min, j.R_max = float(R_min), float(R_max)
    j.out = out.data_ptr()
    j.r_obs = r_obs.data_ptr() if r_obs is not None else None
    j.alpha = alpha.data_ptr() if alpha is not None else None
    j.knn_idx = knn_idx.data_ptr() if knn_idx is not None else None
    return j


def idw(ctx, data_xy, data_z, query_xy, power, out=None):
    """Standard IDW (constant power) over torch tensors on the GPU."""
    import torch

    n = query_xy.shape[-1]
    if out is None:
        out = torch.empty(n, dtype=data_xy.dtype, device=data_xy.device)
    ctx.bind_current_stream()
    p = ctx.problem(data_xy, data_z, query_xy, 1, out, area=1.0)
    check(aidw_idw(ctx.h, p, power))
    return out


def to_device(inst, device="cuda"):
    """Planar device tensors (data_xy [2, m], data_z [m], query_xy [2, n]) of a
    workloads.Instance."""
    import torch

    return (torch.from_numpy(inst.data_xy()).to(device),
            torch.from_numpy(inst.data_z.copy()).to(device),
            torch.from_numpy(inst.query_xy()).to(device))
