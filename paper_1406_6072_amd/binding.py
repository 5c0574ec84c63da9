"""Thin ctypes binding of the C ABI in include/cefield.h.

Argument marshalling only: every step of the generator runs in the HIP
library.  Device buffers are torch CUDA tensors (their data_ptr is passed);
streams default to torch's current stream.  Sizes and dtypes of the tensors
are checked here so the library never receives an undersized buffer.  If the
shared library has not been built, importing fails loudly: there is no CPU
fallback.
"""

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcefield.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libcefield.so is not built; run __graft_entry__.build() (hipcc for gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

OK, E_INVALID, E_NOT_PSD, E_OOM, E_UNSUPPORTED, E_DEVICE, E_SAMPLER = range(7)
F32, F64 = 0, 1
XI_TABLE, XI_EXP, XI_POWEXP = 0, 1, 2
XI_CELL_AVERAGE, XI_LOGNORMAL = 1, 2
MAP_FIELD, MAP_COUNTS_DELTAG = 0, 1

c_void_p = ctypes.c_void_p
c_i32, c_i64, c_u32, c_u64, c_f64, c_size = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                              ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t)


class Geometry(ctypes.Structure):
    _fields_ = [("ndim", c_i32), ("n", c_i64 * 3), ("h", c_f64 * 3)]


class Xi(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("p", c_f64 * 4), ("table", ctypes.POINTER(c_f64)), ("transform", c_i32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("lambda_min", c_f64), ("lambda_max", c_f64), ("sigma2", c_f64),
                ("n_negative", c_i64), ("n_clamped", c_i64), ("device_bytes", c_size)]


class BatchItem(ctypes.Structure):
    _fields_ = [("plan", c_void_p), ("seed", c_u64), ("request_id", c_u32), ("first_realization", c_u64),
                ("count", c_i64), ("nbar", c_f64), ("nbins", c_i32), ("out_pk", c_void_p),
                ("out_counts", c_void_p), ("out_ntot", c_void_p), ("out_cov", c_void_p), ("out_cnorm", c_void_p),
                ("kedges", c_void_p), ("out_fields", c_void_p), ("out_delta", c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", c_i32), ("hbm_budget_bytes", c_size), ("plan_cache_bytes", c_size), ("max_group", c_i32)]


class Request(ctypes.Structure):
    _fields_ = [("geom", Geometry), ("xi", Xi), ("precision", c_i32), ("seed", c_u64), ("request_id", c_u32),
                ("realizations", c_i64), ("nbar", c_f64), ("nbins", c_i32), ("out_pk", c_void_p),
                ("out_counts", c_void_p), ("out_ntot", c_void_p), ("out_cov", c_void_p), ("kedges", c_void_p),
                ("out_fields", c_void_p), ("out_delta", c_void_p)]


class Schedule(ctypes.Structure):
    _fields_ = [("lines_noise", c_i32), ("lines_inner", c_i32), ("lines_last", c_i32), ("lines_bins", c_i32),
                ("noise_order", c_i32), ("noise_block", c_i32), ("noise_pairs", c_i32), ("reserved", c_i32),
                ("bin_lds", c_i64), ("ms", c_f64),
                ("default_ms", c_f64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("failed", c_i64), ("cache_hits", c_i64),
                ("cache_misses", c_i64), ("admission_stalls", c_i64), ("queued", c_i64), ("p50_ms", c_f64),
                ("p99_ms", c_f64), ("elapsed_s", c_f64), ("held_bytes", c_size), ("launches", c_i64),
                ("largest_group", c_i64)]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_status_string = _sig("ce_status_string", ctypes.c_char_p, c_i32)
_version = _sig("ce_version", ctypes.c_char_p)
_ctx_create = _sig("ce_ctx_create", c_i32, c_i32, c_size, ctypes.POINTER(c_void_p))
_ctx_destroy = _sig("ce_ctx_destroy", None, c_void_p)
_ctx_check = _sig("ce_ctx_check", c_i32, c_void_p, c_void_p)
_ctx_trim = _sig("ce_ctx_trim", c_i32, c_void_p)
_ctx_set_option = _sig("ce_ctx_set_option", c_i32, c_void_p, c_i32, c_i64)
_ctx_set_profiling = _sig("ce_ctx_set_profiling", c_i32, c_void_p, c_i32)
_ctx_profile_read = _sig("ce_ctx_profile_read", c_i32, c_void_p, c_i32, c_void_p, c_void_p, c_void_p,
                         ctypes.POINTER(c_i32))
_plan_embedding = _sig("ce_plan_embedding", c_i32, c_void_p, ctypes.POINTER(Geometry), ctypes.POINTER(Xi), c_i32,
                       c_f64, ctypes.POINTER(c_void_p), ctypes.POINTER(PlanInfo))
_plan_release = _sig("ce_plan_release", None, c_void_p)
_plan_periodic = _sig("ce_plan_periodic", c_i32, c_void_p, ctypes.POINTER(Geometry), c_i64, ctypes.POINTER(Xi), c_i32,
                      c_f64, ctypes.POINTER(c_void_p), ctypes.POINTER(PlanInfo))
_xi_lag_octant = _sig("ce_xi_lag_octant", c_i32, c_void_p, ctypes.POINTER(Geometry), ctypes.POINTER(Xi), c_void_p,
                      c_void_p)
_plan_get_info = _sig("ce_plan_get_info", c_i32, c_void_p, ctypes.POINTER(PlanInfo))
_plan_eigenvalues = _sig("ce_plan_eigenvalues", c_i32, c_void_p, c_void_p, c_void_p)
_generate_fields = _sig("ce_generate_fields", c_i32, c_void_p, c_void_p, c_u64, c_u32, c_u64, c_i64, c_void_p,
                        c_void_p)
_lognormal_poisson = _sig("ce_lognormal_poisson", c_i32, c_void_p, c_void_p, c_void_p, c_i64, c_f64, c_void_p, c_u64,
                          c_u32, c_u64, c_void_p, c_void_p, c_void_p, c_void_p)
_estimate_pk = _sig("ce_estimate_pk", c_i32, c_void_p, ctypes.POINTER(Geometry), c_i32, c_i32, c_void_p, c_i64,
                    c_void_p, c_void_p, c_i32, c_void_p, c_void_p, c_void_p, c_void_p)
_estimate_pk_edges = _sig("ce_estimate_pk_edges", c_i32, c_void_p, ctypes.POINTER(Geometry), c_i32, c_i32, c_void_p,
                          c_i64, c_void_p, c_void_p, c_i32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p)
_pk_covariance = _sig("ce_pk_covariance", c_i32, c_void_p, c_void_p, c_i64, c_i32, c_void_p, c_void_p, c_void_p)
_cumulative_information = _sig("ce_cumulative_information", c_i32, c_void_p, c_void_p, c_i32, c_void_p, c_void_p)
_cic_predict = _sig("ce_cic_predict", c_i32, c_void_p, c_void_p, c_i64, c_f64, c_f64, c_i32, c_void_p, c_void_p)
_cic_histogram = _sig("ce_cic_histogram", c_i32, c_void_p, c_void_p, c_i64, c_i64, c_void_p, c_i32, c_void_p, c_void_p)
_astar_map = _sig("ce_astar_map", c_i32, c_void_p, c_void_p, c_i64, c_i64, c_void_p, c_f64, c_f64, c_i32, c_i32,
                  c_void_p, c_void_p, c_void_p)
_pipeline_run = _sig("ce_pipeline_run", c_i32, c_void_p, c_void_p, c_u64, c_u32, c_u64, c_i64, c_f64, c_i32,
                     c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p)
_pipeline_noalloc = _sig("ce_pipeline_run_noalloc", c_i32, c_void_p, c_void_p, c_u64, c_u32, c_u64, c_i64, c_f64,
                         c_i32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p)
_graph_create = _sig("ce_pipeline_graph_create", c_i32, c_void_p, c_void_p, c_u64, c_u32, c_u64, c_i64, c_f64, c_i32,
                     c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_void_p))
_graph_launch = _sig("ce_pipeline_graph_launch", c_i32, c_void_p, c_void_p)
_graph_destroy = _sig("ce_pipeline_graph_destroy", None, c_void_p)
_pipeline_masked = _sig("ce_pipeline_run_masked", c_i32, c_void_p, c_void_p, c_void_p, c_u64, c_u32, c_u64, c_i64,
                        c_f64, c_i32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p)
_pipeline_edges = _sig("ce_pipeline_run_edges", c_i32, c_void_p, c_void_p, c_void_p, c_u64, c_u32, c_u64, c_i64,
                       c_f64, c_i32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                       c_void_p)
_mask_prepare = _sig("ce_mask_prepare", c_i32, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_void_p))
_mask_release = _sig("ce_mask_release", None, c_void_p)
_pipeline_prepared = _sig("ce_pipeline_run_prepared", c_i32, c_void_p, c_void_p, c_void_p, c_void_p, c_u64, c_u32,
                          c_u64, c_i64, c_f64, c_i32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                          c_void_p, c_void_p, c_void_p)
_pipeline_batch = _sig("ce_pipeline_run_batch", c_i32, c_void_p, ctypes.POINTER(BatchItem), c_i64, c_void_p)
_server_create = _sig("ce_server_create", c_i32, c_i32, ctypes.POINTER(ServerConfig), ctypes.POINTER(c_void_p))
_server_submit = _sig("ce_server_submit", c_i32, c_void_p, ctypes.POINTER(Request), ctypes.POINTER(c_u64))
_server_submit_many = _sig("ce_server_submit_many", c_i32, c_void_p, ctypes.POINTER(Request), c_i64,
                           ctypes.POINTER(c_u64))
_server_poll = _sig("ce_server_poll", c_i32, c_void_p, c_u64, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                    ctypes.POINTER(c_f64))
_server_cancel = _sig("ce_server_cancel", c_i32, c_void_p, c_u64)
_server_drain = _sig("ce_server_drain", c_i32, c_void_p, c_i32, c_void_p, c_void_p, c_void_p, c_void_p,
                     ctypes.POINTER(c_i32))
_server_stats = _sig("ce_server_stats_read", c_i32, c_void_p, ctypes.POINTER(ServerStats))
_server_destroy = _sig("ce_server_destroy", None, c_void_p)
_autotune = _sig("ce_autotune", c_i32, c_void_p, c_void_p, c_i64, c_f64, c_i32, c_i32, ctypes.POINTER(Schedule))
_schedule_set = _sig("ce_schedule_set", c_i32, c_void_p, ctypes.POINTER(Geometry), c_i32, ctypes.POINTER(Schedule))
_schedule_get = _sig("ce_schedule_get", c_i32, c_void_p, ctypes.POINTER(Geometry), c_i32, ctypes.POINTER(Schedule))
_schedule_save = _sig("ce_schedule_save", c_i32, c_void_p, ctypes.c_char_p)
_schedule_load = _sig("ce_schedule_load", c_i32, c_void_p, ctypes.c_char_p)
_shell_table = _sig("ce_shell_table", c_i32, ctypes.POINTER(Geometry), c_i32, c_void_p, c_void_p)
_fft_factors = _sig("ce_fft_factors", c_i32, c_i32, c_void_p, c_void_p)
_debug_philox = _sig("ce_debug_philox", c_i32, c_u64, c_void_p, c_i64, c_void_p, c_void_p)
_debug_noise = _sig("ce_debug_noise", c_i32, c_void_p, c_u64, c_u32, c_u64, c_void_p, c_void_p)

EXPORTED = ["ce_status_string", "ce_version", "ce_ctx_create", "ce_ctx_destroy", "ce_ctx_check", "ce_ctx_trim",
            "ce_ctx_set_option", "ce_ctx_set_profiling", "ce_ctx_profile_read",
            "ce_plan_embedding", "ce_plan_release", "ce_plan_get_info", "ce_plan_eigenvalues", "ce_xi_lag_octant",
            "ce_plan_periodic",
            "ce_generate_fields", "ce_lognormal_poisson", "ce_estimate_pk", "ce_estimate_pk_edges", "ce_pk_covariance",
            "ce_cic_histogram", "ce_cic_predict", "ce_astar_map", "ce_cumulative_information",
            "ce_pipeline_run", "ce_pipeline_run_noalloc", "ce_pipeline_run_edges", "ce_pipeline_run_masked", "ce_mask_prepare",
            "ce_mask_release", "ce_pipeline_run_prepared", "ce_pipeline_run_batch", "ce_pipeline_graph_create", "ce_pipeline_graph_launch",
            "ce_pipeline_graph_destroy",
            "ce_server_create", "ce_server_submit", "ce_server_submit_many", "ce_server_poll", "ce_server_drain", "ce_server_cancel",
            "ce_server_stats_read", "ce_server_destroy", "ce_autotune", "ce_schedule_set", "ce_schedule_get",
            "ce_schedule_save", "ce_schedule_load", "ce_shell_table", "ce_fft_factors", "ce_debug_philox", "ce_debug_noise"]


class CeError(RuntimeError):
    def __init__(self, status, where):
        super().__init__("%s: %s (status %d)" % (where, status_string(status), status))
        self.status = status


class NotPSDError(CeError):
    def __init__(self, status, where, info):
        super().__init__(status, where)
        self.info = info


def status_string(s):
    return _status_string(int(s)).decode()


def version():
    return _version().decode()


def _check(st, where):
    if st != OK:
        raise CeError(st, where)


def _stream(stream):
    if stream is None:
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return c_void_p(stream.cuda_stream)
    return c_void_p(int(stream))


def _ptr(t, dtype=None, numel=None, name="buffer"):
    """data_ptr of a CUDA tensor after dtype / contiguity / size checks (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), numel))
    return c_void_p(t.data_ptr())


def geometry(n, h=None):
    n = tuple(int(x) for x in n)
    h = tuple(float(x) for x in (h if h is not None else (1.0,) * len(n)))
    g = Geometry()
    g.ndim = len(n)
    for i in range(3):
        g.n[i] = n[i] if i < len(n) else 1
        g.h[i] = h[i] if i < len(h) else 1.0
    return g


def xi_spec(xi):
    """ctypes Xi from the dict form used by the tests ({'kind': 'exp'|'powexp'|'table', ...})."""
    x = Xi()
    kind = xi["kind"]
    keep = None
    if kind == "exp":
        x.kind = XI_EXP
        x.p[0], x.p[1] = float(xi["sigma2"]), float(xi["a"])
    elif kind == "powexp":
        x.kind = XI_POWEXP
        x.p[0], x.p[1] = float(xi["sigma2"]), float(xi["r0"])
        x.p[2], x.p[3] = float(xi.get("gamma", 1.8)), float(xi.get("rc", 0.0))
    elif kind == "table":
        import numpy as np
        keep = np.ascontiguousarray(xi["table"], dtype=np.float64)
        x.kind = XI_TABLE
        x.table = keep.ctypes.data_as(ctypes.POINTER(c_f64))
    else:
        raise ValueError("unknown xi kind %r" % kind)
    x.transform = (XI_CELL_AVERAGE if xi.get("cell_average") else 0) | (XI_LOGNORMAL if xi.get("lognormal") else 0)
    return x, keep


def _info_dict(pi):
    return dict(lambda_min=pi.lambda_min, lambda_max=pi.lambda_max, sigma2=pi.sigma2,
                n_negative=pi.n_negative, n_clamped=pi.n_clamped, device_bytes=pi.device_bytes)


# ---- entry points (same names as the C ABI, without the ce_ prefix) ----------

def ctx_create(device=0, hbm_budget_bytes=0):
    h = c_void_p()
    _check(_ctx_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)), "ce_ctx_create")
    return h


def ctx_destroy(ctx):
    _ctx_destroy(ctx)


def ctx_check(ctx, stream=None):
    return _ctx_check(ctx, None if stream is None else _stream(stream))


def ctx_trim(ctx):
    _check(_ctx_trim(ctx), "ce_ctx_trim")


OPT_UNPRUNED = 1
CIC_MAX_BINS = 4096
OPT_LINES_NOISE, OPT_LINES_INNER, OPT_LINES_LAST, OPT_LINES_BINS, OPT_NOISE_ORDER, OPT_BIN_LDS = 2, 3, 4, 5, 6, 7
OPT_NOISE_BLOCK = 8
OPT_BATCH_LANES = 9
OPT_NOISE_PAIRS = 10


def ctx_set_option(ctx, option, value):
    _check(_ctx_set_option(ctx, int(option), int(value)), "ce_ctx_set_option")


def ctx_set_profiling(ctx, enable):
    _check(_ctx_set_profiling(ctx, 1 if enable else 0), "ce_ctx_set_profiling")


def ctx_profile_read(ctx, max_entries=64):
    """{kernel name: (total ms, launches)} since the previous read."""
    names = ctypes.create_string_buffer(32 * max_entries)
    ms = (c_f64 * max_entries)()
    nl = (c_i64 * max_entries)()
    n = c_i32()
    _check(_ctx_profile_read(ctx, max_entries, names, ms, nl, ctypes.byref(n)), "ce_ctx_profile_read")
    out = {}
    for i in range(n.value):
        nm = names.raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode()
        out[nm] = (ms[i], nl[i])
    return out


class Plan:
    """Owning handle of a ce_plan with the geometry it was built for."""

    def __init__(self, handle, n, h, precision, info, M=None):
        self.handle, self.n, self.h, self.precision, self.info = handle, tuple(n), tuple(h), precision, info
        # periodic side per axis: 2N (embedding) or the box side (k-space comparator)
        self.M = tuple(2 * x for x in self.n) if M is None else tuple(M)

    @property
    def cells(self):
        c = 1
        for x in self.n:
            c *= x
        return c

    @property
    def embedding_cells(self):
        c = 1
        for x in self.M:
            c *= x
        return c

    @property
    def octant(self):
        """Shape of the eigenvalue octant, (M_i / 2 + 1) per axis."""
        return tuple(m // 2 + 1 for m in self.M)

    @property
    def dtype(self):
        return torch.float64 if self.precision == F64 else torch.float32

    def release(self):
        if self.handle:
            _plan_release(self.handle)
            self.handle = None


def plan_embedding(ctx, n, h, xi, precision, neg_tol=-1.0):
    g = geometry(n, h)
    x, keep = xi_spec(xi)
    out = c_void_p()
    pi = PlanInfo()
    st = _plan_embedding(ctx, ctypes.byref(g), ctypes.byref(x), int(precision), float(neg_tol), ctypes.byref(out),
                         ctypes.byref(pi))
    del keep
    if st == E_NOT_PSD:
        raise NotPSDError(st, "ce_plan_embedding", _info_dict(pi))
    _check(st, "ce_plan_embedding")
    return Plan(out, g.n[:g.ndim], g.h[:g.ndim], int(precision), _info_dict(pi))


def plan_periodic(ctx, n, h, box, xi, precision, neg_tol=-1.0):
    """k-space comparator plan: survey n in the corner of a periodic box of `box` cells per axis."""
    g = geometry(n, h)
    x, keep = xi_spec(xi)
    out = c_void_p()
    pi = PlanInfo()
    st = _plan_periodic(ctx, ctypes.byref(g), int(box), ctypes.byref(x), int(precision), float(neg_tol),
                        ctypes.byref(out), ctypes.byref(pi))
    del keep
    if st == E_NOT_PSD:
        raise NotPSDError(st, "ce_plan_periodic", _info_dict(pi))
    _check(st, "ce_plan_periodic")
    return Plan(out, g.n[:g.ndim], g.h[:g.ndim], int(precision), _info_dict(pi), M=(int(box),) * g.ndim)


def xi_lag_octant(ctx, n, h, xi, out, stream=None):
    """The (transformed) lag octant of xi on the grid (n, h) into a float64 CUDA tensor."""
    g = geometry(n, h)
    x, keep = xi_spec(xi)
    noct = 1
    for v in n:
        noct *= int(v) + 1
    _check(_xi_lag_octant(ctx, ctypes.byref(g), ctypes.byref(x), _ptr(out, torch.float64, noct, "out"),
                          _stream(stream)), "ce_xi_lag_octant")
    del keep


def plan_release(plan):
    plan.release()


def plan_get_info(plan):
    pi = PlanInfo()
    _check(_plan_get_info(plan.handle, ctypes.byref(pi)), "ce_plan_get_info")
    return _info_dict(pi)


def plan_eigenvalues(plan, out, stream=None):
    noct = 1
    for x in plan.octant:
        noct *= x
    _check(_plan_eigenvalues(plan.handle, _ptr(out, torch.float64, noct, "out"), _stream(stream)),
           "ce_plan_eigenvalues")


def generate_fields(ctx, plan, seed, request_id, first_realization, count, out_fields, stream=None):
    _check(_generate_fields(ctx, plan.handle, int(seed), int(request_id), int(first_realization), int(count),
                            _ptr(out_fields, plan.dtype, count * plan.cells, "out_fields"), _stream(stream)),
           "ce_generate_fields")


def lognormal_poisson(ctx, plan, fields, count, nbar, mask_f, seed, request_id, first_realization,
                      out_delta, out_counts, out_ntot, stream=None):
    cells = plan.cells
    _check(_lognormal_poisson(ctx, plan.handle, _ptr(fields, plan.dtype, count * cells, "fields"), int(count),
                              float(nbar), _ptr(mask_f, torch.float32, cells, "mask_f"), int(seed), int(request_id),
                              int(first_realization), _ptr(out_delta, plan.dtype, count * cells, "out_delta"),
                              _ptr(out_counts, torch.int32, count * cells, "out_counts"),
                              _ptr(out_ntot, torch.int64, count, "out_ntot"), _stream(stream)),
           "ce_lognormal_poisson")


def estimate_pk(ctx, n, h, precision, kind, maps, count, ntot, mask_f, nbins, out_pk, out_nmodes=None,
                out_kmean=None, stream=None, edges=None):
    """edges: optional host sequence of nbins + 1 ascending |k| shell edges (ce_estimate_pk_edges)."""
    g = geometry(n, h)
    cells = 1
    for x in n:
        cells *= int(x)
    mdt = torch.int32 if kind == MAP_COUNTS_DELTAG else (torch.float64 if precision == F64 else torch.float32)
    args = (_ptr(maps, mdt, count * cells, "maps"), int(count), _ptr(ntot, torch.int64, count, "ntot"),
            _ptr(mask_f, torch.float32, cells, "mask"), int(nbins))
    outs = (_ptr(out_pk, torch.float64, count * nbins, "out_pk"), _ptr(out_nmodes, torch.int64, nbins, "out_nmodes"),
            _ptr(out_kmean, torch.float64, nbins, "out_kmean"), _stream(stream))
    if edges is None:
        _check(_estimate_pk(ctx, ctypes.byref(g), int(precision), int(kind), *args, *outs), "ce_estimate_pk")
        return
    import numpy as np
    e = np.ascontiguousarray(edges, dtype=np.float64)
    if e.size != nbins + 1:
        raise ValueError("edges must hold nbins + 1 values")
    _check(_estimate_pk_edges(ctx, ctypes.byref(g), int(precision), int(kind), *args,
                              e.ctypes.data_as(c_void_p), *outs), "ce_estimate_pk_edges")


def pk_covariance(ctx, pk, count, nbins, out_cov, out_cnorm, stream=None):
    _check(_pk_covariance(ctx, _ptr(pk, torch.float64, count * nbins, "pk"), int(count), int(nbins),
                          _ptr(out_cov, torch.float64, nbins * nbins, "out_cov"),
                          _ptr(out_cnorm, torch.float64, nbins * nbins, "out_cnorm"), _stream(stream)),
           "ce_pk_covariance")


def cumulative_information(ctx, cnorm, nbins, out_info, stream=None):
    _check(_cumulative_information(ctx, _ptr(cnorm, torch.float64, nbins * nbins, "cnorm"), int(nbins),
                                   _ptr(out_info, torch.float64, nbins, "out_info"), _stream(stream)),
           "ce_cumulative_information")


def cic_predict(ctx, mask_f, cells, nbar, sigma2_A, nhist, out_pred, stream=None):
    _check(_cic_predict(ctx, _ptr(mask_f, torch.float32, cells, "mask_f"), int(cells), float(nbar), float(sigma2_A),
                        int(nhist), _ptr(out_pred, torch.float64, nhist, "out_pred"), _stream(stream)),
           "ce_cic_predict")


def cic_histogram(ctx, counts, cells, count, mask_f, nhist, out_hist, stream=None):
    _check(_cic_histogram(ctx, _ptr(counts, torch.int32, count * cells, "counts"), int(cells), int(count),
                          _ptr(mask_f, torch.float32, cells, "mask_f"), int(nhist),
                          _ptr(out_hist, torch.int64, count * nhist, "out_hist"), _stream(stream)),
           "ce_cic_histogram")


def astar_map(ctx, counts, cells, count, mask_f, nbar, sigma2_A, subtract_mean, precision, out_map,
              out_mean=None, stream=None):
    mdt = torch.float64 if precision == F64 else torch.float32
    _check(_astar_map(ctx, _ptr(counts, torch.int32, count * cells, "counts"), int(cells), int(count),
                      _ptr(mask_f, torch.float32, cells, "mask_f"), float(nbar), float(sigma2_A),
                      1 if subtract_mean else 0, int(precision), _ptr(out_map, mdt, count * cells, "out_map"),
                      _ptr(out_mean, torch.float64, count, "out_mean"), _stream(stream)),
           "ce_astar_map")


def pipeline_run(ctx, plan, seed, request_id, first_realization, count, nbar, nbins, out_pk, out_fields=None,
                 out_delta=None, out_counts=None, out_ntot=None, out_cov=None, out_cnorm=None, stream=None):
    cells = plan.cells
    _check(_pipeline_run(ctx, plan.handle, int(seed), int(request_id), int(first_realization), int(count),
                         float(nbar), int(nbins), _ptr(out_fields, plan.dtype, count * cells, "out_fields"),
                         _ptr(out_delta, plan.dtype, count * cells, "out_delta"),
                         _ptr(out_counts, torch.int32, count * cells, "out_counts"),
                         _ptr(out_ntot, torch.int64, count, "out_ntot"),
                         _ptr(out_pk, torch.float64, count * nbins, "out_pk"),
                         _ptr(out_cov, torch.float64, nbins * nbins, "out_cov"),
                         _ptr(out_cnorm, torch.float64, nbins * nbins, "out_cnorm"), _stream(stream)),
           "ce_pipeline_run")


def pipeline_run_noalloc(ctx, plan, seed, request_id, first_realization, count, nbar, nbins, out_pk, out_fields=None,
                         out_delta=None, out_counts=None, out_ntot=None, out_cov=None, out_cnorm=None, stream=None):
    """ce_pipeline_run with every scratch buffer in the library's static device array (no allocation)."""
    cells = plan.cells
    _check(_pipeline_noalloc(ctx, plan.handle, int(seed), int(request_id), int(first_realization), int(count),
                             float(nbar), int(nbins), _ptr(out_fields, plan.dtype, count * cells, "out_fields"),
                             _ptr(out_delta, plan.dtype, count * cells, "out_delta"),
                             _ptr(out_counts, torch.int32, count * cells, "out_counts"),
                             _ptr(out_ntot, torch.int64, count, "out_ntot"),
                             _ptr(out_pk, torch.float64, count * nbins, "out_pk"),
                             _ptr(out_cov, torch.float64, nbins * nbins, "out_cov"),
                             _ptr(out_cnorm, torch.float64, nbins * nbins, "out_cnorm"), _stream(stream)),
           "ce_pipeline_run_noalloc")


def pipeline_run_edges(ctx, plan, seed, request_id, first_realization, count, nbar, nbins, edges, out_pk,
                       out_fields=None, out_delta=None, out_counts=None, out_ntot=None, out_cov=None, out_cnorm=None,
                       stream=None, mask=None):
    """The fused path with user shell edges (host sequence of nbins + 1 ascending |k| values),
    on a masked survey when mask (float32 CUDA tensor of N^d surface fractions) is given."""
    import numpy as np
    e = np.ascontiguousarray(edges, dtype=np.float64)
    if e.size != nbins + 1:
        raise ValueError("edges must hold nbins + 1 values")
    cells = plan.cells
    _check(_pipeline_edges(ctx, plan.handle, _ptr(mask, torch.float32, cells, "mask"), int(seed), int(request_id), int(first_realization), int(count),
                           float(nbar), int(nbins), e.ctypes.data_as(c_void_p),
                           _ptr(out_fields, plan.dtype, count * cells, "out_fields"),
                           _ptr(out_delta, plan.dtype, count * cells, "out_delta"),
                           _ptr(out_counts, torch.int32, count * cells, "out_counts"),
                           _ptr(out_ntot, torch.int64, count, "out_ntot"),
                           _ptr(out_pk, torch.float64, count * nbins, "out_pk"),
                           _ptr(out_cov, torch.float64, nbins * nbins, "out_cov"),
                           _ptr(out_cnorm, torch.float64, nbins * nbins, "out_cnorm"), _stream(stream)),
           "ce_pipeline_run_edges")


def pipeline_run_masked(ctx, plan, mask, seed, request_id, first_realization, count, nbar, nbins, out_pk,
                        out_fields=None, out_delta=None, out_counts=None, out_ntot=None, out_cov=None, out_cnorm=None,
                        stream=None):
    """The fused path on a masked survey; mask: float32 CUDA tensor of N^d surface fractions."""
    cells = plan.cells
    _check(_pipeline_masked(ctx, plan.handle, _ptr(mask, torch.float32, cells, "mask"), int(seed), int(request_id),
                            int(first_realization), int(count), float(nbar), int(nbins),
                            _ptr(out_fields, plan.dtype, count * cells, "out_fields"),
                            _ptr(out_delta, plan.dtype, count * cells, "out_delta"),
                            _ptr(out_counts, torch.int32, count * cells, "out_counts"),
                            _ptr(out_ntot, torch.int64, count, "out_ntot"),
                            _ptr(out_pk, torch.float64, count * nbins, "out_pk"),
                            _ptr(out_cov, torch.float64, nbins * nbins, "out_cov"),
                            _ptr(out_cnorm, torch.float64, nbins * nbins, "out_cnorm"), _stream(stream)),
           "ce_pipeline_run_masked")


def mask_prepare(ctx, plan, mask, stream=None):
    """Handle holding sum(f) and the window transform of a mask (float32 CUDA tensor)."""
    m = c_void_p()
    _check(_mask_prepare(ctx, plan.handle, _ptr(mask, torch.float32, plan.cells, "mask"), _stream(stream),
                         ctypes.byref(m)), "ce_mask_prepare")
    return m


def mask_release(m):
    _mask_release(m)


def pipeline_run_prepared(ctx, plan, mask, prepared, seed, request_id, first_realization, count, nbar, nbins, out_pk,
                          edges=None, out_fields=None, out_delta=None, out_counts=None, out_ntot=None, out_cov=None,
                          out_cnorm=None, stream=None):
    """The masked fused path with a prepared mask (and optional shell edges)."""
    import numpy as np
    e = None
    if edges is not None:
        e = np.ascontiguousarray(edges, dtype=np.float64)
        if e.size != nbins + 1:
            raise ValueError("edges must hold nbins + 1 values")
    cells = plan.cells
    _check(_pipeline_prepared(ctx, plan.handle, _ptr(mask, torch.float32, cells, "mask"), prepared, int(seed),
                              int(request_id), int(first_realization), int(count), float(nbar), int(nbins),
                              None if e is None else e.ctypes.data_as(c_void_p),
                              _ptr(out_fields, plan.dtype, count * cells, "out_fields"),
                              _ptr(out_delta, plan.dtype, count * cells, "out_delta"),
                              _ptr(out_counts, torch.int32, count * cells, "out_counts"),
                              _ptr(out_ntot, torch.int64, count, "out_ntot"),
                              _ptr(out_pk, torch.float64, count * nbins, "out_pk"),
                              _ptr(out_cov, torch.float64, nbins * nbins, "out_cov"),
                              _ptr(out_cnorm, torch.float64, nbins * nbins, "out_cnorm"), _stream(stream)),
           "ce_pipeline_run_prepared")


class PreparedBatch:
    """The C item array of a batch, marshalled once (tensors are checked and their addresses
    taken here); pipeline_run_batch accepts it in place of the item list, so repeated calls
    on the same buffers cost one C call each.  The tensors must outlive the object."""

    def __init__(self, items):
        import numpy as np
        self.n = len(items)
        self.arr = (BatchItem * max(self.n, 1))()
        self.keep = []
        for k, it in enumerate(items):
            plan, count, nb = it["plan"], int(it["count"]), int(it["nbins"])
            a = self.arr[k]
            a.plan = plan.handle
            a.seed, a.request_id = int(it.get("seed", 0)), int(it.get("request_id", 0))
            a.first_realization, a.count, a.nbar, a.nbins = int(it.get("first_realization", 0)), count, \
                float(it["nbar"]), nb
            a.out_pk = _ptr(it["out_pk"], torch.float64, count * nb, "out_pk")
            a.out_counts = _ptr(it.get("out_counts"), torch.int32, count * plan.cells, "out_counts")
            a.out_ntot = _ptr(it.get("out_ntot"), torch.int64, count, "out_ntot")
            a.out_cov = _ptr(it.get("out_cov"), torch.float64, nb * nb, "out_cov")
            a.out_cnorm = _ptr(it.get("out_cnorm"), torch.float64, nb * nb, "out_cnorm")
            a.out_fields = _ptr(it.get("out_fields"), plan.dtype, count * plan.cells, "out_fields")
            a.out_delta = _ptr(it.get("out_delta"), plan.dtype, count * plan.cells, "out_delta")
            if it.get("edges") is not None:
                e = np.ascontiguousarray(it["edges"], dtype=np.float64)
                if e.size != nb + 1:
                    raise ValueError("edges must hold nbins + 1 values")
                self.keep.append(e)
                a.kedges = e.ctypes.data


def prepare_batch(items):
    return PreparedBatch(items)


def pipeline_run_batch(ctx, items, stream=None):
    """items: a PreparedBatch, or dicts with plan, seed, request_id, first_realization, count,
    nbar, nbins, out_pk and optional out_counts, out_ntot, out_cov, out_cnorm, out_fields,
    out_delta (device tensors) and edges (host sequence of nbins + 1 shell edges)."""
    pb = items if isinstance(items, PreparedBatch) else PreparedBatch(items)
    _check(_pipeline_batch(ctx, pb.arr, pb.n, _stream(stream)), "ce_pipeline_run_batch")


def pipeline_graph_create(ctx, plan, seed, request_id, first_realization, count, nbar, nbins, out_pk,
                          out_fields=None, out_delta=None, out_counts=None, out_ntot=None, out_cov=None,
                          out_cnorm=None):
    cells = plan.cells
    g = c_void_p()
    _check(_graph_create(ctx, plan.handle, int(seed), int(request_id), int(first_realization), int(count),
                         float(nbar), int(nbins), _ptr(out_fields, plan.dtype, count * cells, "out_fields"),
                         _ptr(out_delta, plan.dtype, count * cells, "out_delta"),
                         _ptr(out_counts, torch.int32, count * cells, "out_counts"),
                         _ptr(out_ntot, torch.int64, count, "out_ntot"),
                         _ptr(out_pk, torch.float64, count * nbins, "out_pk"),
                         _ptr(out_cov, torch.float64, nbins * nbins, "out_cov"),
                         _ptr(out_cnorm, torch.float64, nbins * nbins, "out_cnorm"), ctypes.byref(g)),
           "ce_pipeline_graph_create")
    return g


def pipeline_graph_launch(graph, stream=None):
    _check(_graph_launch(graph, _stream(stream)), "ce_pipeline_graph_launch")


def pipeline_graph_destroy(graph):
    _graph_destroy(graph)


def server_create(device=0, slots=4, hbm_budget_bytes=0, plan_cache_bytes=0, max_group=0):
    cfg = ServerConfig(int(slots), int(hbm_budget_bytes), int(plan_cache_bytes), int(max_group))
    s = c_void_p()
    _check(_server_create(int(device), ctypes.byref(cfg), ctypes.byref(s)), "ce_server_create")
    return s


def _fill_request(r, n, h, xi, precision, seed, request_id, realizations, nbar, nbins, out_pk,
                  out_counts=None, out_ntot=None, out_cov=None, edges=None, out_fields=None, out_delta=None):
    cells = 1
    for x in n:
        cells *= int(x)
    r.geom = geometry(n, h)
    x, keep = xi_spec(xi)
    r.xi = x
    r.precision = int(precision)
    r.seed, r.request_id, r.realizations, r.nbar, r.nbins = int(seed), int(request_id), int(realizations), \
        float(nbar), int(nbins)
    r.out_pk = _ptr(out_pk, torch.float64, realizations * nbins, "out_pk")
    r.out_counts = _ptr(out_counts, torch.int32, realizations * cells, "out_counts")
    r.out_ntot = _ptr(out_ntot, torch.int64, realizations, "out_ntot")
    r.out_cov = _ptr(out_cov, torch.float64, nbins * nbins, "out_cov")
    fdt = torch.float64 if int(precision) == F64 else torch.float32
    r.out_fields = _ptr(out_fields, fdt, realizations * cells, "out_fields")
    r.out_delta = _ptr(out_delta, fdt, realizations * cells, "out_delta")
    if edges is not None:
        import numpy as np
        e = np.ascontiguousarray(edges, dtype=np.float64)
        if e.size != nbins + 1:
            raise ValueError("edges must hold nbins + 1 values")
        r.kedges = e.ctypes.data
        keep = (keep, e)
    return keep


def server_submit(server, n, h, xi, precision, seed, request_id, realizations, nbar, nbins, out_pk,
                  out_counts=None, out_ntot=None, out_cov=None, edges=None, out_fields=None, out_delta=None):
    """Queue one request; returns its ticket.  Output tensors must outlive the request; edges
    (nbins + 1 shell edges in |k|, host) are copied."""
    r = Request()
    keep = _fill_request(r, n, h, xi, precision, seed, request_id, realizations, nbar, nbins, out_pk,
                         out_counts, out_ntot, out_cov, edges, out_fields, out_delta)
    t = c_u64()
    _check(_server_submit(server, ctypes.byref(r), ctypes.byref(t)), "ce_server_submit")
    del keep
    return t.value


def server_submit_many(server, requests):
    """Queue several requests at once (dicts with the arguments of server_submit after
    `server`); returns their tickets."""
    arr = (Request * len(requests))()
    keep = [_fill_request(arr[k], **q) for k, q in enumerate(requests)]
    t = (c_u64 * len(requests))()
    _check(_server_submit_many(server, arr, len(requests), t), "ce_server_submit_many")
    del keep
    return list(t)


def server_poll(server, ticket):
    """(state, status, latency_ms); state 0 queued, 1 running, 2 done, 3 failed, 4 cancelled."""
    st, status, lat = c_i32(), c_i32(), c_f64()
    _check(_server_poll(server, int(ticket), ctypes.byref(st), ctypes.byref(status), ctypes.byref(lat)),
           "ce_server_poll")
    return st.value, status.value, lat.value


def server_drain(server, max_n=4096):
    """Finished requests in completion order: list of (ticket, state, status, latency_ms)."""
    t = (c_u64 * max_n)()
    st = (c_i32 * max_n)()
    status = (c_i32 * max_n)()
    lat = (c_f64 * max_n)()
    n = c_i32()
    _check(_server_drain(server, max_n, t, st, status, lat, ctypes.byref(n)), "ce_server_drain")
    return [(t[i], st[i], status[i], lat[i]) for i in range(n.value)]


def server_cancel(server, ticket):
    return _server_cancel(server, int(ticket))


def server_stats(server):
    st = ServerStats()
    _check(_server_stats(server, ctypes.byref(st)), "ce_server_stats_read")
    return {k: getattr(st, k) for k, _ in ServerStats._fields_}


def server_destroy(server):
    _server_destroy(server)


def _sched_dict(s):
    return {k: getattr(s, k) for k, _ in Schedule._fields_}


def autotune(ctx, plan, count, nbar, nbins, reps=3):
    """Tune the launch schedule of plan's shape (installed in ctx); returns it with the timings."""
    s = Schedule()
    _check(_autotune(ctx, plan.handle, int(count), float(nbar), int(nbins), int(reps), ctypes.byref(s)),
           "ce_autotune")
    return _sched_dict(s)


def schedule_set(ctx, n, h, precision, schedule):
    """Install a schedule (dict with the Schedule fields; None removes it) for a shape."""
    g = geometry(n, h)
    if schedule is None:
        _check(_schedule_set(ctx, ctypes.byref(g), int(precision), None), "ce_schedule_set")
        return
    s = Schedule()
    s.noise_block, s.noise_pairs, s.bin_lds = 1, 0, 81920
    for k, v in schedule.items():
        if k in ("ms", "default_ms"):
            continue
        setattr(s, k, int(v))
    _check(_schedule_set(ctx, ctypes.byref(g), int(precision), ctypes.byref(s)), "ce_schedule_set")


def schedule_get(ctx, n, h, precision):
    g = geometry(n, h)
    s = Schedule()
    st = _schedule_get(ctx, ctypes.byref(g), int(precision), ctypes.byref(s))
    if st == E_INVALID:
        return None
    _check(st, "ce_schedule_get")
    return _sched_dict(s)


# launch schedules tuned on gfx950 for the shapes of the package's benchmark workloads
DEFAULT_SCHEDULES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedules_gfx950.json")


def schedule_save(ctx, path):
    _check(_schedule_save(ctx, str(path).encode()), "ce_schedule_save")


def schedule_load(ctx, path):
    _check(_schedule_load(ctx, str(path).encode()), "ce_schedule_load")


def shell_table(n, h, nbins):
    import numpy as np
    g = geometry(n, h)
    nm = np.zeros(nbins, dtype=np.int64)
    km = np.zeros(nbins, dtype=np.float64)
    _check(_shell_table(ctypes.byref(g), int(nbins), nm.ctypes.data_as(c_void_p), km.ctypes.data_as(c_void_p)),
           "ce_shell_table")
    return nm, km


def fft_factors(length):
    import numpy as np
    r = np.zeros(16, dtype=np.int32)
    ns = c_i32()
    _check(_fft_factors(int(length), r.ctypes.data_as(c_void_p), ctypes.byref(ns)), "ce_fft_factors")
    return [int(x) for x in r[:ns.value]]


def debug_philox(seed, ctr, n_calls, out_words, stream=None):
    import numpy as np
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    _check(_debug_philox(int(seed), c.ctypes.data_as(c_void_p), int(n_calls),
                         _ptr(out_words, torch.int32, 4 * n_calls, "out_words"), _stream(stream)),
           "ce_debug_philox")


def debug_noise(plan, seed, request_id, pair, out, stream=None):
    _check(_debug_noise(plan.handle, int(seed), int(request_id), int(pair),
                        _ptr(out, plan.dtype, 2 * plan.embedding_cells, "out"), _stream(stream)),
           "ce_debug_noise")
