"""ctypes binding of libcaskrylov.so (see include/caskrylov.h).

Argument marshalling only: torch tensors become device pointers, torch
streams become hipStream_t, ctypes structs mirror the C structs.  Every
computation happens in the HIP library; if it is missing, loading fails.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcaskrylov.so")
DEFAULT_MODEL = os.path.join(_HERE, "cascade_model.txt")

CK_OK, CK_E_INVALID, CK_E_NOMEM, CK_E_HIP = 0, -1, -2, -3
CK_E_NOT_CONVERGED, CK_E_BREAKDOWN, CK_E_UNSUPPORTED, CK_E_CANCELLED = -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "HIP", -4: "NOT_CONVERGED",
                -5: "BREAKDOWN", -6: "UNSUPPORTED", -7: "CANCELLED"}
CK_FMT_CSR, CK_FMT_ELL, CK_FMT_COO, CK_FMT_DIA, CK_FMT_HYB = 0, 1, 2, 3, 4
CK_ALG_SCALAR, CK_ALG_VECTOR, CK_ALG_MERGE, CK_ALG_PANEL = 0, 1, 2, 3
CK_PREC_FP64, CK_PREC_MIXED = 0, 1
CK_EXEC_DEFAULT, CK_EXEC_ASYNC, CK_EXEC_SEQUENTIAL = 0, 1, 2
CK_KEEP_FP32 = 1
CK_FEAT_NO_SYMMETRY = 1
NUM_CONFIGS = 14
CONFIG_NAMES = ["csr-vector-1", "csr-vector-2", "csr-vector-4", "csr-vector-8",
                "csr-vector-16", "csr-vector-32", "csr-vector-64", "csr-scalar", "csr-merge",
                "ell", "coo", "csr-panel", "dia", "hyb"]
ID_ELL, ID_DIA = 9, 12       # the configurations whose conversion can be refused for fill


class CkError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("format", C.c_int32), ("algorithm", C.c_int32), ("lanes", C.c_int32),
                ("stages_done", C.c_int32)]

    def __repr__(self):
        return (f"Config(format={self.format}, algorithm={self.algorithm}, "
                f"lanes={self.lanes}, stages_done={self.stages_done})")


class Features(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("nrows", "ncols", "nnz", "sum_r", "sum_r2", "max_r",
                                         "min_r", "span_sum", "cluster_sum", "ndiag", "diag_nnz")] + \
               [("hist", C.c_int64 * 16), ("is_symmetric", C.c_int64)] + \
               [(n, C.c_double) for n in ("density", "mean", "sd", "cov", "maxavg", "distavg",
                                          "clusteravg", "fill", "diagfill")]

    def ints(self):
        """The 28 integer accumulators in the C layout order."""
        return [self.nrows, self.ncols, self.nnz, self.sum_r, self.sum_r2, self.max_r,
                self.min_r, self.span_sum, self.cluster_sum, self.ndiag, self.diag_nnz] + \
               list(self.hist) + [self.is_symmetric]

    def derived(self):
        return [self.density, self.mean, self.sd, self.cov, self.maxavg, self.distavg,
                self.clusteravg, self.fill, self.diagfill]

    @classmethod
    def from_model_inputs(cls, f15):
        """A record whose 15 model inputs are f15 (feature-table order); the
        other accumulators stay 0.  For host-only use of the cascade."""
        F = cls()
        ints = {0: "nrows", 1: "ncols", 2: "nnz", 7: "max_r", 8: "min_r", 13: "ndiag"}
        dbls = {3: "density", 4: "mean", 5: "sd", 6: "cov", 9: "maxavg", 10: "distavg",
                11: "clusteravg", 12: "fill", 14: "diagfill"}
        for i, v in enumerate(f15):
            if i in ints:
                assert float(v) == int(v), "integer feature expected"
                setattr(F, ints[i], int(v))
            else:
                setattr(F, dbls[i], float(v))
        return F

    def model_inputs(self):
        return [float(self.nrows), float(self.ncols), float(self.nnz), self.density, self.mean,
                self.sd, self.cov, float(self.max_r), float(self.min_r), self.maxavg,
                self.distavg, self.clusteravg, self.fill, float(self.ndiag), self.diagfill]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("restart", C.c_int32),
                ("precision", C.c_int32), ("async_", C.c_int32), ("check_every", C.c_int32),
                ("use_config", C.c_int32), ("config", Config), ("overhead_aware", C.c_int32),
                ("known_start", C.c_int32)]


class SolveResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32),
                ("switch_iter", C.c_int32 * 3), ("outer_steps", C.c_int32),
                ("true_relres", C.c_double), ("t_features_us", C.c_double),
                ("t_infer_us", C.c_double), ("t_convert_us", C.c_double),
                ("t_total_us", C.c_double), ("final_config", Config),
                ("conversion_gated", C.c_int32), ("est_remaining_iters", C.c_int32)]

    def as_dict(self):
        return dict(status=self.status, iterations=self.iterations,
                    switch_iter=list(self.switch_iter), outer_steps=self.outer_steps,
                    true_relres=self.true_relres, t_features_us=self.t_features_us,
                    t_infer_us=self.t_infer_us, t_convert_us=self.t_convert_us,
                    t_total_us=self.t_total_us, final_config=config_id(self.final_config),
                    conversion_gated=self.conversion_gated,
                    est_remaining_iters=self.est_remaining_iters)


class ServerOpts(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("max_slots", C.c_int32),
                ("chunk_iters", C.c_int32), ("small_n", C.c_int32),
                ("large_workers", C.c_int32), ("precision", C.c_int32),
                ("restart", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double)]


class Completion(C.Structure):
    _fields_ = [("tag", C.c_int64), ("matrix_id", C.c_int32), ("status", C.c_int32),
                ("iterations", C.c_int32), ("path", C.c_int32), ("config_id", C.c_int32),
                ("pad", C.c_int32), ("true_relres", C.c_double), ("t_submit_us", C.c_double),
                ("t_admit_us", C.c_double), ("t_done_us", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "completed", "queued", "in_flight",
                                         "resident_matrices", "evictions", "bytes_in_use",
                                         "batched_launches", "prediction_cache_hits",
                                         "prediction_cache_misses", "window_completed")] + \
               [(n, C.c_double) for n in ("p50_latency_us", "p99_latency_us", "solves_per_s")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class AllocatorStruct(C.Structure):
    """ck_allocator: alloc(bytes, stream, ctx) -> device pointer, free(ptr, stream, ctx)."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class CallbackAllocator:
    """A ck_allocator whose functions are Python callables:
    alloc(nbytes, stream) -> int device pointer (0 on failure) and
    free(ptr, stream).  Keep the object alive while handles use it."""

    def __init__(self, alloc, free):
        def _alloc(nbytes, stream, _ctx):
            try:
                return int(alloc(int(nbytes), int(stream or 0))) or None
            except Exception:          # NULL: the library reports CK_E_NOMEM
                return None

        def _free(ptr, stream, _ctx):
            try:
                free(int(ptr), int(stream or 0))
            except Exception:
                pass

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.struct = AllocatorStruct(self._alloc, self._free, None)


_TORCH_ALLOCATORS = {}


def torch_allocator(device=None):
    """The ck_allocator backed by torch's caching allocator on `device`
    (default: the current device); one per device, kept for the process."""
    import torch
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    if dev is None:
        dev = torch.cuda.current_device()
    if dev not in _TORCH_ALLOCATORS:
        _TORCH_ALLOCATORS[dev] = CallbackAllocator(
            lambda nbytes, stream: torch.cuda.caching_allocator_alloc(nbytes, dev, stream),
            lambda ptr, stream: torch.cuda.caching_allocator_delete(ptr))
    return _TORCH_ALLOCATORS[dev]


_lib = None
_vp = C.c_void_p
_i32, _i64, _u32, _dbl, _flt = C.c_int32, C.c_int64, C.c_uint32, C.c_double, C.c_float

# name -> (restype, argtypes); the C-ABI surface of include/caskrylov.h
SIGNATURES = {
    "spmv_create": (_i32, [C.POINTER(_vp), _i64, _i64, _i64, _vp, _vp, _vp, _u32,
                           C.POINTER(AllocatorStruct), _vp]),
    "spmv_destroy": (None, [_vp]),
    "spmv_features": (_i32, [_vp, C.POINTER(Features), _vp]),
    "spmv_select": (_i32, [C.POINTER(Features), C.c_char_p, C.POINTER(Config)]),
    "ck_select_stages": (_i32, [C.POINTER(Features), C.c_char_p, C.POINTER(_i32)]),
    "ck_default_config": (_i32, [_vp, C.POINTER(Config)]),
    "ck_features_ex": (_i32, [_vp, C.POINTER(Features), C.c_uint32, _vp]),
    "ck_start_config": (_i32, [C.c_int64, C.c_int64, C.c_int64, C.c_char_p, C.POINTER(Config),
                               C.POINTER(_i32)]),
    "spmv_convert": (_i32, [_vp, C.POINTER(Config), _vp]),
    "ck_set_active": (_i32, [_vp, C.POINTER(Config)]),
    "ck_get_active": (_i32, [_vp, C.POINTER(Config)]),
    "spmv_apply": (_i32, [_vp, C.POINTER(Config), _dbl, _vp, _dbl, _vp, _vp]),
    "spmv_apply_f32": (_i32, [_vp, C.POINTER(Config), _flt, _vp, _flt, _vp, _vp]),
    "spmv_apply_noalloc": (_i32, [_vp, C.POINTER(Config), _dbl, _vp, _dbl, _vp, _vp]),
    "ck_select_device": (_i32, [_vp, _vp, _vp]),
    "ck_cascade_eval_device": (_i32, [_vp, _i64, _vp, _vp]),
    "cg_solve": (_i32, [_vp, _vp, _vp, C.POINTER(SolveOpts), C.POINTER(SolveResult), _vp]),
    "gmres_solve": (_i32, [_vp, _vp, _vp, C.POINTER(SolveOpts), C.POINTER(SolveResult), _vp]),
    "ck_export_ell": (_i32, [_vp, _vp, _vp, C.POINTER(_i64), C.POINTER(_i64), _vp]),
    "ck_export_coo_rows": (_i32, [_vp, _vp, _vp]),
    "ck_panel_layout": (_i32, [_vp, C.POINTER(_i32), C.POINTER(_i64), C.POINTER(_i64)]),
    "ck_eval_stage": (_i32, [C.POINTER(Features), C.c_char_p, _i32, C.POINTER(_i32)]),
    "ck_overhead_gate": (_i32, [C.POINTER(Features), C.POINTER(Config), _i32, _dbl, _i32, _dbl,
                                _dbl, C.POINTER(_dbl), C.POINTER(_dbl), C.POINTER(_i32)]),
    "ck_export_dia": (_i32, [_vp, _vp, _vp, C.POINTER(_i64), C.POINTER(_i64), _vp]),
    "ck_export_hyb": (_i32, [_vp, _vp, _vp, _vp, C.POINTER(_i64), C.POINTER(_i64),
                             C.POINTER(_i64), C.POINTER(_i32), _vp]),
    "ck_dot": (_i32, [_i64, _vp, _vp, _vp, _vp]),
    "ck_config_id": (_i32, [C.POINTER(Config)]),
    "ck_config_from_id": (_i32, [_i32, C.POINTER(Config)]),
    "ck_kernel_name": (_i32, [C.POINTER(Config), _i32, C.c_char_p, C.c_size_t]),
    "ck_spmv_bytes": (_i64, [_vp, _i32, _i32]),
    "ck_time_spmv": (_i32, [_vp, C.POINTER(Config), _i32, _vp, _vp, _i32, _i32, _vp,
                            C.POINTER(_dbl)]),
    "ck_server_create": (_i32, [C.POINTER(ServerOpts), C.POINTER(_vp)]),
    "ck_server_add_matrix": (_i32, [_vp, _i32, _i64, _i64, _vp, _vp, _vp]),
    "ck_server_submit": (_i32, [_vp, _i32, _vp, _vp, _i64]),
    "ck_server_poll": (_i32, [_vp, C.POINTER(Completion), _i32]),
    "ck_server_drain": (_i32, [_vp, _dbl]),
    "ck_server_get_stats": (_i32, [_vp, C.POINTER(ServerStats)]),
    "ck_server_reset_stats": (_i32, [_vp]),
    "ck_server_clock_us": (_dbl, [_vp]),
    "ck_server_destroy": (None, [_vp]),
    "ck_last_error": (C.c_char_p, []),
}


def lib():
    """Load libcaskrylov.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2411_10143_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != CK_OK:
        raise CkError(st, lib().ck_last_error().decode())
    return st


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t, dtype=None):
    if t is None:
        return None
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_cuda or not t.is_contiguous():
        raise TypeError("expected a contiguous device tensor")
    return t.data_ptr()


def config(format=CK_FMT_CSR, algorithm=CK_ALG_VECTOR, lanes=4):
    return Config(format, algorithm, lanes, 0)


def config_from_id(i):
    c = Config()
    _check(lib().ck_config_from_id(i, C.byref(c)))
    return c


def config_id(c):
    return int(lib().ck_config_id(C.byref(c)))


def kernel_name(c, fp32=False):
    buf = C.create_string_buffer(128)
    _check(lib().ck_kernel_name(C.byref(c), int(fp32), buf, 128))
    return buf.value.decode()


def _allocator(allocator, device):
    if allocator is None:
        return None
    if allocator == "torch":
        return torch_allocator(device)
    if isinstance(allocator, CallbackAllocator):
        return allocator
    raise TypeError("allocator must be 'torch', None or a CallbackAllocator")


def spmv_create(rp, col, val, ncols=None, keep_fp32=False, stream=None, allocator="torch"):
    """Copy a device CSR (int32 rowptr/col, float64 val) into a new handle.
    allocator: "torch" (torch's caching allocator supplies every device
    block of the handle), None (the library's own cache) or a
    CallbackAllocator; it must outlive the handle."""
    import torch
    n = rp.numel() - 1
    h = _vp()
    a = _allocator(allocator, rp.device)
    _check(lib().spmv_create(C.byref(h), n, n if ncols is None else ncols, col.numel(),
                             _ptr(rp, torch.int32), _ptr(col, torch.int32),
                             _ptr(val, torch.float64), CK_KEEP_FP32 if keep_fp32 else 0,
                             C.byref(a.struct) if a is not None else None, _stream(stream)))
    return h.value


def spmv_destroy(h):
    lib().spmv_destroy(h)


def spmv_features(h, stream=None, symmetry=True):
    """The feature record; symmetry=False skips the symmetry test
    (is_symmetric = -1), which the cascade does not use."""
    f = Features()
    if symmetry:
        _check(lib().spmv_features(h, C.byref(f), _stream(stream)))
    else:
        _check(lib().ck_features_ex(h, C.byref(f), CK_FEAT_NO_SYMMETRY, _stream(stream)))
    return f


def select_device(h, out, stream=None):
    """Device-resident cascade into `out` (int32 device tensor of 8): format,
    algorithm, lanes, stages, the three stage classes, configuration id."""
    import torch
    if out.numel() < 8:
        raise ValueError("out needs 8 int32 entries")
    _check(lib().ck_select_device(h, _ptr(out, torch.int32), _stream(stream)))


def cascade_eval_device(f15, ids, stream=None):
    """Configuration ids for rows of 15 model inputs (float64 device tensor
    of shape (count, 15)) into ids (int32 device tensor of count)."""
    import torch
    if f15.dim() != 2 or f15.shape[1] != 15 or ids.numel() < f15.shape[0]:
        raise ValueError("f15 must be (count, 15) and ids hold count entries")
    _check(lib().ck_cascade_eval_device(_ptr(f15, torch.float64), f15.shape[0],
                                        _ptr(ids, torch.int32), _stream(stream)))


def spmv_select(features, model_path=None):
    c = Config()
    mp = model_path.encode() if model_path else None
    _check(lib().spmv_select(C.byref(features), mp, C.byref(c)))
    return c


def select_stages(features, model_path=None):
    st = (_i32 * 3)()
    mp = model_path.encode() if model_path else None
    _check(lib().ck_select_stages(C.byref(features), mp, st))
    return list(st)


def eval_stage(features, stage, model_path=None):
    """Class of one stage's tree alone (no cascade gating)."""
    cls = _i32()
    mp = model_path.encode() if model_path else None
    _check(lib().ck_eval_stage(C.byref(features), mp, int(stage), C.byref(cls)))
    return cls.value


def overhead_gate(features, target, t0, r0, t1, r1, tol):
    """(remaining iterations, conversion cost in products, convert?) of the
    overhead-aware conversion rule."""
    rem, cost, go = _dbl(), _dbl(), _i32()
    _check(lib().ck_overhead_gate(C.byref(features), C.byref(target), int(t0), float(r0),
                                  int(t1), float(r1), float(tol), C.byref(rem), C.byref(cost),
                                  C.byref(go)))
    return rem.value, cost.value, bool(go.value)


def start_config(nrows, ncols, nnz, model_path=None):
    """(configuration, from_tree) a solve with known_start begins on: the
    model's start tree over the inputs known without a pass over the entries."""
    c, ft = Config(), _i32()
    mp = model_path.encode() if model_path else None
    _check(lib().ck_start_config(int(nrows), int(ncols), int(nnz), mp, C.byref(c), C.byref(ft)))
    return c, bool(ft.value)


def default_config(h):
    c = Config()
    _check(lib().ck_default_config(h, C.byref(c)))
    return c


def spmv_convert(h, cfg, stream=None):
    _check(lib().spmv_convert(h, C.byref(cfg), _stream(stream)))


def set_active(h, cfg):
    _check(lib().ck_set_active(h, C.byref(cfg)))


def get_active(h):
    c = Config()
    _check(lib().ck_get_active(h, C.byref(c)))
    return c


def spmv_apply(h, x, y, alpha=1.0, beta=0.0, cfg=None, stream=None):
    import torch
    _check(lib().spmv_apply(h, C.byref(cfg) if cfg is not None else None, float(alpha),
                            _ptr(x, torch.float64), float(beta), _ptr(y, torch.float64),
                            _stream(stream)))


def spmv_apply_noalloc(h, x, y, alpha=1.0, beta=0.0, cfg=None, stream=None):
    """spmv_apply whose workspace is the library's fixed device array."""
    import torch
    _check(lib().spmv_apply_noalloc(h, C.byref(cfg) if cfg is not None else None, float(alpha),
                                    _ptr(x, torch.float64), float(beta), _ptr(y, torch.float64),
                                    _stream(stream)))


def spmv_apply_f32(h, x, y, alpha=1.0, beta=0.0, cfg=None, stream=None):
    import torch
    _check(lib().spmv_apply_f32(h, C.byref(cfg) if cfg is not None else None, float(alpha),
                                _ptr(x, torch.float32), float(beta), _ptr(y, torch.float32),
                                _stream(stream)))


def _opts(tol, max_iter, restart, precision, async_, check_every, cfg, overhead_aware=False,
          known_start=False):
    o = SolveOpts()
    o.overhead_aware = int(overhead_aware)
    o.known_start = int(known_start)
    o.tol = tol
    o.max_iter = max_iter
    o.restart = restart
    o.precision = precision
    o.async_ = int(async_)
    o.check_every = check_every
    if cfg is not None:
        o.use_config = 1
        o.config = cfg
    return o


def _solve(fn, h, b, x, tol, max_iter, restart, precision, async_, check_every, cfg, stream,
           raise_on_error, overhead_aware=False, known_start=False):
    import torch
    o = _opts(tol, max_iter, restart, precision, async_, check_every, cfg, overhead_aware,
              known_start)
    r = SolveResult()
    st = fn(h, _ptr(b, torch.float64), _ptr(x, torch.float64), C.byref(o), C.byref(r),
            _stream(stream))
    if st not in (CK_OK, CK_E_NOT_CONVERGED, CK_E_BREAKDOWN) or (raise_on_error and st != CK_OK):
        _check(st)
    return r.as_dict()


def cg_solve(h, b, x, tol=1e-10, max_iter=100000, precision=CK_PREC_FP64, async_=False,
             check_every=8, config=None, stream=None, raise_on_error=False,
             overhead_aware=False, known_start=False):
    """x holds x0 on entry and the solution on return; returns the result record.
    async_: CK_EXEC_DEFAULT/False, CK_EXEC_ASYNC/True or CK_EXEC_SEQUENTIAL."""
    return _solve(lib().cg_solve, h, b, x, tol, max_iter, 0, precision, async_, check_every,
                  config, stream, raise_on_error, overhead_aware, known_start)


def gmres_solve(h, b, x, tol=1e-10, max_iter=100000, restart=30, precision=CK_PREC_FP64,
                async_=False, check_every=8, config=None, stream=None, raise_on_error=False,
                overhead_aware=False, known_start=False):
    return _solve(lib().gmres_solve, h, b, x, tol, max_iter, restart, precision, async_,
                  check_every, config, stream, raise_on_error, overhead_aware, known_start)


def export_ell(h, stream=None):
    import torch
    K, pitch = _i64(), _i64()
    _check(lib().ck_export_ell(h, None, None, C.byref(K), C.byref(pitch), _stream(stream)))
    ec = torch.empty(K.value * pitch.value, dtype=torch.int32, device="cuda")
    ev = torch.empty(K.value * pitch.value, dtype=torch.float64, device="cuda")
    _check(lib().ck_export_ell(h, _ptr(ec), _ptr(ev), C.byref(K), C.byref(pitch),
                               _stream(stream)))
    return K.value, pitch.value, ec, ev


def export_dia(h, stream=None):
    """(ndiag, pitch, offsets int32[ndiag], values float64[ndiag*pitch]) on the device."""
    import torch
    nd, pitch = _i64(), _i64()
    _check(lib().ck_export_dia(h, None, None, C.byref(nd), C.byref(pitch), _stream(stream)))
    off = torch.empty(nd.value, dtype=torch.int32, device="cuda")
    dv = torch.empty(nd.value * pitch.value, dtype=torch.float64, device="cuda")
    _check(lib().ck_export_dia(h, _ptr(off) if nd.value else None,
                               _ptr(dv) if nd.value else None, C.byref(nd), C.byref(pitch),
                               _stream(stream)))
    return nd.value, pitch.value, off, dv


def export_hyb(h, stream=None):
    """(K, pitch, lanes, ell_col int32[K*pitch], ell_val float64[K*pitch],
    long rows int32[ntail]) on the device."""
    import torch
    K, pitch, nt, L = _i64(), _i64(), _i64(), _i32()
    _check(lib().ck_export_hyb(h, None, None, None, C.byref(K), C.byref(pitch), C.byref(nt),
                               C.byref(L), _stream(stream)))
    cnt = K.value * pitch.value
    ec = torch.empty(cnt, dtype=torch.int32, device="cuda")
    ev = torch.empty(cnt, dtype=torch.float64, device="cuda")
    rows = torch.empty(nt.value, dtype=torch.int32, device="cuda")
    _check(lib().ck_export_hyb(h, _ptr(ec) if cnt else None, _ptr(ev) if cnt else None,
                               _ptr(rows) if nt.value else None, C.byref(K), C.byref(pitch),
                               C.byref(nt), C.byref(L), _stream(stream)))
    return K.value, pitch.value, L.value, ec, ev, rows


def export_coo_rows(h, nnz, stream=None):
    import torch
    row = torch.empty(nnz, dtype=torch.int32, device="cuda")
    _check(lib().ck_export_coo_rows(h, _ptr(row) if nnz else None, _stream(stream)))
    return row


def panel_layout(h):
    """(panels, columns per panel, stored panel rows) of the CSR-panel copy."""
    P, W, R = _i32(), _i64(), _i64()
    _check(lib().ck_panel_layout(h, C.byref(P), C.byref(W), C.byref(R)))
    return P.value, W.value, R.value


def dot(x, y, out, stream=None):
    import torch
    _check(lib().ck_dot(x.numel(), _ptr(x, torch.float64), _ptr(y, torch.float64),
                        _ptr(out, torch.float64), _stream(stream)))


def time_spmv(h, cfg, x, y, warmup=10, reps=200, fp32=False, stream=None):
    """Mean microseconds per product over `reps` back-to-back launches (HIP
    events on the launch stream)."""
    us = _dbl()
    _check(lib().ck_time_spmv(h, C.byref(cfg), int(fp32), _ptr(x), _ptr(y), int(warmup),
                              int(reps), _stream(stream), C.byref(us)))
    return us.value


def spmv_bytes(h, fp32=False, beta_nonzero=False):
    return int(lib().ck_spmv_bytes(h, int(fp32), int(beta_nonzero)))


def server_create(budget_bytes=64 << 30, max_slots=256, chunk_iters=8, small_n=8192,
                  large_workers=8, precision=CK_PREC_MIXED, restart=30, max_iter=100000,
                  tol=1e-8):
    o = ServerOpts(int(budget_bytes), max_slots, chunk_iters, small_n, large_workers,
                   precision, restart, max_iter, float(tol))
    h = _vp()
    _check(lib().ck_server_create(C.byref(o), C.byref(h)))
    return h.value


def server_add_matrix(srv, mid, rp, col, val):
    import torch
    _check(lib().ck_server_add_matrix(srv, int(mid), rp.numel() - 1, col.numel(),
                                      _ptr(rp, torch.int32), _ptr(col, torch.int32),
                                      _ptr(val, torch.float64)))


def server_submit(srv, mid, b, x, tag):
    import torch
    _check(lib().ck_server_submit(srv, int(mid), _ptr(b, torch.float64), _ptr(x, torch.float64),
                                  int(tag)))


def server_poll(srv, cap=1024):
    buf = (Completion * cap)()
    k = lib().ck_server_poll(srv, buf, cap)
    return [buf[i].as_dict() for i in range(k)]


def server_drain(srv, timeout_s=600.0):
    _check(lib().ck_server_drain(srv, float(timeout_s)))


def server_stats(srv):
    s = ServerStats()
    _check(lib().ck_server_get_stats(srv, C.byref(s)))
    return s.as_dict()


def server_reset_stats(srv):
    _check(lib().ck_server_reset_stats(srv))


def server_clock_us(srv):
    return float(lib().ck_server_clock_us(srv))


def server_destroy(srv):
    lib().ck_server_destroy(srv)


class Matrix:
    """Owns a handle; a convenience wrapper over the C calls."""

    def __init__(self, rp, col, val, ncols=None, keep_fp32=False, stream=None,
                 allocator="torch"):
        self.n = rp.numel() - 1
        self.ncols = self.n if ncols is None else ncols
        self.nnz = col.numel()
        self.allocator = _allocator(allocator, rp.device)   # outlives the handle
        self.handle = spmv_create(rp, col, val, ncols, keep_fp32, stream,
                                  self.allocator if self.allocator is not None else None)

    @classmethod
    def from_csr(cls, A, keep_fp32=False, device="cuda", stream=None, allocator="torch"):
        import torch
        rp = torch.from_numpy(A.rp).to(device)
        col = torch.from_numpy(A.col).to(device)
        val = torch.from_numpy(A.val).to(device)
        return cls(rp, col, val, A.ncols, keep_fp32, stream, allocator)

    def close(self):
        if getattr(self, "handle", None):
            spmv_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
