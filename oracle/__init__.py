"""ctypes binding of the plain-C FP64 oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product package never imports
it, and it imports nothing from the product package.

Every function takes numpy arrays (int32 CSR indices, float64 values) and
returns numpy arrays; see ``oracle.c`` for the definitions and the passages
of the paper each one follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")   # the same source built with OpenMP

OK, INVALID, NOT_CONVERGED, BREAKDOWN, UNSUPPORTED = 0, -1, -4, -5, -6

GCC_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]


def _build_one(out, extra, force):
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *GCC_FLAGS, *extra, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (single-threaded)
    and ``liboracle_omp.so`` (OpenMP over the rows of the SpMV)."""
    _build_one(_LIB_OMP, ["-fopenmp"], force)
    return _build_one(_LIB, [], force)


_lib = None
_lib_omp = None


def lib(parallel: bool = False):
    """The single-threaded oracle, or with parallel=True its OpenMP build
    (same bits; SpMV rows on all threads)."""
    global _lib, _lib_omp
    if parallel:
        if _lib_omp is None:
            _build_one(_LIB_OMP, ["-fopenmp"], False)
            _lib_omp = C.CDLL(_LIB_OMP)
            _declare(_lib_omp)
        return _lib_omp
    if _lib is None:
        alt = os.environ.get("ORACLE_LIB")   # a separately built variant (mutation tests)
        if alt:
            _lib = C.CDLL(alt)
        else:
            build(force=False)
            _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


def threads(parallel: bool = True) -> int:
    """Threads the oracle's SpMV uses in that build."""
    return int(lib(parallel).orc_threads())


_i64 = C.c_int64
_pd = C.POINTER(C.c_double)
_pi32 = C.POINTER(C.c_int32)
_pi64 = C.POINTER(C.c_int64)


def _declare(L):
    L.orc_threads.argtypes = []
    L.orc_threads.restype = C.c_int
    L.orc_spmv.argtypes = [_i64, _pi32, _pi32, _pd, C.c_double, _pd, C.c_double, _pd]
    L.orc_spmv.restype = None
    L.orc_relres.argtypes = [_i64, _pi32, _pi32, _pd, _pd, _pd]
    L.orc_relres.restype = C.c_double
    L.orc_csr_validate.argtypes = [_i64, _i64, _i64, _pi32, _pi32]
    L.orc_csr_validate.restype = C.c_int
    L.orc_features_int.argtypes = [_i64, _i64, _pi32, _pi32, _pd, _pi64]
    L.orc_features_int.restype = C.c_int
    L.orc_features_derive.argtypes = [_pi64, _pd]
    L.orc_features_derive.restype = None
    L.orc_feature_vector.argtypes = [_pi64, _pd, _pd]
    L.orc_feature_vector.restype = None
    L.orc_ell_shape.argtypes = [_i64, _pi32, _pi64, _pi64]
    L.orc_ell_shape.restype = C.c_int
    L.orc_csr_to_ell.argtypes = [_i64, _pi32, _pi32, _pd, _i64, _i64, _pi32, _pd]
    L.orc_csr_to_ell.restype = C.c_int
    L.orc_csr_to_coo_rows.argtypes = [_i64, _pi32, _pi32]
    L.orc_csr_to_coo_rows.restype = None
    L.orc_dia_shape.argtypes = [_i64, _i64, _pi32, _pi32, _pi64, _pi64, _pi32]
    L.orc_dia_shape.restype = C.c_int
    L.orc_csr_to_dia.argtypes = [_i64, _pi32, _pi32, _pd, _i64, _i64, _pi32, _pd]
    L.orc_csr_to_dia.restype = C.c_int
    L.orc_hyb_width.argtypes = [_i64, _pi32]
    L.orc_hyb_width.restype = C.c_int64
    L.orc_hyb_tail_rows.argtypes = [_i64, _pi32, _i64, _pi32]
    L.orc_hyb_tail_rows.restype = C.c_int64
    L.orc_tree_eval.argtypes = [_pi32, _pd, _pi32, _pi32, _pi32, _pd]
    L.orc_tree_eval.restype = C.c_int32
    L.orc_cascade.argtypes = ([_pi32, _pd, _pi32, _pi32, _pi32] * 3) + [_pd, _pi32]
    L.orc_cascade.restype = None
    L.orc_cg.argtypes = [_i64, _pi32, _pi32, _pd, _pd, _pd, C.c_double, _i64, _pi64, _pd,
                         _pd, _pd, _pd, _i64, _pd, _pd, _i64]
    L.orc_cg.restype = C.c_int
    L.orc_arnoldi.argtypes = [_i64, _pi32, _pi32, _pd, _pd, _i64, _pd, _pd, _pi64]
    L.orc_arnoldi.restype = C.c_int
    L.orc_gmres.argtypes = [_i64, _pi32, _pi32, _pd, _pd, _pd, _i64, C.c_double, _i64,
                            _pi64, _pd, _pd, _i64]
    L.orc_gmres.restype = C.c_int


def _p(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ct))


def _csr(A):
    rp = np.ascontiguousarray(A.rp, dtype=np.int32)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, col, val


def spmv(A, x, alpha=1.0, beta=0.0, y=None, parallel=False):
    rp, col, val = _csr(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(A.n) if y is None else np.array(y, dtype=np.float64, copy=True)
    lib(parallel).orc_spmv(A.n, _p(rp, C.c_int32), _p(col, C.c_int32), _p(val, C.c_double),
                   float(alpha), _p(x, C.c_double), float(beta), _p(out, C.c_double))
    return out


def relres(A, b, x, parallel=False):
    rp, col, val = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib(parallel).orc_relres(A.n, _p(rp, C.c_int32), _p(col, C.c_int32), _p(val, C.c_double),
                            _p(b, C.c_double), _p(x, C.c_double))


def validate(A) -> int:
    rp, col, _ = _csr(A)
    return lib().orc_csr_validate(A.n, A.ncols, int(rp[-1]), _p(rp, C.c_int32),
                                  _p(col, C.c_int32))


INT_FIELDS = ["nrows", "ncols", "nnz", "sum_r", "sum_r2", "max_r", "min_r", "span_sum",
              "cluster_sum", "ndiag", "diag_nnz"] + [f"hist{b}" for b in range(16)] + \
             ["is_symmetric"]
DERIVED_FIELDS = ["density", "mean", "sd", "cov", "maxavg", "distavg", "clusteravg",
                  "fill", "diagfill"]
MODEL_FEATURES = ["nrows", "ncols", "nnz", "density", "mean", "sd", "cov", "max", "min",
                  "maxavg", "distavg", "clusteravg", "fill", "ndiag", "diagfill"]


def features(A):
    """Returns (int64[28] accumulators, float64[9] derived, float64[15] model vector)."""
    rp, col, val = _csr(A)
    ints = np.zeros(28, dtype=np.int64)
    st = lib().orc_features_int(A.n, A.ncols, _p(rp, C.c_int32), _p(col, C.c_int32),
                                _p(val, C.c_double), _p(ints, C.c_int64))
    if st != OK:
        raise ValueError("invalid CSR")
    der = np.zeros(9)
    lib().orc_features_derive(_p(ints, C.c_int64), _p(der, C.c_double))
    f15 = np.zeros(15)
    lib().orc_feature_vector(_p(ints, C.c_int64), _p(der, C.c_double), _p(f15, C.c_double))
    return ints, der, f15


def derive(ints):
    ints = np.ascontiguousarray(ints, dtype=np.int64)
    der = np.zeros(9)
    lib().orc_features_derive(_p(ints, C.c_int64), _p(der, C.c_double))
    return der


def ell_shape(A):
    rp = np.ascontiguousarray(A.rp, dtype=np.int32)
    K = C.c_int64()
    pitch = C.c_int64()
    st = lib().orc_ell_shape(A.n, _p(rp, C.c_int32), C.byref(K), C.byref(pitch))
    return st, K.value, pitch.value


def to_ell(A):
    """Returns (status, K, pitch, ell_col int32[K*pitch], ell_val float64[K*pitch])."""
    st, K, pitch = ell_shape(A)
    if st != OK:
        return st, K, pitch, None, None
    rp, col, val = _csr(A)
    ec = np.empty(K * pitch, dtype=np.int32)
    ev = np.empty(K * pitch, dtype=np.float64)
    lib().orc_csr_to_ell(A.n, _p(rp, C.c_int32), _p(col, C.c_int32), _p(val, C.c_double),
                         K, pitch, _p(ec, C.c_int32), _p(ev, C.c_double))
    return st, K, pitch, ec, ev


def to_coo_rows(A):
    rp = np.ascontiguousarray(A.rp, dtype=np.int32)
    row = np.empty(int(rp[-1]), dtype=np.int32)
    lib().orc_csr_to_coo_rows(A.n, _p(rp, C.c_int32), _p(row, C.c_int32))
    return row


def dia_shape(A):
    """Returns (status, ndiag, pitch, offsets int32[ndiag])."""
    rp, col, _ = _csr(A)
    nd = C.c_int64()
    pitch = C.c_int64()
    lib().orc_dia_shape(A.n, A.ncols, _p(rp, C.c_int32), _p(col, C.c_int32), C.byref(nd),
                        C.byref(pitch), None)
    off = np.empty(max(nd.value, 1), dtype=np.int32)
    st = lib().orc_dia_shape(A.n, A.ncols, _p(rp, C.c_int32), _p(col, C.c_int32), C.byref(nd),
                             C.byref(pitch), _p(off, C.c_int32))
    return st, nd.value, pitch.value, off[:nd.value]


def to_dia(A):
    """Returns (status, ndiag, pitch, offsets int32[ndiag], values float64[ndiag*pitch])."""
    st, nd, pitch, off = dia_shape(A)
    if st != OK:
        return st, nd, pitch, off, None
    rp, col, val = _csr(A)
    dv = np.empty(nd * pitch, dtype=np.float64)
    off = np.ascontiguousarray(off, dtype=np.int32)
    lib().orc_csr_to_dia(A.n, _p(rp, C.c_int32), _p(col, C.c_int32), _p(val, C.c_double), nd,
                         pitch, _p(off, C.c_int32), _p(dv, C.c_double))
    return st, nd, pitch, off, dv


def hyb_width(A):
    rp = np.ascontiguousarray(A.rp, dtype=np.int32)
    return int(lib().orc_hyb_width(A.n, _p(rp, C.c_int32)))


def to_hyb(A):
    """Returns (K, pitch, ell_col int32[K*pitch], ell_val float64[K*pitch],
    tail_rows int32[nt]): the ELL part of width K and the rows longer than K."""
    rp, col, val = _csr(A)
    K = hyb_width(A)
    pitch = (A.n + 63) // 64 * 64
    ec = np.empty(K * pitch, dtype=np.int32)
    ev = np.empty(K * pitch, dtype=np.float64)
    lib().orc_csr_to_ell(A.n, _p(rp, C.c_int32), _p(col, C.c_int32), _p(val, C.c_double),
                         K, pitch, _p(ec, C.c_int32), _p(ev, C.c_double))
    nt = int(lib().orc_hyb_tail_rows(A.n, _p(rp, C.c_int32), K, None))
    tr = np.empty(max(nt, 1), dtype=np.int32)
    lib().orc_hyb_tail_rows(A.n, _p(rp, C.c_int32), K, _p(tr, C.c_int32))
    return K, pitch, ec, ev, tr[:nt]


def _tree_arrays(tree):
    return (np.ascontiguousarray(tree["feature"], dtype=np.int32),
            np.ascontiguousarray(tree["threshold"], dtype=np.float64),
            np.ascontiguousarray(tree["left"], dtype=np.int32),
            np.ascontiguousarray(tree["right"], dtype=np.int32),
            np.ascontiguousarray(tree["cls"], dtype=np.int32))


def tree_eval(tree, f15):
    fe, th, le, ri, cl = _tree_arrays(tree)
    f = np.ascontiguousarray(f15, dtype=np.float64)
    return int(lib().orc_tree_eval(_p(fe, C.c_int32), _p(th, C.c_double), _p(le, C.c_int32),
                                   _p(ri, C.c_int32), _p(cl, C.c_int32), _p(f, C.c_double)))


def cascade(trees, f15):
    """trees: three dicts with feature/threshold/left/right/cls arrays."""
    args = []
    keep = []
    for t in trees:
        arrs = _tree_arrays(t)
        keep.append(arrs)
        fe, th, le, ri, cl = arrs
        args += [_p(fe, C.c_int32), _p(th, C.c_double), _p(le, C.c_int32),
                 _p(ri, C.c_int32), _p(cl, C.c_int32)]
    f = np.ascontiguousarray(f15, dtype=np.float64)
    out = np.zeros(3, dtype=np.int32)
    lib().orc_cascade(*args, _p(f, C.c_double), _p(out, C.c_int32))
    return [int(v) for v in out]


def cg(A, b, x0=None, tol=1e-10, maxit=100000, hist=0, nrec=0, parallel=False):
    rp, col, val = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    it = C.c_int64()
    rr = C.c_double()
    ah = np.zeros(hist) if hist else None
    bh = np.zeros(hist) if hist else None
    rh = np.full(hist, np.nan) if hist else None
    R = np.zeros((nrec, A.n)) if nrec else None
    P = np.zeros((nrec, A.n)) if nrec else None
    st = lib(parallel).orc_cg(A.n, _p(rp, C.c_int32), _p(col, C.c_int32), _p(val, C.c_double),
                      _p(b, C.c_double), _p(x, C.c_double), float(tol), int(maxit),
                      C.byref(it), C.byref(rr), _p(ah, C.c_double), _p(bh, C.c_double),
                      _p(rh, C.c_double), int(hist), _p(R, C.c_double), _p(P, C.c_double),
                      int(nrec))
    return dict(status=st, x=x, iters=it.value, relres=rr.value, alpha=ah, beta=bh,
                res=rh, R=R, P=P)


def arnoldi(A, v0, m):
    rp, col, val = _csr(A)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    V = np.zeros((m + 1, A.n))       # row t = basis vector t (column-major n x (m+1))
    H = np.zeros((m, m + 1))         # row j = column j of H
    steps = C.c_int64()
    st = lib().orc_arnoldi(A.n, _p(rp, C.c_int32), _p(col, C.c_int32), _p(val, C.c_double),
                           _p(v0, C.c_double), int(m), _p(V, C.c_double), _p(H, C.c_double),
                           C.byref(steps))
    return st, V.T.copy(), H.T.copy(), steps.value


def gmres(A, b, x0=None, m=30, tol=1e-10, maxit=100000, hist=0, parallel=False):
    rp, col, val = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    it = C.c_int64()
    rr = C.c_double()
    rh = np.full(hist, np.nan) if hist else None
    st = lib(parallel).orc_gmres(A.n, _p(rp, C.c_int32), _p(col, C.c_int32), _p(val, C.c_double),
                         _p(b, C.c_double), _p(x, C.c_double), int(m), float(tol), int(maxit),
                         C.byref(it), C.byref(rr), _p(rh, C.c_double), int(hist))
    return dict(status=st, x=x, iters=it.value, relres=rr.value, res=rh)
