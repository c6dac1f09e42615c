"""ctypes front end of the FP64 C oracle (ft_oracle.c).

Test infrastructure only (see the package docstring). Arrays:
  A[n]  float64 (I_n, J_n) C-contiguous, updated in place by the epoch calls
  B[n]  float64 (J_n, R)   C-contiguous, updated in place by core_epoch
  idx   int32   (N, nnz)   coordinates, row n holds i_n (0-based)
  vals  float64 (nnz,)
  perm  int64   (nnz,)     visiting order of the training set
Each wrapper cites the passage of the paper its C function follows.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ft_oracle.c")
_SRC_PAR = os.path.join(_HERE, "ft_oracle_par.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)


def lib_path():
    return _LIB


def build(force=False):
    """Compile ft_oracle.c with gcc (strict IEEE: no fast-math; OpenMP only
    spreads the *_par functions' independent samples over threads)."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                         os.path.getmtime(_SRC_PAR))):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-fopenmp", "-ffp-contract=off", _SRC_PAR,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def use_library(path=None):
    """Load the oracle from another build of ft_oracle.c (None: the default
    one). Only the test suite's planted-mistake check uses this."""
    global _lib, _override
    _override = path
    _lib = None


_override = None


def _load():
    global _lib
    if _lib is None:
        if _override is None:
            build()
        lib = C.CDLL(_override or _LIB)
        pp = C.POINTER(_dp)
        lib.orc_predict.argtypes = [C.c_int, _i32p, C.c_int32, pp, pp,
                                    C.c_int64, _i32p, _dp]
        lib.orc_residual_stats.argtypes = [C.c_int, _i32p, C.c_int32, pp, pp,
                                           C.c_int64, _i32p, _dp, _dp, _dp]
        lib.orc_loss.argtypes = [C.c_int, _i64p, _i32p, C.c_int32, pp, pp,
                                 C.c_int64, _i32p, _dp, C.c_double,
                                 C.c_double]
        lib.orc_loss.restype = C.c_double
        lib.orc_factor_minibatch.argtypes = [
            C.c_int, _i64p, _i32p, C.c_int32, pp, pp, C.c_int64, _i32p, _dp,
            C.c_double, C.c_double, C.c_int, C.c_int, pp,
            C.POINTER(_i64p)]
        lib.orc_factor_minibatch.restype = C.c_double
        lib.orc_factor_epoch.argtypes = [
            C.c_int, _i64p, _i32p, C.c_int32, pp, pp, C.c_int64, _i32p, _dp,
            _i64p, C.c_int64, C.c_double, C.c_double, C.c_int, _dp]
        lib.orc_core_grad.argtypes = [C.c_int, _i32p, C.c_int32, pp, pp,
                                      C.c_int64, _i32p, _dp, pp]
        lib.orc_core_grad.restype = C.c_double
        lib.orc_core_epoch.argtypes = [
            C.c_int, _i64p, _i32p, C.c_int32, pp, pp, C.c_int64, _i32p, _dp,
            _i64p, C.c_int64, C.c_double, C.c_double, C.c_int]
        lib.orc_core_epoch.restype = C.c_double
        if not hasattr(lib, "orc_factor_minibatch_par"):
            _lib = lib       # a build of ft_oracle.c alone (mutant checks)
            return _lib
        lib.orc_factor_minibatch_par.argtypes = \
            lib.orc_factor_minibatch.argtypes
        lib.orc_factor_minibatch_par.restype = C.c_double
        lib.orc_factor_epoch_par.argtypes = lib.orc_factor_epoch.argtypes
        lib.orc_core_grad_par.argtypes = lib.orc_core_grad.argtypes
        lib.orc_core_grad_par.restype = C.c_double
        lib.orc_core_epoch_par.argtypes = [
            C.c_int, _i32p, C.c_int32, pp, pp, C.c_int64, _i32p, _dp,
            C.c_double, C.c_double]
        lib.orc_core_epoch_par.restype = C.c_double
        lib.orc_residual_stats_par.argtypes = lib.orc_residual_stats.argtypes
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_set_threads.restype = C.c_int
        _lib = lib
    return _lib


def _f64(a, name):
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64
            and a.flags.c_contiguous):
        raise TypeError(f"{name} must be a C-contiguous float64 ndarray")
    return a


def _ptrs(mats, name):
    arr = (_dp * len(mats))()
    for n, m in enumerate(mats):
        arr[n] = _f64(m, f"{name}[{n}]").ctypes.data_as(_dp)
    return arr


def _shape(A, B):
    N = len(A)
    if N < 1 or N > 10 or len(B) != N:
        raise ValueError("need 1..10 modes and one B per A")
    R = B[0].shape[1]
    J = np.array([a.shape[1] for a in A], dtype=np.int32)
    dims = np.array([a.shape[0] for a in A], dtype=np.int64)
    for n in range(N):
        if B[n].shape != (J[n], R):
            raise ValueError(f"B[{n}] must be ({J[n]}, {R})")
    return N, dims, J, R


def _coords(idx, N, dims):
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    if idx.ndim != 2 or idx.shape[0] != N:
        raise ValueError("idx must be (N, nnz)")
    if idx.shape[1] and (idx.min() < 0 or np.any(idx.max(axis=1) >= dims)):
        raise ValueError("index out of range")
    return idx


def _vals(v, nnz):
    v = np.ascontiguousarray(v, dtype=np.float64)
    if v.shape != (nnz,):
        raise ValueError("vals must be (nnz,)")
    return v


def predict(A, B, idx):
    """Eq. (3): xhat for every nonzero."""
    lib = _load()
    N, dims, J, R = _shape(A, B)
    idx = _coords(idx, N, dims)
    out = np.empty(idx.shape[1], dtype=np.float64)
    lib.orc_predict(N, J.ctypes.data_as(_i32p), R, _ptrs(A, "A"),
                    _ptrs(B, "B"), idx.shape[1], idx.ctypes.data_as(_i32p),
                    out.ctypes.data_as(_dp))
    return out


def set_threads(n=0):
    """Host threads of the parallel forms (n < 1: every core); returns the
    count in force."""
    return _load().orc_set_threads(int(n))


def residual_stats(A, B, idx, vals, parallel=False):
    """(sum (x - xhat)^2, sum |x - xhat|) over a set (Section 5.2 RMSE/MAE).
    parallel: chunk sums over threads, added in chunk order."""
    lib = _load()
    N, dims, J, R = _shape(A, B)
    idx = _coords(idx, N, dims)
    vals = _vals(vals, idx.shape[1])
    sse, sae = C.c_double(), C.c_double()
    fn = lib.orc_residual_stats_par if parallel else lib.orc_residual_stats
    fn(N, J.ctypes.data_as(_i32p), R, _ptrs(A, "A"),
                           _ptrs(B, "B"), idx.shape[1],
                           idx.ctypes.data_as(_i32p), vals.ctypes.data_as(_dp),
                           C.byref(sse), C.byref(sae))
    return sse.value, sae.value


def loss(A, B, idx, vals, lamA, lamB):
    """Objective of Eq. (4), regularisers summed over the modes."""
    lib = _load()
    N, dims, J, R = _shape(A, B)
    idx = _coords(idx, N, dims)
    vals = _vals(vals, idx.shape[1])
    return lib.orc_loss(N, dims.ctypes.data_as(_i64p),
                        J.ctypes.data_as(_i32p), R, _ptrs(A, "A"),
                        _ptrs(B, "B"), idx.shape[1], idx.ctypes.data_as(_i32p),
                        vals.ctypes.data_as(_dp), lamA, lamB)


def factor_minibatch(A, B, idx, vals, lrA, lamA, row_mean, apply=True,
                     want_grad=False, parallel=False):
    """One minibatch of Algorithm 3's factor loop, rule Eq. (12), Jacobi in
    the minibatch. Returns loss (sum r^2/2), and with want_grad the dense row
    gradients G[n] (I_n, J_n) (lamA * a included once per occurrence) and the
    occurrence counts k[n] (I_n,). parallel: per-sample work over threads,
    bitwise the same results."""
    lib = _load()
    N, dims, J, R = _shape(A, B)
    idx = _coords(idx, N, dims)
    vals = _vals(vals, idx.shape[1])
    G = cnt = None
    gp = cp = None
    if want_grad:
        G = [np.zeros((dims[n], J[n])) for n in range(N)]
        cnt = [np.zeros(dims[n], dtype=np.int64) for n in range(N)]
        gp = _ptrs(G, "G")
        cp = (_i64p * N)(*[c.ctypes.data_as(_i64p) for c in cnt])
    fn = lib.orc_factor_minibatch_par if parallel else \
        lib.orc_factor_minibatch
    l = fn(
        N, dims.ctypes.data_as(_i64p), J.ctypes.data_as(_i32p), R,
        _ptrs(A, "A"), _ptrs(B, "B"), idx.shape[1], idx.ctypes.data_as(_i32p),
        vals.ctypes.data_as(_dp), lrA, lamA, int(row_mean), int(apply), gp, cp)
    if want_grad:
        return l, G, cnt
    return l


def factor_epoch(A, B, idx, vals, perm, M, lrA, lamA, row_mean,
                 parallel=False):
    """Factor loop of Algorithm 3 over one permutation pass; returns the
    per-minibatch losses (sum r^2/2). parallel: bitwise the same results."""
    lib = _load()
    N, dims, J, R = _shape(A, B)
    idx = _coords(idx, N, dims)
    nnz = idx.shape[1]
    vals = _vals(vals, nnz)
    perm = np.ascontiguousarray(perm, dtype=np.int64)
    if perm.shape != (nnz,):
        raise ValueError("perm must be (nnz,)")
    nmb = (nnz + M - 1) // M
    out = np.zeros(nmb)
    fn = lib.orc_factor_epoch_par if parallel else lib.orc_factor_epoch
    fn(N, dims.ctypes.data_as(_i64p),
                         J.ctypes.data_as(_i32p), R, _ptrs(A, "A"),
                         _ptrs(B, "B"), nnz, idx.ctypes.data_as(_i32p),
                         vals.ctypes.data_as(_dp), perm.ctypes.data_as(_i64p),
                         M, lrA, lamA, int(row_mean), out.ctypes.data_as(_dp))
    return out


def core_grad(A, B, idx, vals, parallel=False):
    """Grad^(n) = sum r a^T d over a set (Algorithm 5 accumulation).
    parallel: chunk sums over threads, added in chunk order."""
    lib = _load()
    N, dims, J, R = _shape(A, B)
    idx = _coords(idx, N, dims)
    vals = _vals(vals, idx.shape[1])
    Grad = [np.zeros((J[n], R)) for n in range(N)]
    fn = lib.orc_core_grad_par if parallel else lib.orc_core_grad
    l = fn(N, J.ctypes.data_as(_i32p), R, _ptrs(A, "A"),
                          _ptrs(B, "B"), idx.shape[1],
                          idx.ctypes.data_as(_i32p), vals.ctypes.data_as(_dp),
                          _ptrs(Grad, "Grad"))
    return l, Grad


def core_epoch(A, B, idx, vals, lrB, lamB, perm=None, M=0,
               per_minibatch=False, parallel=False):
    """Algorithm 5 (one update per epoch) or, with per_minibatch, one update
    per minibatch of the order perm. Returns sum r^2/2. parallel (Algorithm 5
    only): the gradient's chunk sums over threads, added in chunk order."""
    lib = _load()
    N, dims, J, R = _shape(A, B)
    idx = _coords(idx, N, dims)
    nnz = idx.shape[1]
    vals = _vals(vals, nnz)
    if parallel and not per_minibatch:
        return lib.orc_core_epoch_par(
            N, J.ctypes.data_as(_i32p), R, _ptrs(A, "A"), _ptrs(B, "B"), nnz,
            idx.ctypes.data_as(_i32p), vals.ctypes.data_as(_dp), lrB, lamB)
    pp = None
    if per_minibatch:
        perm = np.ascontiguousarray(perm, dtype=np.int64)
        if perm.shape != (nnz,) or M < 1:
            raise ValueError("per-minibatch core step needs perm and M")
        pp = perm.ctypes.data_as(_i64p)
    return lib.orc_core_epoch(N, dims.ctypes.data_as(_i64p),
                              J.ctypes.data_as(_i32p), R, _ptrs(A, "A"),
                              _ptrs(B, "B"), nnz, idx.ctypes.data_as(_i32p),
                              vals.ctypes.data_as(_dp), pp, int(M), lrB, lamB,
                              int(per_minibatch))
