"""MI355X sparse FastTucker SGD (FastTuckerPlus hot path) -- Python binding.

A thin ctypes layer over libft.so (include/ft.h): it converts numpy arrays
to pointers and status codes to exceptions. Every step of the SGD sweep runs
in the library's HIP kernels.
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import (FT_TRAIN, FT_TEST, FT_FP32, FT_BF16, FT_FP8_E4M3,  # noqa
                   FT_ROW_SUM, FT_ROW_MEAN, FT_CORE_PER_EPOCH,
                   FT_CORE_PER_MINIBATCH, KERNELS, Options)

__all__ = ["FastTucker", "FtError", "default_options", "FT_TRAIN", "FT_TEST",
           "FT_ROW_SUM", "FT_ROW_MEAN", "FT_CORE_PER_EPOCH",
           "FT_CORE_PER_MINIBATCH", "KERNELS"]


class FtError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def default_options():
    o = Options()
    _check(_lib.load().ft_default_options(C.byref(o)), None)
    return o


def _check(status, handle):
    if status != 0:
        msg = _lib.load().ft_last_error(handle)
        raise FtError(status, msg.decode() if msg else "")


class FastTucker:
    """One sparse FastTucker problem on the current HIP device."""

    def __init__(self, dims, J, R, seed=0):
        lib = _lib.load()
        self.dims = [int(d) for d in dims]
        self.N = len(self.dims)
        self.J = [int(J)] * self.N if np.isscalar(J) else [int(j) for j in J]
        self.R = int(R)
        d = np.array(self.dims, dtype=np.int64)
        j = np.array(self.J, dtype=np.int32)
        h = C.c_void_p()
        _check(lib.ft_create(self.N, _ptr(d, C.c_int64), _ptr(j, C.c_int32),
                             self.R, C.c_uint64(seed), C.byref(h)), None)
        self._h = h
        self._lib = lib
        self.nnz = {FT_TRAIN: 0, FT_TEST: 0}

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.ft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _c(self, status):
        _check(status, self._h)

    # -- configuration ----------------------------------------------------
    @property
    def options(self):
        o = Options()
        self._c(self._lib.ft_get_options(self._h, C.byref(o)))
        return o

    def set_options(self, **kw):
        o = self.options
        for k, v in kw.items():
            if not hasattr(o, k):
                raise AttributeError(k)
            setattr(o, k, v)
        self._c(self._lib.ft_set_options(self._h, C.byref(o)))
        return o

    def set_stream(self, stream_handle):
        self._c(self._lib.ft_set_stream(self._h, C.c_void_p(stream_handle)))

    # -- data -------------------------------------------------------------
    def set_nonzeros(self, which, idx, vals):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.float32)
        if idx.ndim != 2 or idx.shape[0] != self.N or \
                vals.shape != (idx.shape[1],):
            raise ValueError("idx must be (order, nnz) and vals (nnz,)")
        nnz = idx.shape[1]
        self._c(self._lib.ft_set_nonzeros(self._h, which, nnz,
                                          _ptr(idx, C.c_int32),
                                          _ptr(vals, C.c_float)))
        self.nnz[which] = nnz

    def set_epoch_order(self, perm):
        if perm is None:
            self._c(self._lib.ft_set_epoch_order(self._h, None))
            return
        perm = np.ascontiguousarray(perm, dtype=np.int64)
        if perm.shape != (self.nnz[FT_TRAIN],):
            raise ValueError("perm must have one entry per training nonzero")
        self._c(self._lib.ft_set_epoch_order(self._h, _ptr(perm, C.c_int64)))

    def num_minibatches(self):
        v = C.c_int64()
        self._c(self._lib.ft_num_minibatches(self._h, C.byref(v)))
        return v.value

    # -- parameters -------------------------------------------------------
    def get_params(self):
        A, B = [], []
        for n in range(self.N):
            a = np.empty((self.dims[n], self.J[n]), dtype=np.float32)
            self._c(self._lib.ft_get_params(self._h, n, 0, _ptr(a, C.c_float)))
            b = np.empty((self.J[n], self.R), dtype=np.float32)
            self._c(self._lib.ft_get_params(self._h, n, 1, _ptr(b, C.c_float)))
            A.append(a)
            B.append(b)
        return A, B

    def set_params(self, A=None, B=None):
        for n in range(self.N):
            if A is not None:
                a = np.ascontiguousarray(A[n], dtype=np.float32)
                if a.shape != (self.dims[n], self.J[n]):
                    raise ValueError(f"A[{n}] must be {(self.dims[n], self.J[n])}")
                self._c(self._lib.ft_set_params(self._h, n, 0,
                                                _ptr(a, C.c_float)))
            if B is not None:
                b = np.ascontiguousarray(B[n], dtype=np.float32)
                if b.shape != (self.J[n], self.R):
                    raise ValueError(f"B[{n}] must be {(self.J[n], self.R)}")
                self._c(self._lib.ft_set_params(self._h, n, 1,
                                                _ptr(b, C.c_float)))

    # -- SGD epochs -------------------------------------------------------
    def epoch_factors(self):
        out = np.zeros(self.num_minibatches(), dtype=np.float64)
        self._c(self._lib.ft_epoch_factors(self._h, _ptr(out, C.c_double)))
        return out

    def prepare_epoch(self):
        self._c(self._lib.ft_prepare_epoch(self._h))

    def factor_minibatch(self, b, apply=True):
        loss = C.c_double()
        if apply:
            self._c(self._lib.ft_factor_minibatch(self._h, b, 1,
                                                  C.byref(loss), None, None))
            return loss.value
        G = [np.zeros((self.dims[n], self.J[n]), dtype=np.float32)
             for n in range(self.N)]
        K = [np.zeros(self.dims[n], dtype=np.int32) for n in range(self.N)]
        gp = (C.POINTER(C.c_float) * self.N)(*[_ptr(g, C.c_float) for g in G])
        kp = (C.POINTER(C.c_int32) * self.N)(*[_ptr(k, C.c_int32) for k in K])
        self._c(self._lib.ft_factor_minibatch(self._h, b, 0, C.byref(loss),
                                              gp, kp))
        return loss.value, G, K

    def epoch_core(self):
        loss = C.c_double()
        self._c(self._lib.ft_epoch_core(self._h, C.byref(loss)))
        return loss.value

    def core_grad(self):
        G = [np.zeros((self.J[n], self.R), dtype=np.float32)
             for n in range(self.N)]
        gp = (C.POINTER(C.c_float) * self.N)(*[_ptr(g, C.c_float) for g in G])
        loss = C.c_double()
        self._c(self._lib.ft_core_grad(self._h, gp, C.byref(loss)))
        return loss.value, G

    # -- evaluation -------------------------------------------------------
    def eval(self, which=FT_TEST):
        sse, sae = C.c_double(), C.c_double()
        self._c(self._lib.ft_eval(self._h, which, C.byref(sse), C.byref(sae)))
        return sse.value, sae.value

    def rmse(self, which=FT_TEST):
        v = C.c_double()
        self._c(self._lib.ft_rmse(self._h, which, C.byref(v)))
        return v.value

    def loss(self, which=FT_TRAIN):
        v = C.c_double()
        self._c(self._lib.ft_loss(self._h, which, C.byref(v)))
        return v.value

    # -- builder output ---------------------------------------------------
    def epoch_order(self):
        out = np.empty(self.nnz[FT_TRAIN], dtype=np.int64)
        self._c(self._lib.ft_get_epoch_order(self._h, _ptr(out, C.c_int64)))
        return out

    def minibatch_sort(self, b, mode):
        M = self.options.minibatch
        m = min(M, self.nnz[FT_TRAIN] - b * M)
        pos = np.empty(max(m, 0), dtype=np.int32)
        rows = np.empty(max(m, 0), dtype=np.int32)
        self._c(self._lib.ft_get_minibatch_sort(self._h, b, mode,
                                                _ptr(pos, C.c_int32),
                                                _ptr(rows, C.c_int32)))
        return pos, rows

    # -- profiling --------------------------------------------------------
    def profile(self, on=True):
        self._c(self._lib.ft_profile_enable(self._h, 1 if on else 0))

    def profile_reset(self):
        self._c(self._lib.ft_profile_reset(self._h))

    def profile_get(self, kernel):
        k = KERNELS.index(kernel) if isinstance(kernel, str) else int(kernel)
        n, ms = C.c_int64(), C.c_double()
        self._c(self._lib.ft_profile_get(self._h, k, C.byref(n), C.byref(ms)))
        return n.value, ms.value
