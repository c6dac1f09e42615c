"""Seeded generators for sparse tensors shaped like the paper's workloads.

Section 5.1 evaluates on rating tensors (users x items x time; values 1..5)
and on synthetic tensors of order 3..10. Neither data set ships here; these
generators stand in for them with the shapes, value ranges and skewed
(Zipf) index distributions of such data.

Every function takes an explicit seed or numpy Generator, so both the oracle
and the GPU library receive identical inputs.
"""
import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "_synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force=False):
    """Compile the generators' multi-threaded kernels (_synth.c) with gcc."""
    if force or not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-fopenmp", "-ffp-contract=off", _SRC, "-o",
                               tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        vp = C.c_void_p
        lib.syn_zipf_lookup.argtypes = [vp, C.c_int64, vp, vp, C.c_int64, vp]
        lib.syn_first_distinct.argtypes = [C.c_int, vp, C.c_int64, vp]
        lib.syn_planted.argtypes = [C.c_int, C.c_int, vp, vp, C.c_int64,
                                    C.c_double, vp]
        lib.syn_planted.restype = None
        _lib = lib
    return _lib


def _p(a):
    return C.c_void_p(a.ctypes.data)


def _rng(seed):
    return seed if isinstance(seed, np.random.Generator) else \
        np.random.Generator(np.random.PCG64(seed))


def _first_distinct(idx, dims):
    """Indices of the first occurrence of every distinct tuple, in draw
    order (exact: hash buckets, full-tuple comparison)."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    n = idx.shape[1]
    keep = np.empty(n, dtype=np.uint8)
    if n and _load().syn_first_distinct(idx.shape[0], _p(idx), n,
                                        _p(keep)) != 0:
        raise MemoryError("duplicate removal ran out of memory")
    return np.flatnonzero(keep)


def uniform_distinct(seed, dims, count):
    """count distinct coordinates drawn uniformly, kept in first-drawn order."""
    rng = _rng(seed)
    dims = [int(d) for d in dims]
    space = int(np.prod(np.array(dims, dtype=object)))
    if count > space:
        raise ValueError("more nonzeros than cells")
    idx = np.zeros((len(dims), 0), dtype=np.int32)
    while idx.shape[1] < count:
        need = count - idx.shape[1]
        draw = np.stack([rng.integers(0, d, size=int(need * 1.2) + 16,
                                      dtype=np.int32) for d in dims])
        idx = np.concatenate([idx, draw], axis=1)
        idx = idx[:, _first_distinct(idx, dims)]
    return np.ascontiguousarray(idx[:, :count])


class _Zipf:
    """Inverse-CDF sampler of P(k) ~ k^-s over k = 1..I, mapped to row ids by a
    seeded random relabelling so that hot rows are not adjacent."""

    def __init__(self, rng, I, s):
        w = np.arange(1, I + 1, dtype=np.float64) ** (-float(s))
        self.cdf = np.cumsum(w)
        self.cdf /= self.cdf[-1]
        self.label = rng.permutation(I).astype(np.int32)

    def draw(self, rng, size):
        u = rng.random(size)
        out = np.empty(size, dtype=np.int32)
        if _load().syn_zipf_lookup(_p(self.cdf), len(self.cdf),
                                   _p(self.label), _p(u), size,
                                   _p(out)) != 0:
            raise MemoryError("zipf lookup table")
        return out


def zipf_distinct(seed, dims, s, count, progress=None):
    """count distinct coordinates with every mode's index drawn Zipf(s); the
    tuples are deduplicated and redrawn until enough are distinct, kept in
    first-drawn order. progress(msg), if given, hears about every round."""
    rng = _rng(seed)
    dims = [int(d) for d in dims]
    samplers = [_Zipf(rng, d, s) for d in dims]
    idx = np.zeros((len(dims), 0), dtype=np.int32)
    rounds = 0
    ratio = 2.0
    while idx.shape[1] < count:
        have = idx.shape[1]
        need = count - have
        m = int(need * ratio) + 64
        draw = np.stack([z.draw(rng, m) for z in samplers])
        idx = np.concatenate([idx, draw], axis=1)
        idx = idx[:, _first_distinct(idx, dims)]
        gained = max(idx.shape[1] - have, 1)
        ratio = min(64.0, 1.1 * m / gained)
        rounds += 1
        if progress:
            progress(f"zipf round {rounds}: {min(idx.shape[1], count)} of "
                     f"{count} distinct")
        if rounds > 200:
            raise RuntimeError("cannot draw enough distinct coordinates")
    return np.ascontiguousarray(idx[:, :count])


def planted_values(seed, dims, idx, J, R, a_std, b_std, scale=1.0,
                   progress=None):
    """Values of a planted low-rank tensor at the coordinates idx.

    Data synthesis only: draws planted matrices P^(n) (I_n x J) and
    Q^(n) (J x R) with normal entries of the given standard deviations and
    returns scale * sum_r prod_n (P^(n) Q^(n))[i_n, r] as float64. The values
    are an input to both sides of every comparison; whether the structure is
    truly low-rank is pinned by the planted-recovery test, not assumed.
    """
    rng = _rng(seed)
    U = []
    for d in dims:
        P = rng.normal(0.0, a_std, size=(int(d), J))
        Q = rng.normal(0.0, b_std, size=(J, R))
        U.append(np.ascontiguousarray(P @ Q, dtype=np.float64))
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    nnz = idx.shape[1]
    out = np.empty(nnz, dtype=np.float64)
    up = (C.c_void_p * len(U))(*[u.ctypes.data for u in U])
    _load().syn_planted(len(U), R, up, _p(idx), nnz, float(scale), _p(out))
    if progress:
        progress(f"planted values for {nnz} nonzeros")
    return out


@dataclass
class Tensor:
    dims: list
    train_idx: np.ndarray          # int32 (N, nnz_train)
    train_val: np.ndarray          # float32 (nnz_train,)
    test_idx: np.ndarray           # int32 (N, nnz_test)
    test_val: np.ndarray           # float32 (nnz_test,)
    meta: dict = field(default_factory=dict)

    @property
    def order(self):
        return len(self.dims)


def make_tensor(w, seed=None, cache_dir=None, progress=None):
    """Build the synthetic tensor of a Workload (see configs.py). With
    cache_dir, a tensor generated before for the same workload and seed is
    loaded from there (a plain .npz, no pickles) instead. progress(msg), if
    given, hears about the generation steps."""
    seed = w.data_seed if seed is None else seed
    if cache_dir:
        import hashlib
        import os
        key = hashlib.sha256(repr((w, seed)).encode()).hexdigest()[:16]
        path = os.path.join(cache_dir, f"tensor_{key}.npz")
        if os.path.exists(path):
            z = np.load(path, allow_pickle=False)
            return Tensor(dims=list(w.dims), train_idx=z["train_idx"],
                          train_val=z["train_val"], test_idx=z["test_idx"],
                          test_val=z["test_val"],
                          meta={"workload": w.name, "seed": seed})
        T = make_tensor(w, seed, progress=progress)
        os.makedirs(cache_dir, exist_ok=True)
        tmp = path + ".tmp.npz"
        np.savez(tmp, train_idx=T.train_idx, train_val=T.train_val,
                 test_idx=T.test_idx, test_val=T.test_val)
        os.replace(tmp, path)
        return T
    rng = _rng(seed)
    if w.index_dist == "uniform":
        idx = uniform_distinct(rng, w.dims, w.nnz)
    else:
        idx = zipf_distinct(rng, w.dims, w.zipf_s, w.nnz, progress=progress)
    x = planted_values(rng, w.dims, idx, w.planted_rank, w.planted_rank,
                       w.planted_a_std, w.planted_b_std, w.planted_scale,
                       progress=progress)
    x = x + rng.normal(0.0, w.noise_std, size=x.shape)
    if w.values == "rating":
        x = np.clip(np.rint(w.rating_offset + x), 1.0, 5.0)
    order = rng.permutation(w.nnz)
    n_test = int(round(w.nnz * w.test_frac))
    # the test set is order[:n_test]; both sets keep first-drawn order
    in_test = np.zeros(w.nnz, dtype=bool)
    in_test[order[:n_test]] = True
    del order
    te, tr = np.flatnonzero(in_test), np.flatnonzero(~in_test)
    return Tensor(dims=list(w.dims),
                  train_idx=np.ascontiguousarray(idx[:, tr]),
                  train_val=x[tr].astype(np.float32),
                  test_idx=np.ascontiguousarray(idx[:, te]),
                  test_val=x[te].astype(np.float32),
                  meta={"workload": w.name, "seed": seed})


def init_params(seed, dims, J, R, a_std, b_std=None, dist="normal"):
    """Initial factor and core matrices as float32 (the starting point of
    Algorithm 3). dist 'normal': N(0, std^2) entries; 'uniform': U(0, std)."""
    rng = _rng(seed)
    b_std = a_std if b_std is None else b_std
    Js = [J] * len(dims) if np.isscalar(J) else list(J)
    A, B = [], []
    for d, j in zip(dims, Js):
        if dist == "normal":
            A.append(rng.normal(0.0, a_std, size=(int(d), j)).astype(np.float32))
        else:
            A.append(rng.uniform(0.0, a_std, size=(int(d), j)).astype(np.float32))
    for j in Js:
        if dist == "normal":
            B.append(rng.normal(0.0, b_std, size=(j, R)).astype(np.float32))
        else:
            B.append(rng.uniform(0.0, b_std, size=(j, R)).astype(np.float32))
    return A, B


def epoch_perm(seed, epoch, nnz):
    """Visiting order of the training set for one epoch (a permutation)."""
    rng = _rng(np.random.SeedSequence([int(seed), int(epoch)]))
    return rng.permutation(nnz).astype(np.int64)
