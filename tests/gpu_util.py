"""Helpers shared by the GPU parity tests: build a problem from a workload on
both sides with identical seeded inputs."""
import numpy as np

import synth
from paper_2404_10087_amd import FT_TEST, FT_TRAIN, FastTucker

EPS32 = np.finfo(np.float32).eps


def f64(mats):
    return [np.array(m, dtype=np.float64) for m in mats]


def setup(w, with_test=True, tensor=None):
    T = synth.make_tensor(w) if tensor is None else tensor
    ft = FastTucker(w.dims, w.J, w.R, seed=1)
    ft.set_options(minibatch=w.M, lr_A=w.lr_A, lr_B=w.lr_B,
                   lambda_A=w.lam_A, lambda_B=w.lam_B,
                   row_scale=int(w.row_mean))
    ft.set_nonzeros(FT_TRAIN, T.train_idx, T.train_val)
    if with_test and T.test_idx.shape[1]:
        ft.set_nonzeros(FT_TEST, T.test_idx, T.test_val)
    A0, B0 = synth.init_params(w.init_seed, w.dims, w.J, w.R, w.init_a_std,
                               w.init_b_std, w.init_dist)
    ft.set_params(A0, B0)
    return ft, T, A0, B0


def rel_norm(got, ref):
    num = np.sqrt(sum(np.sum((np.asarray(g, np.float64) - r) ** 2)
                      for g, r in zip(got, ref)))
    den = np.sqrt(sum(np.sum(np.asarray(r, np.float64) ** 2) for r in ref))
    return num / den if den > 0 else num


def minibatch_slice(T, perm, M, b):
    s = perm[b * M:(b + 1) * M]
    return (np.ascontiguousarray(T.train_idx[:, s]),
            T.train_val[s].astype(np.float64))
