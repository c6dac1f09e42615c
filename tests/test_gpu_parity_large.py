"""GPU parity at the shapes of the large workloads, on reduced tensors.

Order 4 (1,000,000 x 500,000 x 1,000 x 100, Zipf(1.2)) and order 5
(200,000 x 200,000 x 50,000 x 1,000 x 24, Zipf(1.1)), both with J = R = 32
and minibatches of 262,144 samples, but 700,000 nonzeros instead of 1e8 and
2e8 so that the FP64 oracle runs whole epochs. At that minibatch size every
wave of the factor kernel loops over several tiles with the next tile's
loads in flight, and the hottest rows (tens of thousands of samples of one
row in a minibatch) are summed in several parts: the code paths the full
workloads take.

Checks (same seeded inputs and injected orders on both sides):
  FP32: per-minibatch loss and row gradients (first, middle, last
        minibatch) to relative 1e-5, counts exact; core gradient to 1e-5;
        free-running epochs' train and test RMSE to 1e-4.
  BF16, FP8 e4m3: free-running test RMSE within 1% of the oracle's.
The oracle runs in its all-core form (its factor epoch is bitwise the serial
one; its core sums differ only in the order of the additions).
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2404_10087_amd import FT_TEST, FT_TRAIN
from tests.gpu_util import f64, minibatch_slice, rel_norm, setup

pytestmark = pytest.mark.gpu

LOSS_RTOL = 1e-5
GRAD_RTOL = 1e-5
RMSE_RTOL = 1e-4
LOWP_RTOL = 1e-2
NNZ = 700_000

W = {
    "order4_zipf1.2_J32": synth.get("c2", nnz=NNZ, data_seed=1202,
                                    init_seed=2202, order_seed=3202),
    "order5_zipf1.1_J32": synth.get("c3", nnz=NNZ, data_seed=1203,
                                    init_seed=2203, order_seed=3203),
}
_T = {}


def tensor(name):
    if name not in _T:
        _T[name] = synth.make_tensor(W[name])
    return _T[name]


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(0)
    yield


def perm_for(w, T, epoch=0):
    return synth.epoch_perm(w.order_seed, epoch, T.train_idx.shape[1])


@pytest.mark.parametrize("name", list(W))
def test_large_shape_minibatch_gradients_fp32(name):
    w = W[name]
    print(f"[large] minibatch gradients {name}", flush=True)
    ft, T, A0, B0 = setup(w, with_test=False, tensor=tensor(name))
    p = perm_for(w, T)
    ft.set_epoch_order(p)
    ft.prepare_epoch()
    nmb = ft.num_minibatches()
    assert nmb == 3
    for b in range(nmb):
        loss, G, K = ft.factor_minibatch(b, apply=False)
        idx, val = minibatch_slice(T, p, w.M, b)
        oloss, OG, OK = oracle.factor_minibatch(
            f64(A0), f64(B0), idx, val, w.lr_A, w.lam_A, w.row_mean,
            apply=False, want_grad=True, parallel=True)
        assert loss == pytest.approx(oloss, rel=LOSS_RTOL), b
        for n in range(w.order):
            np.testing.assert_array_equal(K[n], OK[n])
            err = rel_norm([G[n]], [OG[n]])
            assert err < GRAD_RTOL, (b, n, err)
        if b == 0:
            # the skew these shapes are about: some row of some mode holds
            # more than 16,384 samples of the minibatch (summed in parts)
            assert max(k.max() for k in K) > 16_384


@pytest.mark.parametrize("name", list(W))
def test_large_shape_core_gradient_fp32(name):
    w = W[name]
    print(f"[large] core gradient {name}", flush=True)
    ft, T, A0, B0 = setup(w, with_test=False, tensor=tensor(name))
    loss, G = ft.core_grad()
    oloss, OG = oracle.core_grad(f64(A0), f64(B0), T.train_idx,
                                 T.train_val.astype(np.float64),
                                 parallel=True)
    assert loss == pytest.approx(oloss, rel=LOSS_RTOL)
    for n in range(w.order):
        assert rel_norm([G[n]], [OG[n]]) < GRAD_RTOL, n


def _free_run(w, T, ft, A0, B0, epochs, check_each):
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    sv = T.test_val.astype(np.float64)
    out = []
    for ep in range(epochs):
        p = perm_for(w, T, ep)
        ft.set_epoch_order(p)
        ft.epoch_factors()
        ft.epoch_core()
        oracle.factor_epoch(A, B, T.train_idx, tv, p, w.M, w.lr_A, w.lam_A,
                            w.row_mean, parallel=True)
        oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B,
                          parallel=True)
        osse, _ = oracle.residual_stats(A, B, T.test_idx, sv, parallel=True)
        ormse, grmse = np.sqrt(osse / len(sv)), ft.rmse(FT_TEST)
        out.append((grmse, ormse))
        if check_each:
            check_each(ep, A, B, grmse, ormse)
    return out


@pytest.mark.parametrize("name", list(W))
def test_large_shape_free_running_fp32(name):
    w = W[name]
    print(f"[large] free-running fp32 {name}", flush=True)
    ft, T, A0, B0 = setup(w, tensor=tensor(name))
    tv = T.train_val.astype(np.float64)

    def check(ep, A, B, grmse, ormse):
        osse, _ = oracle.residual_stats(A, B, T.train_idx, tv, parallel=True)
        assert ft.rmse(FT_TRAIN) == pytest.approx(
            np.sqrt(osse / len(tv)), rel=RMSE_RTOL), ep
        assert grmse == pytest.approx(ormse, rel=RMSE_RTOL), ep

    out = _free_run(w, T, ft, A0, B0, 2, check)
    print(f"[large] {name} fp32 test RMSE per epoch (device, oracle): {out}")


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16", "fp8_e4m3"])
@pytest.mark.parametrize("name", list(W))
def test_large_shape_low_precision_within_one_percent(name, prec):
    w = W[name]
    print(f"[large] free-running precision {prec} {name}", flush=True)
    ft, T, A0, B0 = setup(w, tensor=tensor(name))
    ft.set_options(precision=prec)
    out = _free_run(w, T, ft, A0, B0, 3, None)
    print(f"[large] {name} precision {prec} test RMSE per epoch "
          f"(device, oracle): {out}")
    for ep, (g, o) in enumerate(out):
        assert np.isfinite(g), ep
    g, o = out[-1]
    assert g == pytest.approx(o, rel=LOWP_RTOL)
