"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
identical seeded inputs and identical minibatch orders.

Tolerances (FP32 device arithmetic against FP64):
  per-minibatch loss                relative 1e-5
  per-minibatch row / core gradient normwise relative 1e-5 per mode
  per-epoch train / test RMSE       relative 1e-4 (free-running epochs)
  integer builder output            bit-exact
Every checked minibatch starts both sides from the same seeded parameters.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2404_10087_amd import (FT_CORE_PER_MINIBATCH, FT_TEST, FT_TRAIN,
                                  FastTucker, FtError)
from tests import _fp8, _ref
from tests.gpu_util import EPS32, f64, minibatch_slice, rel_norm, setup

pytestmark = pytest.mark.gpu

LOSS_RTOL = 1e-5
GRAD_RTOL = 1e-5
RMSE_RTOL = 1e-4
FP8_RMSE_RTOL = 1e-2

W = {
    "c0": synth.get("c0"),
    "zipf": synth.get("c0", name="zipf-300x200x50", dims=(300, 200, 50),
                      nnz=40_000, J=16, R=16, M=8192, index_dist="zipf",
                      zipf_s=1.2, row_mean=True, init_a_std=0.3,
                      init_b_std=0.3),
    "pad_J3_R5": synth.get("c0", name="pad", dims=(40, 50, 30), nnz=3000, J=3,
                           R=5, M=256),
    "order2": synth.get("c0", name="o2", dims=(60, 70), nnz=2000, J=8, R=16,
                        M=128),
    "order4": synth.get("c0", name="o4", dims=(20, 30, 25, 10), nnz=4000, J=8,
                        R=16, M=300, init_a_std=0.4, init_b_std=0.4),
    "order5_J32_R32": synth.get("c0", name="o5", dims=(12, 10, 9, 8, 7),
                                nnz=3000, J=32, R=32, M=512, init_a_std=0.2,
                                init_b_std=0.2),
    "J12_R20": synth.get("c0", name="j12r20", dims=(50, 40, 30), nnz=3000,
                         J=12, R=20, M=400, init_a_std=0.3, init_b_std=0.3),
    "M1": synth.get("c0", name="m1", dims=(5, 6, 7), nnz=60, J=4, R=4, M=1),
    "nnz_lt_M": synth.get("c0", name="small", dims=(20, 20, 20), nnz=120,
                          J=4, R=4, M=512),
    # orders above 5 (FP32 verify path, J4 padded to 8 / 16 / 32); an
    # initial spread of 0.6 makes these products diverge on both sides
    "order6": synth.get("c0", name="o6", dims=(12, 10, 9, 8, 7, 6),
                        nnz=3000, J=8, R=16, M=400, init_a_std=0.45,
                        init_b_std=0.45),
    "order8_J12_R20": synth.get("c0", name="o8", dims=(9, 8, 7, 6, 5, 6, 7,
                                                       8),
                                nnz=3000, J=12, R=20, M=512, init_a_std=0.45,
                                init_b_std=0.45),
    "order10_J16": synth.get("c0", name="o10", dims=(6, 5, 7, 4, 6, 5, 4, 6,
                                                     5, 7),
                             nnz=4000, J=16, R=16, M=700, init_a_std=0.45,
                             init_b_std=0.45),
    # rows of ~20,000-30,000 samples per minibatch: long crossing rows
    # summed in several parts and combined
    "hot": synth.get("c0", name="hot", dims=(2000, 1500, 4), nnz=250_000,
                     J=16, R=16, M=65536, index_dist="zipf", zipf_s=1.1,
                     row_mean=True, init_a_std=0.3, init_b_std=0.3),
}


def perm_for(w, T, epoch=0):
    return synth.epoch_perm(w.order_seed, epoch, T.train_idx.shape[1])


# ----------------------------------------------------------------- eval
@pytest.mark.parametrize("name", ["c0", "pad_J3_R5", "order5_J32_R32",
                                  "J12_R20", "order6", "order8_J12_R20",
                                  "order10_J16"])
def test_eval_and_loss(name):
    w = W[name]
    ft, T, A0, B0 = setup(w)
    A, B = f64(A0), f64(B0)
    for which, idx, val in ((FT_TRAIN, T.train_idx, T.train_val),
                            (FT_TEST, T.test_idx, T.test_val)):
        sse, sae = ft.eval(which)
        osse, osae = oracle.residual_stats(A, B, idx, val.astype(np.float64))
        assert sse == pytest.approx(osse, rel=LOSS_RTOL)
        assert sae == pytest.approx(osae, rel=LOSS_RTOL)
        assert ft.rmse(which) == pytest.approx(np.sqrt(osse / len(val)),
                                               rel=LOSS_RTOL)
    ol = oracle.loss(A, B, T.train_idx, T.train_val.astype(np.float64),
                     w.lam_A, w.lam_B)
    assert ft.loss(FT_TRAIN) == pytest.approx(ol, rel=LOSS_RTOL)


# ----------------------------------------------------------------- builder
@pytest.mark.parametrize("name", ["c0", "zipf", "M1", "nnz_lt_M"])
def test_epoch_order_and_minibatch_sort_bit_exact(name):
    w = W[name]
    ft, T, _, _ = setup(w, with_test=False)
    ft.set_options(shuffle_seed=77)
    nnz = T.train_idx.shape[1]
    ft.prepare_epoch()
    perm = ft.epoch_order()
    ref = _ref.feistel_order(nnz, _ref.epoch_key(77, 0))
    np.testing.assert_array_equal(perm, ref)
    nmb = ft.num_minibatches()
    assert nmb == -(-nnz // w.M)
    for b in sorted({0, nmb // 2, nmb - 1}):
        s = perm[b * w.M:(b + 1) * w.M]
        for n in range(w.order):
            pos, rows = ft.minibatch_sort(b, n)
            rpos, rrows = _ref.minibatch_sort(T.train_idx[n, s])
            np.testing.assert_array_equal(pos, rpos)
            np.testing.assert_array_equal(rows, rrows)


def test_injected_order_is_used():
    w = W["c0"]
    ft, T, _, _ = setup(w, with_test=False)
    p = perm_for(w, T, 5)
    ft.set_epoch_order(p)
    ft.prepare_epoch()
    np.testing.assert_array_equal(ft.epoch_order(), p)
    with pytest.raises(FtError):
        bad = p.copy()
        bad[0] = bad[1]
        ft.set_epoch_order(bad)


# ----------------------------------------------------------------- factor
@pytest.mark.parametrize("name", list(W))
def test_factor_minibatch_gradients(name):
    w = W[name]
    ft, T, A0, B0 = setup(w, with_test=False)
    p = perm_for(w, T)
    ft.set_epoch_order(p)
    ft.prepare_epoch()
    nmb = ft.num_minibatches()
    for b in sorted({0, nmb // 2, nmb - 1}):
        loss, G, K = ft.factor_minibatch(b, apply=False)
        idx, val = minibatch_slice(T, p, w.M, b)
        A, B = f64(A0), f64(B0)
        oloss, OG, OK = oracle.factor_minibatch(A, B, idx, val, w.lr_A,
                                                w.lam_A, w.row_mean,
                                                apply=False, want_grad=True)
        assert loss == pytest.approx(oloss, rel=LOSS_RTOL)
        for n in range(w.order):
            np.testing.assert_array_equal(K[n], OK[n])
            err = rel_norm([G[n]], [OG[n]])
            assert err < GRAD_RTOL, (b, n, err)


@pytest.mark.parametrize("name,row_mean", [("c0", False), ("c0", True),
                                           ("zipf", True), ("order4", False),
                                           ("pad_J3_R5", True), ("hot", True),
                                           ("hot", False), ("order6", True),
                                           ("order10_J16", False)])
def test_factor_minibatch_update(name, row_mean):
    w = W[name]
    ft, T, A0, B0 = setup(w, with_test=False)
    ft.set_options(row_scale=int(row_mean))
    p = perm_for(w, T)
    ft.set_epoch_order(p)
    ft.prepare_epoch()
    b = ft.num_minibatches() // 2
    loss = ft.factor_minibatch(b, apply=True)
    A1, B1 = ft.get_params()
    idx, val = minibatch_slice(T, p, w.M, b)
    A, B = f64(A0), f64(B0)
    oloss = oracle.factor_minibatch(A, B, idx, val, w.lr_A, w.lam_A, row_mean)
    assert loss == pytest.approx(oloss, rel=LOSS_RTOL)
    for n in range(w.order):
        np.testing.assert_array_equal(B1[n], B0[n])
        d_gpu = A1[n].astype(np.float64) - A0[n]
        d_orc = A[n] - A0[n]
        # the update itself to 1e-5, plus the rounding of the stored FP32 A
        tol = GRAD_RTOL * np.linalg.norm(d_orc) + \
            2 * EPS32 * np.linalg.norm(A[n])
        assert np.linalg.norm(d_gpu - d_orc) <= tol, n


@pytest.mark.parametrize("name", ["c0", "order4", "zipf", "order6",
                                  "order10_J16"])
def test_free_running_epochs(name):
    """Alternating factor and core epochs on both sides from the same start
    and orders: per-epoch train/test RMSE to 1e-4, first-epoch minibatch
    losses to 1e-5."""
    w = W[name]
    ft, T, A0, B0 = setup(w)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    sv = T.test_val.astype(np.float64)
    for ep in range(w.epochs):
        p = perm_for(w, T, ep)
        ft.set_epoch_order(p)
        mb = ft.epoch_factors()
        omb = oracle.factor_epoch(A, B, T.train_idx, tv, p, w.M, w.lr_A,
                                  w.lam_A, w.row_mean)
        if ep == 0:
            np.testing.assert_allclose(mb, omb, rtol=LOSS_RTOL)
        cl = ft.epoch_core()
        ocl = oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B)
        assert cl == pytest.approx(ocl, rel=RMSE_RTOL)
        for which, idx, val in ((FT_TRAIN, T.train_idx, tv),
                                (FT_TEST, T.test_idx, sv)):
            osse, _ = oracle.residual_stats(A, B, idx, val)
            assert ft.rmse(which) == pytest.approx(
                np.sqrt(osse / len(val)), rel=RMSE_RTOL), (ep, which)


# ----------------------------------------------------------------- core
@pytest.mark.parametrize("name", ["c0", "pad_J3_R5", "order2", "order4",
                                  "order5_J32_R32", "J12_R20", "zipf",
                                  "order6", "order8_J12_R20", "order10_J16"])
def test_core_gradient_and_update(name):
    w = W[name]
    ft, T, A0, B0 = setup(w, with_test=False)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    loss, G = ft.core_grad()
    oloss, OG = oracle.core_grad(A, B, T.train_idx, tv)
    assert loss == pytest.approx(oloss, rel=LOSS_RTOL)
    for n in range(w.order):
        assert rel_norm([G[n]], [OG[n]]) < GRAD_RTOL, n
    cl = ft.epoch_core()
    assert cl == pytest.approx(oloss, rel=LOSS_RTOL)
    oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B)
    A1, B1 = ft.get_params()
    for n in range(w.order):
        np.testing.assert_array_equal(A1[n], A0[n])
        d_gpu = B1[n].astype(np.float64) - B0[n]
        d_orc = B[n] - B0[n]
        tol = GRAD_RTOL * np.linalg.norm(d_orc) + \
            2 * EPS32 * np.linalg.norm(B[n])
        assert np.linalg.norm(d_gpu - d_orc) <= tol, n


def test_core_per_minibatch_steps():
    w = W["c0"]
    ft, T, A0, B0 = setup(w, with_test=False)
    ft.set_options(core_step=FT_CORE_PER_MINIBATCH)
    p = perm_for(w, T, 2)
    ft.set_epoch_order(p)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    cl = ft.epoch_core()
    ocl = oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B, perm=p,
                            M=w.M, per_minibatch=True)
    assert cl == pytest.approx(ocl, rel=RMSE_RTOL)
    _, B1 = ft.get_params()
    assert rel_norm(B1, B) < RMSE_RTOL


# ----------------------------------------------------------------- properties
def test_bitwise_reproducible():
    """Verify mode has no float atomics: two runs from the same state agree
    bit for bit (the race check of the deterministic path)."""
    w = W["zipf"]
    outs = []
    for _ in range(2):
        ft, T, A0, B0 = setup(w, with_test=False)
        ft.set_options(shuffle_seed=5)
        l1 = ft.epoch_factors()
        l2 = ft.epoch_core()
        l3 = ft.epoch_factors()
        A, B = ft.get_params()
        outs.append((l1, l2, l3, A, B))
        ft.close()
    (a1, a2, a3, aA, aB), (b1, b2, b3, bA, bB) = outs
    np.testing.assert_array_equal(a1, b1)
    assert a2 == b2
    np.testing.assert_array_equal(a3, b3)
    for x, y in zip(aA + aB, bA + bB):
        np.testing.assert_array_equal(x, y)


def test_zero_learning_rate_leaves_parameters():
    w = W["c0"]
    ft, T, A0, B0 = setup(w)
    ft.set_options(lr_A=0.0, lr_B=0.0)
    l0 = ft.loss(FT_TRAIN)
    ft.epoch_factors()
    ft.epoch_core()
    A1, B1 = ft.get_params()
    for x, y in zip(A1 + B1, A0 + B0):
        np.testing.assert_array_equal(x, y)
    assert ft.loss(FT_TRAIN) == l0


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("where", ["A", "B"])
@pytest.mark.parametrize("value", [np.nan, np.inf])
def test_nonfinite_parameter_is_reported(prec, where, value):
    """A NaN or an infinity in a factor or core matrix makes the epoch fail
    with FT_ENONFINITE in every contraction precision (the low-precision
    shadows and operands must not turn it into a finite code)."""
    w = W["c0"]
    ft, T, A0, B0 = setup(w, with_test=False)
    ft.set_options(precision=prec)
    if where == "A":
        A0[1][3, 2] = value
        ft.set_params(A=A0)
    else:
        B0[2][1, 3] = value
        ft.set_params(B=B0)
    with pytest.raises(FtError) as e:
        ft.epoch_factors()
    assert e.value.status == 5


def test_bad_nonzeros_leave_state_unchanged():
    w = W["c0"]
    ft, T, A0, B0 = setup(w)
    r0 = ft.rmse(FT_TEST)
    bad = T.test_idx.copy()
    bad[2, 7] = w.dims[2]
    with pytest.raises(FtError) as e:
        ft.set_nonzeros(FT_TEST, bad, T.test_val)
    assert e.value.status == 1
    assert ft.rmse(FT_TEST) == r0


def test_empty_test_set():
    w = W["c0"]
    ft, T, _, _ = setup(w, with_test=False)
    ft.set_nonzeros(FT_TEST, np.zeros((3, 0), np.int32), np.zeros(0, np.float32))
    assert ft.rmse(FT_TEST) == 0.0
    assert ft.eval(FT_TEST) == (0.0, 0.0)


def test_unequal_ranks_per_mode():
    dims, J, R = (30, 40, 20), (3, 8, 5), 6
    T = synth.make_tensor(synth.get("c0", dims=dims, nnz=2000, J=4, R=4))
    A0, B0 = synth.init_params(9, dims, list(J), R, 0.4)
    ft = FastTucker(dims, list(J), R)
    ft.set_options(minibatch=128, lr_A=0.02, lambda_A=0.01)
    ft.set_nonzeros(FT_TRAIN, T.train_idx, T.train_val)
    ft.set_params(A0, B0)
    p = synth.epoch_perm(1, 0, T.train_idx.shape[1])
    ft.set_epoch_order(p)
    ft.prepare_epoch()
    loss, G, K = ft.factor_minibatch(3, apply=False)
    idx, val = minibatch_slice(T, p, 128, 3)
    ol, OG, OK = oracle.factor_minibatch(f64(A0), f64(B0), idx, val, 0.02,
                                         0.01, False, apply=False,
                                         want_grad=True)
    assert loss == pytest.approx(ol, rel=LOSS_RTOL)
    for n in range(3):
        np.testing.assert_array_equal(K[n], OK[n])
        assert rel_norm([G[n]], [OG[n]]) < GRAD_RTOL
    l2, CG = ft.core_grad()
    _, OCG = oracle.core_grad(f64(A0), f64(B0), T.train_idx,
                              T.train_val.astype(np.float64))
    for n in range(3):
        assert rel_norm([CG[n]], [OCG[n]]) < GRAD_RTOL


# ----------------------------------------------------------------- fast mode
def test_hogwild_fast_mode_tracks_sequential_tiles():
    """The fast mode applies per-sample steps from concurrent 16-sample tiles
    with float atomics (no determinism). On uniformly spread rows its
    trajectory stays close to the oracle's sequential execution of the same
    tiles (M = 16, summed rows) on the same order: test RMSE after three
    alternating epochs within 2%."""
    w = W["c0"]
    ft, T, A0, B0 = setup(w)
    ft.set_options(deterministic=0, row_scale=0)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    sv = T.test_val.astype(np.float64)
    for ep in range(3):
        p = perm_for(w, T, ep)
        ft.set_epoch_order(p)
        mb = ft.epoch_factors()
        assert mb.shape == (ft.num_minibatches(),) and np.all(np.isfinite(mb))
        oracle.factor_epoch(A, B, T.train_idx, tv, p, 16, w.lr_A, w.lam_A,
                            False)
        ft.epoch_core()
        oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B)
    osse, _ = oracle.residual_stats(A, B, T.test_idx, sv)
    ormse = np.sqrt(osse / len(sv))
    assert ft.rmse(FT_TEST) == pytest.approx(ormse, rel=0.02)


@pytest.mark.parametrize("lr", [1e-3, 3e-3])
def test_hogwild_fast_mode_on_skewed_rows_tracks_sequential_tiles(lr):
    """Zipf(1.2) rows (the hottest rows appear in hundreds of tiles of one
    epoch): the fast mode runs every tile at once, so a hot row takes steps
    computed from stale values; the oracle runs the same 16-sample tiles one
    after another (M = 16, summed rows). Statistical tolerance: after three
    alternating epochs the test RMSE is within 1% of the oracle's (measured
    0.3-0.4% at these steps, which move the RMSE by 5-7%), and the epoch
    improves on the initial point like the oracle's."""
    w = W["zipf"]
    ft, T, A0, B0 = setup(w)
    ft.set_options(deterministic=0, row_scale=0, lr_A=lr)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    sv = T.test_val.astype(np.float64)
    r0 = ft.rmse(FT_TEST)
    for ep in range(3):
        p = perm_for(w, T, ep)
        ft.set_epoch_order(p)
        assert np.all(np.isfinite(ft.epoch_factors()))
        ft.epoch_core()
        oracle.factor_epoch(A, B, T.train_idx, tv, p, 16, lr, w.lam_A, False)
        oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B)
    osse, _ = oracle.residual_stats(A, B, T.test_idx, sv)
    ormse = np.sqrt(osse / len(sv))
    g = ft.rmse(FT_TEST)
    print(f"hogwild zipf lr {lr}: device {g:.6f} oracle {ormse:.6f} "
          f"initial {r0:.6f}")
    assert ormse < 0.97 * r0
    assert g == pytest.approx(ormse, rel=0.01)


def test_fast_mode_rejects_minibatch_not_multiple_of_tile():
    w = W["c0"]
    ft, T, _, _ = setup(w, with_test=False)
    with pytest.raises(FtError) as e:
        ft.set_options(deterministic=0, minibatch=500)
    assert e.value.status == 1


# ----------------------------------------------------------------- BF16
@pytest.mark.parametrize("name", ["c0", "zipf", "order5_J32_R32"])
def test_bf16_contraction_training_within_one_percent(name):
    """BF16 contraction (FP32 masters and updates): after free-running
    alternating epochs the test RMSE is within 1% of the FP64 oracle's."""
    w = W[name]
    ft, T, A0, B0 = setup(w)
    ft.set_options(precision=1)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    sv = T.test_val.astype(np.float64)
    osse0, _ = oracle.residual_stats(A, B, T.test_idx, sv)
    assert ft.rmse(FT_TEST) == pytest.approx(np.sqrt(osse0 / len(sv)),
                                             rel=1e-2)
    for ep in range(w.epochs):
        p = perm_for(w, T, ep)
        ft.set_epoch_order(p)
        ft.epoch_factors()
        ft.epoch_core()
        oracle.factor_epoch(A, B, T.train_idx, tv, p, w.M, w.lr_A, w.lam_A,
                            w.row_mean)
        oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B)
    osse, _ = oracle.residual_stats(A, B, T.test_idx, sv)
    assert ft.rmse(FT_TEST) == pytest.approx(np.sqrt(osse / len(sv)),
                                             rel=1e-2)
    # switching back to FP32 evaluates the FP32 masters
    ft.set_options(precision=0)
    A1, B1 = ft.get_params()
    gsse, _ = oracle.residual_stats(f64(A1), f64(B1), T.test_idx, sv)
    assert ft.rmse(FT_TEST) == pytest.approx(np.sqrt(gsse / len(sv)),
                                             rel=LOSS_RTOL)


def test_bf16_shadow_follows_set_params():
    w = W["c0"]
    ft, T, A0, B0 = setup(w, with_test=False)
    ft.set_options(precision=1)
    r1 = ft.rmse(FT_TRAIN)
    A2, B2 = synth.init_params(77, w.dims, w.J, w.R, 0.4)
    ft.set_params(A2, B2)
    osse, _ = oracle.residual_stats(f64(A2), f64(B2), T.train_idx,
                                    T.train_val.astype(np.float64))
    r2 = ft.rmse(FT_TRAIN)
    assert r2 != r1
    assert r2 == pytest.approx(np.sqrt(osse / T.train_idx.shape[1]), rel=1e-2)
    with pytest.raises(FtError):
        ft.set_options(deterministic=0)


# ----------------------------------------------------------------- FP8
@pytest.mark.parametrize("name", ["c0", "J12_R20", "order5_J32_R32", "zipf"])
def test_fp8_contraction_matches_emulated_quantisation(name):
    """FP8 e4m3 contraction: every row of A is quantised with one scale per
    row and every column of B with one scale per column (the codes and
    scales of the format definition, tests/_fp8.py). The device's SSE and
    SAE equal the FP64 oracle's on the dequantised parameters, before and
    after a factor epoch, so the shadow rows rewritten by the row updates
    are checked too."""
    w = W[name]
    ft, T, _, _ = setup(w)
    ft.set_options(precision=2)
    for step in range(2):
        A1, B1 = ft.get_params()
        Aq = [_fp8.quantize(a, axis=1) for a in A1]
        Bq = [_fp8.quantize(b, axis=0) for b in B1]
        for which, idx, val in ((FT_TRAIN, T.train_idx, T.train_val),
                                (FT_TEST, T.test_idx, T.test_val)):
            sse, sae = ft.eval(which)
            osse, osae = oracle.residual_stats(Aq, Bq, idx,
                                               val.astype(np.float64))
            assert sse == pytest.approx(osse, rel=LOSS_RTOL)
            assert sae == pytest.approx(osae, rel=LOSS_RTOL)
        if step == 0:
            ft.set_epoch_order(perm_for(w, T))
            ft.epoch_factors()


@pytest.mark.parametrize("name", ["c0", "zipf"])
def test_fp8_contraction_training_tracks_oracle(name):
    """FP8 contraction (FP32 masters, FP32 gradient product and updates):
    after free-running alternating epochs the test RMSE stays within
    FP8_RMSE_RTOL of the FP64 oracle's; switching back to FP32 evaluates
    the FP32 masters exactly."""
    w = W[name]
    ft, T, A0, B0 = setup(w)
    ft.set_options(precision=2)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    sv = T.test_val.astype(np.float64)
    for ep in range(w.epochs):
        p = perm_for(w, T, ep)
        ft.set_epoch_order(p)
        ft.epoch_factors()
        ft.epoch_core()
        oracle.factor_epoch(A, B, T.train_idx, tv, p, w.M, w.lr_A, w.lam_A,
                            w.row_mean)
        oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B)
    osse, _ = oracle.residual_stats(A, B, T.test_idx, sv)
    ormse, grmse = np.sqrt(osse / len(sv)), ft.rmse(FT_TEST)
    print(f"fp8 {name}: device {grmse:.6g} oracle {ormse:.6g} "
          f"rel {abs(grmse / ormse - 1):.3g}")
    assert grmse == pytest.approx(ormse, rel=FP8_RMSE_RTOL)
    ft.set_options(precision=0)
    A1, B1 = ft.get_params()
    gsse, _ = oracle.residual_stats(f64(A1), f64(B1), T.test_idx, sv)
    assert ft.rmse(FT_TEST) == pytest.approx(np.sqrt(gsse / len(sv)),
                                             rel=LOSS_RTOL)


def test_fp8_needs_verify_mode():
    w = W["c0"]
    ft, _, _, _ = setup(w, with_test=False)
    ft.set_options(precision=2)
    with pytest.raises(FtError):
        ft.set_options(deterministic=0)


# ----------------------------------------------------------------- builder ahead
def test_epoch_builder_ahead_matches_injected_orders():
    """The next epoch's order, permutation and sort are built on a second
    stream while the current epoch's core phase runs. Epochs that use those
    sets give
    bitwise the same parameters as epochs whose orders (the same
    counter-based permutations, from their definition) are injected one by
    one and built in line."""
    w = W["zipf"]
    ft1, T, _, _ = setup(w, with_test=False)
    ft2, _, _, _ = setup(w, with_test=False)
    for ft in (ft1, ft2):
        ft.set_options(shuffle_seed=91, reshuffle_each_epoch=1)
    nnz = T.train_idx.shape[1]
    for ep in range(3):
        ft1.epoch_factors()
        ft1.epoch_core()
        ft2.set_epoch_order(_ref.feistel_order(nnz, _ref.epoch_key(91, ep)))
        ft2.epoch_factors()
        ft2.epoch_core()
    A1, B1 = ft1.get_params()
    A2, B2 = ft2.get_params()
    for a1, a2 in zip(A1 + B1, A2 + B2):
        assert np.array_equal(a1, a2)


# ----------------------------------------------------------------- vector ALU
@pytest.mark.parametrize("name", ["c0", "zipf", "hot", "order4",
                                  "order5_J32_R32", "M1", "nnz_lt_M",
                                  "pad_J3_R5"])
def test_vector_alu_factor_kernel_matches_oracle(name):
    """The matrix-core ablation's factor kernel (vector FP32 FMAs, one sample
    per lane) gives the same minibatch losses, row gradients and counts as
    the oracle, to the same tolerance as the matrix-core kernel."""
    w = W[name]
    ft, T, A0, B0 = setup(w, with_test=False)
    ft.set_options(vector_alu=1)
    p = perm_for(w, T)
    ft.set_epoch_order(p)
    ft.prepare_epoch()
    nmb = ft.num_minibatches()
    for b in sorted({0, nmb - 1}):
        loss, G, K = ft.factor_minibatch(b, apply=False)
        idx, val = minibatch_slice(T, p, w.M, b)
        oloss, OG, OK = oracle.factor_minibatch(f64(A0), f64(B0), idx, val,
                                                w.lr_A, w.lam_A, w.row_mean,
                                                apply=False, want_grad=True)
        assert loss == pytest.approx(oloss, rel=LOSS_RTOL)
        for n in range(w.order):
            np.testing.assert_array_equal(K[n], OK[n])
            assert rel_norm([G[n]], [OG[n]]) < GRAD_RTOL, (b, n)


@pytest.mark.parametrize("name", ["c0", "pad_J3_R5", "order2", "order4",
                                  "order5_J32_R32", "J12_R20", "zipf", "M1",
                                  "nnz_lt_M"])
def test_vector_alu_core_gradient_matches_oracle(name):
    """The matrix-core ablation's core kernel (register-blocked outer
    products on vector FMAs) gives the oracle's core loss, gradient and
    update."""
    w = W[name]
    ft, T, A0, B0 = setup(w, with_test=False)
    ft.set_options(vector_alu=1)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    loss, G = ft.core_grad()
    oloss, OG = oracle.core_grad(A, B, T.train_idx, tv)
    assert loss == pytest.approx(oloss, rel=LOSS_RTOL)
    for n in range(w.order):
        assert rel_norm([G[n]], [OG[n]]) < GRAD_RTOL, n
    cl = ft.epoch_core()
    assert cl == pytest.approx(oloss, rel=LOSS_RTOL)
    oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B)
    _, B1 = ft.get_params()
    for n in range(w.order):
        d_gpu = B1[n].astype(np.float64) - B0[n]
        d_orc = B[n] - B0[n]
        tol = GRAD_RTOL * np.linalg.norm(d_orc) + \
            2 * EPS32 * np.linalg.norm(B[n])
        assert np.linalg.norm(d_gpu - d_orc) <= tol, n


def test_vector_alu_core_per_minibatch_steps():
    w = W["c0"]
    ft, T, A0, B0 = setup(w, with_test=False)
    ft.set_options(core_step=FT_CORE_PER_MINIBATCH, vector_alu=1)
    p = perm_for(w, T, 2)
    ft.set_epoch_order(p)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    cl = ft.epoch_core()
    ocl = oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B, perm=p,
                            M=w.M, per_minibatch=True)
    assert cl == pytest.approx(ocl, rel=RMSE_RTOL)
    _, B1 = ft.get_params()
    assert rel_norm(B1, B) < RMSE_RTOL


def test_vector_alu_rejects_unsupported_settings():
    ft, _, _, _ = setup(W["c0"], with_test=False)
    ft.set_options(precision=1)
    with pytest.raises(FtError):
        ft.set_options(vector_alu=1)          # BF16
    ft.set_options(precision=0, deterministic=0)
    with pytest.raises(FtError):
        ft.set_options(vector_alu=1)          # Hogwild fast mode


# ----------------------------------------------------------------- storage
@pytest.mark.parametrize("name", ["c0", "pad_J3_R5", "order2", "order4",
                                  "order5_J32_R32", "J12_R20", "zipf", "M1",
                                  "nnz_lt_M"])
def test_core_storage_variant_matches_oracle(name):
    """The storage form of the core phase (C = A B stored once per pass, rows
    of C gathered per sample) gives the oracle's core loss, gradient and
    update to the calculation form's tolerances."""
    w = W[name]
    ft, T, A0, B0 = setup(w, with_test=False)
    ft.set_options(core_storage=1)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    loss, G = ft.core_grad()
    oloss, OG = oracle.core_grad(A, B, T.train_idx, tv)
    assert loss == pytest.approx(oloss, rel=LOSS_RTOL)
    for n in range(w.order):
        assert rel_norm([G[n]], [OG[n]]) < GRAD_RTOL, n
    cl = ft.epoch_core()
    assert cl == pytest.approx(oloss, rel=LOSS_RTOL)
    oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B)
    A1, B1 = ft.get_params()
    for n in range(w.order):
        np.testing.assert_array_equal(A1[n], A0[n])
        d_gpu = B1[n].astype(np.float64) - B0[n]
        d_orc = B[n] - B0[n]
        tol = GRAD_RTOL * np.linalg.norm(d_orc) + \
            2 * EPS32 * np.linalg.norm(B[n])
        assert np.linalg.norm(d_gpu - d_orc) <= tol, n


def test_core_storage_per_minibatch_steps_and_free_running():
    """Per-minibatch core steps re-store C after every step of B; free-
    running alternating epochs with the storage form track the oracle's
    per-epoch RMSE to 1e-4."""
    w = W["zipf"]
    ft, T, A0, B0 = setup(w)
    ft.set_options(core_storage=1, core_step=FT_CORE_PER_MINIBATCH)
    p = perm_for(w, T, 2)
    ft.set_epoch_order(p)
    A, B = f64(A0), f64(B0)
    tv = T.train_val.astype(np.float64)
    cl = ft.epoch_core()
    ocl = oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B, perm=p,
                            M=w.M, per_minibatch=True)
    assert cl == pytest.approx(ocl, rel=RMSE_RTOL)
    _, B1 = ft.get_params()
    assert rel_norm(B1, B) < RMSE_RTOL
    ft.set_options(core_step=0)
    sv = T.test_val.astype(np.float64)
    for ep in range(3):
        p = perm_for(w, T, ep)
        ft.set_epoch_order(p)
        ft.epoch_factors()
        ft.epoch_core()
        oracle.factor_epoch(A, B, T.train_idx, tv, p, w.M, w.lr_A, w.lam_A,
                            w.row_mean)
        oracle.core_epoch(A, B, T.train_idx, tv, w.lr_B, w.lam_B)
        osse, _ = oracle.residual_stats(A, B, T.test_idx, sv)
        assert ft.rmse(FT_TEST) == pytest.approx(np.sqrt(osse / len(sv)),
                                                 rel=RMSE_RTOL), ep


def test_core_storage_rejects_unsupported_settings():
    ft, _, _, _ = setup(W["c0"], with_test=False)
    for bad in ({"precision": 1}, {"deterministic": 0}, {"vector_alu": 1}):
        ft.set_options(precision=0, deterministic=1, vector_alu=0,
                       core_storage=0)
        ft.set_options(**bad)
        with pytest.raises(FtError):
            ft.set_options(core_storage=1)


# ----------------------------------------------------------------- high orders
def test_high_order_unequal_ranks_and_builder():
    """Order 7 with unequal J_n (A rows padded to 16) and R = 24: minibatch
    gradients and counts, the core gradient, and the bit-exact builder
    (records of 16 words above order 7 are exercised by order 8 and 10)."""
    dims, J, R = (9, 11, 8, 7, 10, 6, 5), (3, 12, 5, 7, 2, 9, 4), 24
    T = synth.make_tensor(synth.get("c0", dims=dims, nnz=3000, J=4, R=4))
    A0, B0 = synth.init_params(19, dims, list(J), R, 0.7)
    ft = FastTucker(dims, list(J), R)
    ft.set_options(minibatch=256, lr_A=0.02, lambda_A=0.01, shuffle_seed=8)
    ft.set_nonzeros(FT_TRAIN, T.train_idx, T.train_val)
    ft.set_params(A0, B0)
    ft.prepare_epoch()
    perm = ft.epoch_order()
    nnz = T.train_idx.shape[1]
    np.testing.assert_array_equal(perm,
                                  _ref.feistel_order(nnz, _ref.epoch_key(8, 0)))
    for b in (0, ft.num_minibatches() - 1):
        loss, G, K = ft.factor_minibatch(b, apply=False)
        s = perm[b * 256:(b + 1) * 256]
        idx = np.ascontiguousarray(T.train_idx[:, s])
        val = T.train_val[s].astype(np.float64)
        ol, OG, OK = oracle.factor_minibatch(f64(A0), f64(B0), idx, val, 0.02,
                                             0.01, False, apply=False,
                                             want_grad=True)
        assert loss == pytest.approx(ol, rel=LOSS_RTOL)
        for n in range(7):
            np.testing.assert_array_equal(K[n], OK[n])
            assert rel_norm([G[n]], [OG[n]]) < GRAD_RTOL, (b, n)
            pos, rows = ft.minibatch_sort(b, n)
            rpos, rrows = _ref.minibatch_sort(T.train_idx[n, s])
            np.testing.assert_array_equal(pos, rpos)
            np.testing.assert_array_equal(rows, rrows)
    l2, CG = ft.core_grad()
    _, OCG = oracle.core_grad(f64(A0), f64(B0), T.train_idx,
                              T.train_val.astype(np.float64))
    for n in range(7):
        assert rel_norm([CG[n]], [OCG[n]]) < GRAD_RTOL, n


@pytest.mark.parametrize("opts", [{"precision": 1}, {"precision": 2},
                                  {"deterministic": 0}, {"vector_alu": 1},
                                  {"core_storage": 1}])
def test_high_orders_reject_the_variants(opts):
    ft, _, _, _ = setup(W["order6"], with_test=False)
    with pytest.raises(FtError) as e:
        ft.set_options(**opts)
    assert e.value.status == 1
