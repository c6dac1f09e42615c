"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself:
  * brute-force dense Tucker (Eq. (1) with the Kruskal core of Eq. (2)),
    built with numpy tensordot -- P1;
  * torch autograd through that dense-Tucker graph, for the factor-row and
    core gradients of Eqs. (8)/(9), (12)/(13) and the minibatch Jacobi
    semantics of Algorithm 3 -- P2/P5;
  * central finite differences of the oracle's own prediction -- P2;
  * closed forms: zero learning rate, residual-free decay, the
    matrix-factorisation special case -- P3/P4/P6;
  * invariances: gauge, sample order (Algorithm 5 is a sum), zero padding of
    J and R -- P7/P8/P9;
  * recovery of a planted tensor to its noise level -- P10.
Shapes use J_n != R and unequal J_n so that a transposed operand or a swapped
index cannot pass.
"""
import numpy as np
import pytest
import torch

import synth

RNG = np.random.default_rng(12345)


def rand_problem(dims, J, R, nnz, seed, std=0.6):
    rng = np.random.default_rng(seed)
    N = len(dims)
    A = [rng.normal(0, std, size=(dims[n], J[n])) for n in range(N)]
    B = [rng.normal(0, std, size=(J[n], R)) for n in range(N)]
    idx = np.stack([rng.integers(0, dims[n], size=nnz) for n in range(N)]
                   ).astype(np.int32)
    vals = rng.normal(0, 1, size=nnz)
    return A, B, idx, vals


# ---------------------------------------------------------------- P1 -------
def dense_tucker_predict(A, B, idx):
    """Eq. (2): G = sum_r b1_r o ... o bN_r ; Eq. (1): n-mode products."""
    N = len(A)
    R = B[0].shape[1]
    G = np.zeros([b.shape[0] for b in B])
    for r in range(R):
        t = B[0][:, r]
        for n in range(1, N):
            t = np.multiply.outer(t, B[n][:, r])
        G += t
    out = np.empty(idx.shape[1])
    for s in range(idx.shape[1]):
        t = G
        for n in range(N):       # contract the leading mode each time
            t = np.tensordot(A[n][idx[n, s]], t, axes=([0], [0]))
        out[s] = float(t)
    return out


@pytest.mark.parametrize("dims,J,R", [
    ((4, 5), (2, 3), 3),
    ((4, 5, 6), (2, 3, 4), 3),
    ((3, 4, 5, 2), (2, 3, 2, 3), 5),
    ((3, 3, 3, 3, 3), (2, 1, 2, 3, 2), 2),
])
def test_p1_dense_tucker_brute_force(oracle_mod, dims, J, R):
    A, B, idx, _ = rand_problem(dims, J, R, 40, seed=sum(dims) + R)
    ref = dense_tucker_predict(A, B, idx)
    got = oracle_mod.predict(A, B, idx)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


# ------------------------------------------- autograd through dense Tucker --
def torch_dense_xhat(At, Bt, idx):
    """xhat via the dense Tucker core (Eqs. (1)-(2)) in torch, differentiable;
    shares nothing with the oracle's Eq. (3) loops."""
    N = len(At)
    R = Bt[0].shape[1]
    G = None
    for r in range(R):
        t = Bt[0][:, r]
        for n in range(1, N):
            t = torch.tensordot(t, Bt[n][:, r], dims=0)
        G = t if G is None else G + t
    rows = [At[n][torch.as_tensor(idx[n].astype(np.int64))]
            for n in range(N)]
    # contract every mode of G with the gathered rows, batched over samples
    t = G.unsqueeze(0).expand(idx.shape[1], *G.shape)
    for n in range(N):
        t = torch.einsum("sj,sj...->s...", rows[n], t)
    return t


def torch_minibatch_grads(A, B, idx, vals, lamA):
    """d/dA and d/dB of sum_s r_s^2/2 + lamA/2 sum_s sum_n ||a^(n)_{i_n}||^2."""
    At = [torch.tensor(a, requires_grad=True) for a in A]
    Bt = [torch.tensor(b, requires_grad=True) for b in B]
    xh = torch_dense_xhat(At, Bt, idx)
    r = xh - torch.as_tensor(vals)
    f = 0.5 * (r * r).sum()
    for n in range(len(A)):
        rows = At[n][torch.as_tensor(idx[n].astype(np.int64))]
        f = f + 0.5 * lamA * (rows * rows).sum()
    f.backward()
    return ([a.grad.numpy() for a in At], [b.grad.numpy() for b in Bt],
            float(0.5 * (r * r).sum().detach()))


@pytest.mark.parametrize("dims,J,R,m,seed", [
    ((6, 7, 5), (2, 3, 4), 3, 60, 1),
    ((5, 4, 6, 3), (3, 2, 2, 3), 4, 80, 2),
    ((4, 5), (3, 2), 5, 30, 3),
])
def test_p2_factor_and_core_gradients_vs_autograd(oracle_mod, dims, J, R, m,
                                                  seed):
    A, B, idx, vals = rand_problem(dims, J, R, m, seed)
    lam = 0.03
    gA, gB, ref_loss = torch_minibatch_grads(A, B, idx, vals, lam)
    Acopy = [a.copy() for a in A]
    loss, G, cnt = oracle_mod.factor_minibatch(Acopy, B, idx, vals, 0.1, lam,
                                               row_mean=False, apply=False,
                                               want_grad=True)
    assert loss == pytest.approx(ref_loss, rel=1e-12)
    for n in range(len(A)):
        np.testing.assert_allclose(G[n], gA[n], rtol=1e-10, atol=1e-12)
        np.testing.assert_array_equal(cnt[n], np.bincount(idx[n],
                                                          minlength=dims[n]))
        np.testing.assert_array_equal(Acopy[n], A[n])   # apply=False
    # core gradient (data term only; Algorithm 5 accumulation)
    _, gB0, _ = torch_minibatch_grads(A, B, idx, vals, 0.0)
    closs, Grad = oracle_mod.core_grad(A, B, idx, vals)
    assert closs == pytest.approx(ref_loss, rel=1e-12)
    for n in range(len(B)):
        np.testing.assert_allclose(Grad[n], gB0[n], rtol=1e-10, atol=1e-12)


def test_p2_finite_differences(oracle_mod):
    """Central differences of sum r^2/2 through the oracle's prediction."""
    w = synth.get("c4")
    T = synth.make_tensor(w)
    A, B = synth.init_params(w.init_seed, w.dims, w.J, w.R, 0.5)
    A = [a.astype(np.float64) for a in A]
    B = [b.astype(np.float64) for b in B]
    idx, vals = T.train_idx, T.train_val.astype(np.float64)

    def f():
        return 0.5 * np.sum((oracle_mod.predict(A, B, idx) - vals) ** 2)

    _, G, _ = oracle_mod.factor_minibatch([a.copy() for a in A], B, idx, vals,
                                          0.0, 0.0, False, apply=False,
                                          want_grad=True)
    _, Grad = oracle_mod.core_grad(A, B, idx, vals)
    for mats, grads in ((A, G), (B, Grad)):
        for n in range(len(mats)):
            fd = np.zeros_like(mats[n])
            it = np.nditer(mats[n], flags=["multi_index"])
            for _ in it:
                k = it.multi_index
                w0 = mats[n][k]
                h = 1e-6 * max(1.0, abs(w0))
                mats[n][k] = w0 + h
                fp = f()
                mats[n][k] = w0 - h
                fm = f()
                mats[n][k] = w0
                fd[k] = (fp - fm) / (2 * h)
            err = np.linalg.norm(fd - grads[n]) / np.linalg.norm(grads[n])
            assert err < 1e-6, (n, err)


# ---------------------------------------------------------------- P3 -------
def test_p3_zero_learning_rate(oracle_mod):
    A, B, idx, vals = rand_problem((9, 8, 7), (3, 2, 4), 3, 200, 7)
    A0 = [a.copy() for a in A]
    B0 = [b.copy() for b in B]
    l0 = oracle_mod.loss(A, B, idx, vals, 1e-3, 1e-3)
    perm = np.random.default_rng(0).permutation(200)
    oracle_mod.factor_epoch(A, B, idx, vals, perm, 16, 0.0, 1e-3, False)
    oracle_mod.core_epoch(A, B, idx, vals, 0.0, 1e-3)
    for a, a0 in zip(A, A0):
        np.testing.assert_array_equal(a, a0)
    for b, b0 in zip(B, B0):
        np.testing.assert_array_equal(b, b0)
    assert oracle_mod.loss(A, B, idx, vals, 1e-3, 1e-3) == l0


# ---------------------------------------------------------------- P4 -------
@pytest.mark.parametrize("row_mean", [False, True])
def test_p4_residual_free_decay(oracle_mod, row_mean):
    A, B, idx, _ = rand_problem((9, 8, 7), (3, 2, 4), 3, 120, 8)
    vals = oracle_mod.predict(A, B, idx)     # r = 0 exactly
    lr, lam = 0.05, 0.2
    A1 = [a.copy() for a in A]
    oracle_mod.factor_minibatch(A1, B, idx, vals, lr, lam, row_mean)
    for n in range(3):
        k = np.bincount(idx[n], minlength=A[n].shape[0])[:, None]
        factor = 1 - lr * lam * (np.minimum(k, 1) if row_mean else k)
        np.testing.assert_allclose(A1[n], A[n] * factor, rtol=1e-13,
                                   atol=1e-15)
    B1 = [b.copy() for b in B]
    oracle_mod.core_epoch(A, B1, idx, vals, lr, lam)
    for n in range(3):
        np.testing.assert_allclose(B1[n], B[n] * (1 - lr * lam), rtol=1e-13)


# ---------------------------------------------------------------- P5 -------
def test_p5_minibatch_of_one_is_sequential_sgd(oracle_mod):
    A, B, idx, vals = rand_problem((5, 6, 4), (2, 3, 2), 3, 25, 9)
    lr, lam = 0.05, 0.01
    perm = np.random.default_rng(1).permutation(25)
    As = [a.copy() for a in A]
    Am = [a.copy() for a in A]
    oracle_mod.factor_epoch(As, B, idx, vals, perm, 1, lr, lam, False)
    oracle_mod.factor_epoch(Am, B, idx, vals, perm, 1, lr, lam, True)
    # sequential per-sample SGD with autograd gradients of r^2/2 + lam/2|a|^2
    Ar = [a.copy() for a in A]
    for s in perm:
        gA, _, _ = torch_minibatch_grads(Ar, B, idx[:, s:s + 1],
                                         vals[s:s + 1], lam)
        for n in range(3):
            Ar[n] -= lr * gA[n]
    for n in range(3):
        np.testing.assert_array_equal(As[n], Am[n])
        np.testing.assert_allclose(As[n], Ar[n], rtol=1e-11, atol=1e-13)


def test_p5_jacobi_minibatch_matches_autograd_step(oracle_mod):
    """A minibatch step uses parameters as they stand at its start
    (Jacobi), summing duplicate-row contributions."""
    A, B, idx, vals = rand_problem((4, 3, 5), (3, 2, 2), 4, 40, 10)
    lr, lam = 0.02, 0.05
    gA, _, _ = torch_minibatch_grads(A, B, idx, vals, lam)
    A1 = [a.copy() for a in A]
    oracle_mod.factor_minibatch(A1, B, idx, vals, lr, lam, row_mean=False)
    A2 = [a.copy() for a in A]
    oracle_mod.factor_minibatch(A2, B, idx, vals, lr, lam, row_mean=True)
    for n in range(3):
        np.testing.assert_allclose(A1[n], A[n] - lr * gA[n], rtol=1e-11,
                                   atol=1e-13)
        k = np.maximum(np.bincount(idx[n], minlength=A[n].shape[0]), 1)
        np.testing.assert_allclose(A2[n], A[n] - lr * gA[n] / k[:, None],
                                   rtol=1e-11, atol=1e-13)


# ---------------------------------------------------------------- P6 -------
def test_p6_matrix_factorisation_special_case(oracle_mod):
    """N=2, J=R, B1=B2=I: xhat = a1.a2 and the factor step is the textbook
    matrix-factorisation SGD step."""
    rng = np.random.default_rng(3)
    a1 = rng.normal(size=(1, 4))
    a2 = rng.normal(size=(1, 4))
    x = 0.7
    lr, lam = 0.1, 0.05
    A = [a1.copy(), a2.copy()]
    B = [np.eye(4), np.eye(4)]
    idx = np.zeros((2, 1), dtype=np.int32)
    l = oracle_mod.factor_minibatch(A, B, idx, np.array([x]), lr, lam, False)
    e = float((a1 @ a2.T)[0, 0]) - x
    assert l == pytest.approx(0.5 * e * e, rel=1e-14)
    np.testing.assert_allclose(A[0], a1 - lr * (e * a2 + lam * a1), rtol=1e-14)
    np.testing.assert_allclose(A[1], a2 - lr * (e * a1 + lam * a2), rtol=1e-14)
    _, Grad = oracle_mod.core_grad([a1, a2], B, idx, np.array([x]))
    np.testing.assert_allclose(Grad[0], e * np.outer(a1, a2), rtol=1e-14)
    np.testing.assert_allclose(Grad[1], e * np.outer(a2, a1), rtol=1e-14)


# ---------------------------------------------------------------- P7 -------
def test_p7_gauge_invariance(oracle_mod):
    A, B, idx, _ = rand_problem((6, 5, 7), (3, 3, 3), 4, 50, 11)
    ref = oracle_mod.predict(A, B, idx)
    rng = np.random.default_rng(4)
    T = [rng.normal(size=(3, 3)) + 3 * np.eye(3) for _ in range(3)]
    A2 = [np.ascontiguousarray(A[n] @ T[n]) for n in range(3)]
    B2 = [np.ascontiguousarray(np.linalg.solve(T[n], B[n])) for n in range(3)]
    np.testing.assert_allclose(oracle_mod.predict(A2, B2, idx), ref,
                               rtol=1e-9, atol=1e-11)
    s0 = rng.uniform(0.5, 2.0, size=4)
    s1 = rng.uniform(0.5, 2.0, size=4)
    S = [s0, s1, 1.0 / (s0 * s1)]
    B3 = [np.ascontiguousarray(B[n] * S[n][None, :]) for n in range(3)]
    np.testing.assert_allclose(oracle_mod.predict(A, B3, idx), ref,
                               rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------- P8 -------
def test_p8_core_epoch_order_invariance(oracle_mod):
    A, B, idx, vals = rand_problem((8, 9, 7), (3, 2, 4), 3, 300, 12)
    perm = np.random.default_rng(5).permutation(300)
    B1 = [b.copy() for b in B]
    B2 = [b.copy() for b in B]
    l1 = oracle_mod.core_epoch(A, B1, idx, vals, 0.1, 0.01)
    l2 = oracle_mod.core_epoch(A, B2, np.ascontiguousarray(idx[:, perm]),
                               vals[perm], 0.1, 0.01)
    assert l1 == pytest.approx(l2, rel=1e-12)
    for n in range(3):
        np.testing.assert_allclose(B1[n], B2[n], rtol=1e-12, atol=1e-14)
    # the per-minibatch variant with one minibatch is Algorithm 5's step
    B3 = [b.copy() for b in B]
    oracle_mod.core_epoch(A, B3, idx, vals, 0.1, 0.01, perm=perm, M=300,
                          per_minibatch=True)
    for n in range(3):
        np.testing.assert_allclose(B3[n], B1[n], rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- P9 -------
def test_p9_zero_padding_invariance(oracle_mod):
    dims, J, R = (7, 6, 5), (3, 2, 3), 3
    A, B, idx, vals = rand_problem(dims, J, R, 90, 13)
    Jp, Rp = (4, 4, 5), 6
    Ap = [np.zeros((dims[n], Jp[n])) for n in range(3)]
    Bp = [np.zeros((Jp[n], Rp)) for n in range(3)]
    for n in range(3):
        Ap[n][:, :J[n]] = A[n]
        Bp[n][:J[n], :R] = B[n]
    np.testing.assert_allclose(oracle_mod.predict(Ap, Bp, idx),
                               oracle_mod.predict(A, B, idx), rtol=1e-13,
                               atol=1e-14)
    lr, lam = 0.05, 0.01
    perm = np.random.default_rng(6).permutation(90)
    oracle_mod.factor_epoch(A, B, idx, vals, perm, 16, lr, lam, True)
    oracle_mod.factor_epoch(Ap, Bp, idx, vals, perm, 16, lr, lam, True)
    oracle_mod.core_epoch(A, B, idx, vals, lr, lam)
    oracle_mod.core_epoch(Ap, Bp, idx, vals, lr, lam)
    for n in range(3):
        np.testing.assert_allclose(Ap[n][:, :J[n]], A[n], rtol=1e-12,
                                   atol=1e-14)
        assert not Ap[n][:, J[n]:].any()
        np.testing.assert_allclose(Bp[n][:J[n], :R], B[n], rtol=1e-12,
                                   atol=1e-14)
        assert not Bp[n][J[n]:, :].any() and not Bp[n][:, R:].any()


# --------------------------------------------------------------- P10 -------
def test_p10_planted_recovery(oracle_mod):
    """A planted J=R=3 FastTucker tensor plus N(0, 0.01^2) noise (c0's recipe
    at 38% density, 25^3 with 6,000 nonzeros, where completion from a random
    start is well posed) is recovered by alternating factor and core epochs
    to the noise level on held-out entries."""
    w = synth.get("c0", dims=(25, 25, 25), nnz=6000, J=3, R=3,
                  planted_rank=3, M=64)
    T = synth.make_tensor(w)
    A, B = synth.init_params(w.init_seed, w.dims, w.J, w.R, 0.5, 0.5)
    A = [a.astype(np.float64) for a in A]
    B = [b.astype(np.float64) for b in B]
    tv = T.train_val.astype(np.float64)
    sv = T.test_val.astype(np.float64)
    sse0, _ = oracle_mod.residual_stats(A, B, T.test_idx, sv)
    for ep in range(400):
        perm = synth.epoch_perm(w.order_seed, ep, T.train_idx.shape[1])
        oracle_mod.factor_epoch(A, B, T.train_idx, tv, perm, w.M, 0.05,
                                1e-5, False)
        oracle_mod.core_epoch(A, B, T.train_idx, tv, 0.5, 1e-5)
    sse, _ = oracle_mod.residual_stats(A, B, T.test_idx, sv)
    rmse0 = np.sqrt(sse0 / len(sv))
    rmse = np.sqrt(sse / len(sv))
    assert rmse < 2 * w.noise_std < 0.5 * rmse0, (rmse0, rmse)


# ------------------------------------------------ loss / RMSE definitions --
def test_loss_and_residual_stats_definitions(oracle_mod):
    """Eq. (4) (regularisers summed over modes) and the RMSE/MAE sums of
    Section 5.2, against the brute-force dense-Tucker predictions."""
    A, B, idx, vals = rand_problem((6, 5, 4), (3, 2, 4), 3, 70, 21)
    xh = dense_tucker_predict(A, B, idx)
    sse, sae = oracle_mod.residual_stats(A, B, idx, vals)
    assert sse == pytest.approx(np.sum((vals - xh) ** 2), rel=1e-12)
    assert sae == pytest.approx(np.sum(np.abs(vals - xh)), rel=1e-12)
    lamA, lamB = 0.3, 0.7
    ref = (np.sum((vals - xh) ** 2) + lamA * sum((a * a).sum() for a in A)
           + lamB * sum((b * b).sum() for b in B))
    assert oracle_mod.loss(A, B, idx, vals, lamA, lamB) == pytest.approx(
        ref, rel=1e-12)


def test_core_epoch_step_matches_autograd(oracle_mod):
    """Algorithm 5: B <- B - lr (Grad / |Omega| + lambda B), with Grad the
    autograd gradient of sum r^2/2 over the set (all modes at once)."""
    A, B, idx, vals = rand_problem((7, 6, 5), (3, 2, 4), 3, 90, 31)
    lr, lam = 0.3, 0.05
    _, gB, _ = torch_minibatch_grads(A, B, idx, vals, 0.0)
    B1 = [b.copy() for b in B]
    oracle_mod.core_epoch(A, B1, idx, vals, lr, lam)
    for n in range(3):
        np.testing.assert_allclose(B1[n], B[n] - lr * (gB[n] / 90 + lam * B[n]),
                                   rtol=1e-11, atol=1e-13)


# ----------------------------- minibatch split of an epoch (Algorithm 3) ----
def _slices(nnz, M):
    return [(f, min(f + M, nnz)) for f in range(0, nnz, M)]


@pytest.mark.parametrize("row_mean", [False, True])
def test_factor_epoch_splits_into_minibatches_with_tail(oracle_mod, row_mean):
    """Algorithm 3's factor loop over one permutation pass: consecutive
    slices of M samples of the order, the last one shorter (25 samples,
    M = 7: slices 7, 7, 7, 4), each a Jacobi step from the parameters left
    by the previous slice. Reference: per-slice gradients from torch
    autograd through the dense-Tucker graph (Eq. (12) summed per row, or
    divided by the row's occurrence count in the slice)."""
    dims, J, R = (5, 4, 6), (3, 2, 4), 3
    A, B, idx, vals = rand_problem(dims, J, R, 25, 41)
    lr, lam, M = 0.04, 0.02, 7
    perm = np.random.default_rng(7).permutation(25)
    Ao = [a.copy() for a in A]
    mb = oracle_mod.factor_epoch(Ao, B, idx, vals, perm, M, lr, lam, row_mean)
    assert mb.shape == (4,)
    Ar = [a.copy() for a in A]
    ref_losses = []
    for f, e in _slices(25, M):
        sel = perm[f:e]
        sidx = np.ascontiguousarray(idx[:, sel])
        gA, _, l = torch_minibatch_grads(Ar, B, sidx, vals[sel], lam)
        ref_losses.append(l)
        for n in range(3):
            k = np.bincount(sidx[n], minlength=dims[n])[:, None]
            step = gA[n] / np.maximum(k, 1) if row_mean else gA[n]
            Ar[n] = Ar[n] - lr * step
    np.testing.assert_allclose(mb, ref_losses, rtol=1e-11)
    for n in range(3):
        np.testing.assert_allclose(Ao[n], Ar[n], rtol=1e-11, atol=1e-13)


def test_core_epoch_per_minibatch_steps_with_tail(oracle_mod):
    """The per-minibatch core step (Algorithm 3's second loop with the
    minibatch mean of Eq. (5)) over four slices of the order (7, 7, 7, 4):
    B <- B - lr_B (Grad_slice / |slice| + lambda_B B) after every slice,
    with Grad_slice the autograd gradient of sum r^2/2 over the slice at
    the current B and A held fixed. The returned loss sums each slice's
    loss at the B in force when it was visited."""
    dims, J, R = (6, 5, 4), (3, 2, 4), 3
    A, B, idx, vals = rand_problem(dims, J, R, 25, 43)
    lr, lam, M = 0.3, 0.05, 7
    perm = np.random.default_rng(8).permutation(25)
    Bo = [b.copy() for b in B]
    lo = oracle_mod.core_epoch(A, Bo, idx, vals, lr, lam, perm=perm, M=M,
                               per_minibatch=True)
    Br = [b.copy() for b in B]
    lref = 0.0
    for f, e in _slices(25, M):
        sel = perm[f:e]
        _, gB, l = torch_minibatch_grads(A, Br, np.ascontiguousarray(
            idx[:, sel]), vals[sel], 0.0)
        lref += l
        Br = [Br[n] - lr * (gB[n] / (e - f) + lam * Br[n]) for n in range(3)]
    assert lo == pytest.approx(lref, rel=1e-11)
    for n in range(3):
        np.testing.assert_allclose(Bo[n], Br[n], rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("dims,J,R", [((9, 8, 7), (3, 4, 2), 5),
                                      ((5, 4, 6, 3, 4, 5, 3), (2, 3, 2, 4, 2,
                                                               3, 2), 3)])
def test_parallel_forms_equal_the_serial_oracle(oracle_mod, dims, J, R):
    """The all-core forms (timing only) give the serial loops' results: the
    factor epoch bit for bit, the chunked core and residual sums to rounding
    of the addition order."""
    nnz = 9000
    A, B, idx, vals = rand_problem(dims, J, R, nnz, 17)
    perm = np.random.default_rng(3).permutation(nnz)
    for threads in (1, 4):
        oracle_mod.set_threads(threads)
        for row_mean in (False, True):
            A1 = [a.copy() for a in A]
            A2 = [a.copy() for a in A]
            l1 = oracle_mod.factor_epoch(A1, B, idx, vals, perm, 700, 0.05,
                                         0.01, row_mean)
            l2 = oracle_mod.factor_epoch(A2, B, idx, vals, perm, 700, 0.05,
                                         0.01, row_mean, parallel=True)
            np.testing.assert_array_equal(l1, l2)
            for a1, a2 in zip(A1, A2):
                np.testing.assert_array_equal(a1, a2)
        l1, G1 = oracle_mod.core_grad(A, B, idx, vals)
        l2, G2 = oracle_mod.core_grad(A, B, idx, vals, parallel=True)
        assert l2 == pytest.approx(l1, rel=1e-13)
        for g1, g2 in zip(G1, G2):
            np.testing.assert_allclose(g2, g1, rtol=1e-12,
                                       atol=1e-13 * np.abs(g1).max())
        s1 = oracle_mod.residual_stats(A, B, idx, vals)
        s2 = oracle_mod.residual_stats(A, B, idx, vals, parallel=True)
        np.testing.assert_allclose(s2, s1, rtol=1e-13)
        B1 = [b.copy() for b in B]
        B2 = [b.copy() for b in B]
        oracle_mod.core_epoch(A, B1, idx, vals, 0.3, 0.01)
        oracle_mod.core_epoch(A, B2, idx, vals, 0.3, 0.01, parallel=True)
        for b1, b2 in zip(B1, B2):
            np.testing.assert_allclose(b2, b1, rtol=1e-12, atol=1e-14)
    oracle_mod.set_threads(0)
