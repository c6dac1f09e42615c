"""ft_mb_backward_noalloc (the backward with its workspace in the library's
static device scratch) against ft_mb_backward with a caller workspace: two
calls in a row on the same device, the second with a smaller minibatch, in
the dense and the sparse gradient forms. The kernels are the same, so the
outputs must agree bit for bit."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from paper_2404_10087_amd import _lib
from paper_2404_10087_amd.autograd import _desc, _ptr_array, _rows, j4_of

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _problem(m, seed):
    w = synth.get("c0", dims=(3000, 2000, 40, 7), nnz=int(m / 0.9) + 1,
                  J=12, R=20, index_dist="zipf", zipf_s=1.1, data_seed=seed)
    T = synth.make_tensor(w)
    A0, B0 = synth.init_params(seed + 1, w.dims, w.J, w.R, 0.4)
    J = [w.J] * w.order
    J4 = j4_of(J)
    A = []
    for n in range(w.order):
        a = torch.zeros((w.dims[n], J4), dtype=torch.float32, device=DEV)
        a[:, :w.J] = torch.as_tensor(A0[n], device=DEV)
        A.append(a)
    B = [torch.as_tensor(b, device=DEV).contiguous() for b in B0]
    idx = torch.as_tensor(T.train_idx, device=DEV).contiguous()
    val = torch.as_tensor(T.train_val, device=DEV).contiguous()
    return w, J, J4, A, B, idx, val


def _outputs(w, J, J4, m, sparse):
    N = w.order
    gB = [torch.full((J[n], w.R), np.nan, dtype=torch.float32, device=DEV)
          for n in range(N)]
    if sparse:
        rows = [torch.full((m,), -7, dtype=torch.int32, device=DEV)
                for _ in range(N)]
        vals = [torch.full((m, J4), np.nan, dtype=torch.float32, device=DEV)
                for _ in range(N)]
        cnt = torch.full((N,), -1, dtype=torch.int64, device=DEV)
        return gB, None, (rows, vals, cnt)
    gA = [torch.full((w.dims[n], J4), np.nan, dtype=torch.float32,
                     device=DEV) for n in range(N)]
    return gB, gA, None


def _call(noalloc, w, J, J4, A, B, idx, val, gout, sparse):
    lib = _lib.load()
    m = idx.shape[1]
    desc = _desc(w.dims, J, w.R)
    gB, gA, sp = _outputs(w, J, J4, m, sparse)
    stream = C.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    args = [C.byref(desc), _ptr_array([a.data_ptr() for a in A]),
            _ptr_array([b.data_ptr() for b in B]), _ptr_array(_rows(idx)),
            C.c_void_p(val.data_ptr()), m, C.c_void_p(gout.data_ptr())]
    if sparse:
        rows, vals, cnt = sp
        args += [None, _ptr_array([r.data_ptr() for r in rows]),
                 _ptr_array([v.data_ptr() for v in vals]),
                 C.c_void_p(cnt.data_ptr())]
    else:
        args += [_ptr_array([g.data_ptr() for g in gA]), None, None, None]
    args.append(_ptr_array([b.data_ptr() for b in gB]))
    if noalloc:
        st = lib.ft_mb_backward_noalloc(*args, stream)
    else:
        nbytes = C.c_size_t()
        assert lib.ft_mb_workspace_size(C.byref(desc), m,
                                        C.byref(nbytes)) == 0
        # stale contents, as the static scratch has after an earlier call
        ws = torch.full((nbytes.value,), 0xA5, dtype=torch.uint8, device=DEV)
        st = lib.ft_mb_backward(*args, C.c_void_p(ws.data_ptr()),
                                ws.numel(), stream)
    assert st == 0, lib.ft_last_error(None)
    torch.cuda.synchronize()
    if sparse:
        rows, vals, cnt = sp
        k = cnt.cpu().numpy()
        return ([r[:k[n]].cpu().numpy() for n, r in enumerate(rows)],
                [v[:k[n]].cpu().numpy() for n, v in enumerate(vals)],
                k, [b.cpu().numpy() for b in gB])
    return [g.cpu().numpy() for g in gA], [b.cpu().numpy() for b in gB]


def _same(x, y):
    if isinstance(x, (list, tuple)):
        assert len(x) == len(y)
        for a, b in zip(x, y):
            _same(a, b)
    else:
        np.testing.assert_array_equal(np.asarray(x), np.asarray(y))


@pytest.mark.parametrize("sparse", [False, True])
def test_noalloc_backward_matches_workspace_backward(sparse):
    gout = torch.tensor([1.75], dtype=torch.float32, device=DEV)
    # the second call is smaller than the first, so it runs on what the
    # first left in the scratch
    for m, seed in ((60000, 41), (9001, 43)):
        print(f"[noalloc] sparse={sparse} m={m} seed={seed}", flush=True)
        w, J, J4, A, B, idx, val = _problem(m, seed)
        m = idx.shape[1]
        ref = _call(False, w, J, J4, A, B, idx, val, gout, sparse)
        got = _call(True, w, J, J4, A, B, idx, val, gout, sparse)
        _same(got, ref)
        assert all(np.isfinite(b).all() for b in got[-1])


def test_noalloc_rejects_a_minibatch_beyond_the_scratch():
    lib = _lib.load()
    w, J, J4, A, B, idx, val = _problem(1000, 47)
    m = 4_000_000
    desc = _desc(w.dims, J, w.R)
    nbytes = C.c_size_t()
    assert lib.ft_mb_workspace_size(C.byref(desc), m, C.byref(nbytes)) == 0
    assert nbytes.value > _lib.NOALLOC_SCRATCH_BYTES
    gB = [torch.empty((J[n], w.R), device=DEV) for n in range(w.order)]
    fake = _ptr_array([idx.data_ptr()] * w.order)
    st = lib.ft_mb_backward_noalloc(
        C.byref(desc), _ptr_array([a.data_ptr() for a in A]),
        _ptr_array([b.data_ptr() for b in B]), fake,
        C.c_void_p(val.data_ptr()), m, None, None, None, None, None,
        _ptr_array([b.data_ptr() for b in gB]), None)
    assert st == _lib.FT_EINVAL
    assert b"static scratch" in lib.ft_last_error(None)
