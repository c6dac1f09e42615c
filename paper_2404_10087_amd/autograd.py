"""torch.autograd.Function over the stateless minibatch entry points.

FastTuckerLoss computes L = sum_{s in Psi} (xhat_s - x_s)^2 / 2 for one
minibatch Psi (Eq. (3) forward; the data term of Eq. (4) with the factor 1/2
whose gradients are Eqs. (8)/(9)). Its backward runs the library's kernels:
c^(n) is recomputed, the row gradients are summed per unique row by the
deterministic sorted reduction (sparse rows or a dense matrix) and the core
gradients are reduced in a fixed order. torch provides device memory and the
stream only.

Layout: A[n] is (I_n, J4) float32 with J4 = max J_n rounded up to 4 (to 8,
16 or 32 above order 5) and zero columns beyond J_n (FastTuckerModel keeps it
so); B[n] is (J_n, R) float32.
"""
import ctypes as C

import torch

from . import _lib
from . import FtError


def _check(status):
    if status != 0:
        msg = _lib.load().ft_last_error(None)
        raise FtError(status, msg.decode() if msg else "")


def j4_of(J):
    """Row stride of A: max J_n rounded up to 4 (orders up to 5), or to 8,
    16 or 32 (orders 6..10), as the library pads it."""
    j4 = (max(J) + 3) // 4 * 4
    if len(J) <= 5:
        return j4
    return 8 if j4 <= 8 else 16 if j4 <= 16 else 32


def _desc(dims, J, R):
    d = _lib.ProblemDesc()
    d.order = len(dims)
    for n, (I, j) in enumerate(zip(dims, J)):
        d.dims[n] = int(I)
        d.J[n] = int(j)
    d.R = int(R)
    return d


def _ptr_array(ptrs):
    arr = (C.c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = C.c_void_p(p)
    return arr


def _rows(idx):
    m = idx.shape[1]
    return [idx.data_ptr() + n * m * 4 for n in range(idx.shape[0])]


def _workspace(desc, m, device):
    nbytes = C.c_size_t()
    _check(_lib.load().ft_mb_workspace_size(C.byref(desc), m,
                                            C.byref(nbytes)))
    return torch.empty(nbytes.value, dtype=torch.uint8, device=device)


def _validate(idx, val, A, B, dims, J, R):
    N = len(dims)
    if idx.dtype != torch.int32 or idx.dim() != 2 or idx.shape[0] != N:
        raise ValueError("idx must be an int32 (order, m) tensor")
    if not idx.is_contiguous() or not val.is_contiguous():
        raise ValueError("idx and val must be contiguous")
    if val.dtype != torch.float32 or val.shape != (idx.shape[1],):
        raise ValueError("val must be float32 (m,)")
    J4 = j4_of(J)
    for n in range(N):
        if A[n].shape != (dims[n], J4) or A[n].dtype != torch.float32 or \
                not A[n].is_contiguous():
            raise ValueError(f"A[{n}] must be contiguous float32 "
                             f"({dims[n]}, {J4})")
        if B[n].shape != (J[n], R) or B[n].dtype != torch.float32 or \
                not B[n].is_contiguous():
            raise ValueError(f"B[{n}] must be contiguous float32 ({J[n]}, {R})")


class FastTuckerLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, idx, val, dims, J, R, sparse, *params):
        N = len(dims)
        A, B = params[:N], params[N:]
        _validate(idx, val, A, B, dims, J, R)
        m = idx.shape[1]
        desc = _desc(dims, J, R)
        ws = _workspace(desc, m, val.device)
        loss = torch.empty((), dtype=torch.float64, device=val.device)
        stream = torch.cuda.current_stream(val.device).cuda_stream
        _check(_lib.load().ft_mb_forward(
            C.byref(desc), _ptr_array([a.data_ptr() for a in A]),
            _ptr_array([b.data_ptr() for b in B]), _ptr_array(_rows(idx)),
            C.c_void_p(val.data_ptr()), m, C.c_void_p(loss.data_ptr()),
            C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(stream)))
        ctx.save_for_backward(idx, val, *params)
        ctx.meta = (list(dims), list(J), int(R), bool(sparse))
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        idx, val, *params = ctx.saved_tensors
        dims, J, R, sparse = ctx.meta
        N = len(dims)
        A, B = params[:N], params[N:]
        m = idx.shape[1]
        dev = val.device
        J4 = j4_of(J)
        desc = _desc(dims, J, R)
        ws = _workspace(desc, m, dev)
        g = grad_loss.detach().to(torch.float32).reshape(1).contiguous()
        gB = [torch.empty((J[n], R), dtype=torch.float32, device=dev)
              for n in range(N)]
        stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        lib = _lib.load()
        common = (C.byref(desc), _ptr_array([a.data_ptr() for a in A]),
                  _ptr_array([b.data_ptr() for b in B]),
                  _ptr_array(_rows(idx)), C.c_void_p(val.data_ptr()), m,
                  C.c_void_p(g.data_ptr()))
        if sparse:
            rows = [torch.empty(m, dtype=torch.int32, device=dev)
                    for _ in range(N)]
            vals = [torch.empty((m, J4), dtype=torch.float32, device=dev)
                    for _ in range(N)]
            count = torch.empty(N, dtype=torch.int64, device=dev)
            _check(lib.ft_mb_backward(
                *common, None, _ptr_array([r.data_ptr() for r in rows]),
                _ptr_array([v.data_ptr() for v in vals]),
                C.c_void_p(count.data_ptr()),
                _ptr_array([b.data_ptr() for b in gB]),
                C.c_void_p(ws.data_ptr()), ws.numel(), stream))
            k = count.cpu().tolist()
            gA = [torch.sparse_coo_tensor(
                rows[n][:k[n]].long().unsqueeze(0), vals[n][:k[n]],
                size=(dims[n], J4), is_coalesced=True) for n in range(N)]
        else:
            gA = [torch.empty((dims[n], J4), dtype=torch.float32, device=dev)
                  for n in range(N)]
            _check(lib.ft_mb_backward(
                *common, _ptr_array([a.data_ptr() for a in gA]), None, None,
                None, _ptr_array([b.data_ptr() for b in gB]),
                C.c_void_p(ws.data_ptr()), ws.numel(), stream))
        return (None, None, None, None, None, None, *gA, *gB)


class FastTuckerModel(torch.nn.Module):
    """Factor matrices A^(n) (kept zero-padded to J4 columns) and core
    matrices B^(n) as parameters; loss(idx, val) is the minibatch loss."""

    def __init__(self, dims, J, R, A0=None, B0=None, device="cuda"):
        super().__init__()
        self.dims = [int(d) for d in dims]
        N = len(self.dims)
        self.J = [int(J)] * N if isinstance(J, int) else [int(j) for j in J]
        self.R = int(R)
        J4 = j4_of(self.J)
        self.A = torch.nn.ParameterList()
        self.B = torch.nn.ParameterList()
        for n in range(N):
            a = torch.zeros((self.dims[n], J4), dtype=torch.float32,
                            device=device)
            b = torch.zeros((self.J[n], self.R), dtype=torch.float32,
                            device=device)
            if A0 is not None:
                a[:, :self.J[n]] = torch.as_tensor(A0[n], device=device)
            if B0 is not None:
                b.copy_(torch.as_tensor(B0[n], device=device))
            self.A.append(torch.nn.Parameter(a))
            self.B.append(torch.nn.Parameter(b))

    def factors(self):
        """Unpadded views of A^(n)."""
        return [a[:, :j] for a, j in zip(self.A, self.J)]

    def loss(self, idx, val, sparse=False):
        return FastTuckerLoss.apply(idx, val, self.dims, self.J, self.R,
                                    sparse, *self.A, *self.B)
