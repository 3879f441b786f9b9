"""Python face of libcountgauss.so: torch tensors in, torch tensors out.

torch supplies device memory (inputs, outputs, workspace) and the current
stream; every step of the transform runs in the library's HIP kernels.
Nothing here computes any part of T.X.
"""
import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

_PREC = {"native": L.CG_PREC_NATIVE, "fp32": L.CG_PREC_NATIVE, "fp64": L.CG_PREC_NATIVE,
         "bf16": L.CG_PREC_BF16, "fp8": L.CG_PREC_FP8}
_ALGO = {"auto": L.CG_SX_AUTO, "atomic": L.CG_SX_ATOMIC, "sorted": L.CG_SX_SORTED,
         "binned": L.CG_SX_BINNED, "rows": L.CG_SX_ROWS, "fused": L.CG_SX_FUSED}


@dataclass
class CsrMatrix:
    """CSR matrix on the GPU: row_ptr int32[n+1], col_idx int32[nnz],
    vals float32/float64[nnz]."""
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    vals: torch.Tensor
    n: int
    d: int

    @property
    def nnz(self):
        return int(self.col_idx.numel())

    @classmethod
    def from_torch(cls, t):
        """From a torch.sparse_csr tensor (indices converted to int32)."""
        return cls(t.crow_indices().to(torch.int32).contiguous(),
                   t.col_indices().to(torch.int32).contiguous(),
                   t.values().contiguous(), int(t.shape[0]), int(t.shape[1]))


def _dtype_code(t):
    if t.dtype == torch.float32:
        return L.CG_DTYPE_F32
    if t.dtype == torch.float64:
        return L.CG_DTYPE_F64
    raise TypeError(f"unsupported dtype {t.dtype}; use float32 or float64")


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require_cuda(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("CountGauss runs on the GPU only: tensors must be on a CUDA/HIP device")


def _workspace(nbytes, device):
    """Device scratch of at least nbytes, 256-byte aligned (the buffer is
    returned too, to keep it alive until the call's work is queued)."""
    if nbytes == 0:
        return None, None, 0
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    addr = buf.data_ptr()
    pad = (-addr) % 256
    return buf, addr + pad, nbytes


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _as_csr(X):
    if isinstance(X, CsrMatrix):
        return X
    if isinstance(X, torch.Tensor) and X.layout == torch.sparse_csr:
        return CsrMatrix.from_torch(X)
    return None


def sketch(X, m, B, seed, precision="native", algo="auto", row_offset=0, kc=0, sx_out=None):
    """Y = T X = G (S X) (m x d) for dense X (n x d, unit column stride) or
    CSR X (CsrMatrix or torch.sparse_csr).  precision: native (FP32/FP64),
    bf16 or fp8 inputs to the G (S X) contraction.  algo: auto, atomic,
    sorted (bitwise reproducible), binned S X, rows (FP32 CSR, native
    precision: no S X, Y summed over the nonempty rows) or fused (FP32 CSR,
    native precision: each bucket range's S X summed in LDS and contracted
    at once, never written).  sx_out: optional B x d tensor that receives
    S X (not with rows or fused)."""
    lib = L.load()
    prec = _PREC[precision]
    sx_algo = _ALGO[algo]
    csr = _as_csr(X)
    if csr is not None:
        vals = csr.vals
        _require_cuda(csr.row_ptr, csr.col_idx, vals)
        if csr.row_ptr.dtype != torch.int32 or csr.col_idx.dtype != torch.int32:
            raise TypeError("CSR indices must be int32")
        if csr.row_ptr.numel() != csr.n + 1:
            raise ValueError("row_ptr must have n + 1 entries")
        if vals.numel() != csr.col_idx.numel():
            raise ValueError("vals and col_idx differ in length")
        device, dt, n, d = vals.device, vals.dtype, csr.n, csr.d
    else:
        if not isinstance(X, torch.Tensor) or X.dim() != 2:
            raise TypeError("X must be a 2-D dense tensor or a CSR matrix")
        _require_cuda(X)
        if X.stride(1) != 1:
            X = X.contiguous()
        device, dt, (n, d) = X.device, X.dtype, X.shape
    code = _dtype_code(torch.empty(0, dtype=dt))
    Y = torch.empty((m, d), dtype=dt, device=device)
    if sx_out is not None:
        if sx_out.shape != (B, d) or sx_out.dtype != dt or not sx_out.is_contiguous():
            raise ValueError("sx_out must be a contiguous B x d tensor of X's dtype")
    opts = L.make_opts(prec, sx_algo, kc, _stream(device), None, 0, row_offset,
                       _ptr(sx_out) if sx_out is not None else None)
    nbytes = ctypes.c_size_t(0)
    kind = L.CG_KIND_CSR if csr is not None else L.CG_KIND_DENSE
    nnz = csr.nnz if csr is not None else 0
    L.check(lib.cg_workspace_bytes(kind, code, n, d, m, B, nnz, ctypes.byref(opts),
                                   ctypes.byref(nbytes)), "cg_workspace_bytes")
    buf, addr, size = _workspace(nbytes.value, device)
    opts.workspace, opts.workspace_bytes = addr, size
    if csr is not None:
        st = lib.cg_sketch_csr(_ptr(csr.row_ptr), _ptr(csr.col_idx), _ptr(csr.vals), code, n, d,
                               nnz, m, B, ctypes.c_uint64(seed & (2 ** 64 - 1)), _ptr(Y),
                               ctypes.byref(opts))
        L.check(st, "cg_sketch_csr")
    else:
        st = lib.cg_sketch_dense(_ptr(X), X.stride(0), code, n, d, m, B,
                                 ctypes.c_uint64(seed & (2 ** 64 - 1)), _ptr(Y), ctypes.byref(opts))
        L.check(st, "cg_sketch_dense")
    del buf
    return Y


def gaussian(X, m, seed, row_offset=0, kc=0):
    """Y~ = G~ X (m x d) with G~ an m x n Gaussian generated in registers:
    the dense Gaussian projection that T X stands in for.  Dense X (FP32 or
    FP64) or CSR X (FP32)."""
    lib = L.load()
    csr = _as_csr(X)
    if csr is not None:
        _require_cuda(csr.row_ptr, csr.col_idx, csr.vals)
        device, dt, n, d = csr.vals.device, csr.vals.dtype, csr.n, csr.d
        kind, nnz = L.CG_KIND_GAUSSIAN_CSR, csr.nnz
    else:
        if not isinstance(X, torch.Tensor) or X.dim() != 2:
            raise TypeError("X must be a 2-D dense tensor or a CSR matrix")
        _require_cuda(X)
        if X.stride(1) != 1:
            X = X.contiguous()
        device, dt, (n, d) = X.device, X.dtype, X.shape
        kind, nnz = L.CG_KIND_GAUSSIAN_DENSE, 0
    code = _dtype_code(torch.empty(0, dtype=dt))
    Y = torch.empty((m, d), dtype=dt, device=device)
    opts = L.make_opts(L.CG_PREC_NATIVE, L.CG_SX_AUTO, kc, _stream(device), None, 0, row_offset)
    nbytes = ctypes.c_size_t(0)
    L.check(lib.cg_workspace_bytes(kind, code, n, d, m, 1, nnz, ctypes.byref(opts),
                                   ctypes.byref(nbytes)), "cg_workspace_bytes")
    buf, addr, size = _workspace(nbytes.value, device)
    opts.workspace, opts.workspace_bytes = addr, size
    sd = ctypes.c_uint64(seed & (2 ** 64 - 1))
    if csr is not None:
        L.check(lib.cg_gaussian_csr(_ptr(csr.row_ptr), _ptr(csr.col_idx), _ptr(csr.vals), code, n, d,
                                    nnz, m, sd, _ptr(Y), ctypes.byref(opts)), "cg_gaussian_csr")
    else:
        L.check(lib.cg_gaussian_dense(_ptr(X), X.stride(0), code, n, d, m, sd, _ptr(Y),
                                      ctypes.byref(opts)), "cg_gaussian_dense")
    del buf
    return Y


def row_extrema(Z):
    """Step 3 of Algorithm 1: for every row of Z (m x d), the lowest column
    of its largest and of its smallest value (int32 tensors imax, imin; NaNs
    never win, -1 for a row of NaNs)."""
    lib = L.load()
    _require_cuda(Z)
    if Z.dim() != 2:
        raise TypeError("Z must be 2-D")
    if Z.stride(1) != 1:
        Z = Z.contiguous()
    m, d = Z.shape
    imax = torch.empty(m, dtype=torch.int32, device=Z.device)
    imin = torch.empty(m, dtype=torch.int32, device=Z.device)
    L.check(lib.cg_row_extrema(_ptr(Z), _dtype_code(Z), m, d, Z.stride(0), _ptr(imax), _ptr(imin),
                               _stream(Z.device)), "cg_row_extrema")
    return imax, imin


def anchors(X, m, B, seed, projection="countgauss"):
    """Algorithm 1 (CountGauss NMF) on dense X (features x points): the row
    extrema (imax, imin) of Z = T X, or of Z = G~ X with
    projection="gaussian" (the Gaussian baseline; B unused)."""
    lib = L.load()
    _require_cuda(X)
    if X.dim() != 2:
        raise TypeError("X must be 2-D")
    if X.stride(1) != 1:
        X = X.contiguous()
    n, d = X.shape
    proj = {"countgauss": L.CG_PROJ_COUNTGAUSS, "gaussian": L.CG_PROJ_GAUSSIAN}[projection]
    kind = L.CG_KIND_ANCHORS_COUNTGAUSS if proj == L.CG_PROJ_COUNTGAUSS else L.CG_KIND_ANCHORS_GAUSSIAN
    code = _dtype_code(X)
    imax = torch.empty(m, dtype=torch.int32, device=X.device)
    imin = torch.empty(m, dtype=torch.int32, device=X.device)
    opts = L.make_opts(L.CG_PREC_NATIVE, L.CG_SX_AUTO, 0, _stream(X.device))
    nbytes = ctypes.c_size_t(0)
    L.check(lib.cg_workspace_bytes(kind, code, n, d, m, max(B, 1), 0, ctypes.byref(opts),
                                   ctypes.byref(nbytes)), "cg_workspace_bytes")
    buf, addr, size = _workspace(nbytes.value, X.device)
    opts.workspace, opts.workspace_bytes = addr, size
    L.check(lib.cg_anchors_dense(_ptr(X), X.stride(0), code, n, d, m, max(B, 1),
                                 ctypes.c_uint64(seed & (2 ** 64 - 1)), proj, _ptr(imax), _ptr(imin),
                                 ctypes.byref(opts)), "cg_anchors_dense")
    del buf
    return imax, imin


LEMMA_STATS = ("pair_deviation", "frobenius_gap", "kl", "tv_pinsker_bound", "offdiag_pairs",
               "positive_definite")


def lemma_stats(Y, SU=None):
    """Section 7 statistics of Y = T U (or G~ U), m x d, and optionally
    S U (B x d), for U with orthonormal columns (d <= 64): a float64 tensor
    of 6 values on the device, named by LEMMA_STATS (all but the first NaN
    without S U)."""
    lib = L.load()
    _require_cuda(Y)
    Y = Y.contiguous()
    m, d = Y.shape
    B = 1
    if SU is not None:
        _require_cuda(SU)
        if SU.dtype != Y.dtype or SU.dim() != 2 or SU.shape[1] != d:
            raise ValueError("SU must be B x d with Y's dtype")
        SU = SU.contiguous()
        B = SU.shape[0]
    code = _dtype_code(Y)
    out = torch.empty(6, dtype=torch.float64, device=Y.device)
    opts = L.make_opts(L.CG_PREC_NATIVE, L.CG_SX_AUTO, 0, _stream(Y.device))
    nbytes = ctypes.c_size_t(0)
    L.check(lib.cg_workspace_bytes(L.CG_KIND_LEMMA, code, 1, d, m, B, 0, ctypes.byref(opts),
                                   ctypes.byref(nbytes)), "cg_workspace_bytes")
    buf, addr, size = _workspace(nbytes.value, Y.device)
    opts.workspace, opts.workspace_bytes = addr, size
    L.check(lib.cg_lemma_stats(_ptr(Y), _ptr(SU), code, m, B, d, _ptr(out), ctypes.byref(opts)),
            "cg_lemma_stats")
    del buf
    return out


def sketch_adjoint(dY, n, m, B, seed, row_offset=0, out=None):
    """dX = T^T dY = S^T (G^T dY) (n x d) for a dense m x d upstream dY."""
    lib = L.load()
    _require_cuda(dY)
    dY = dY.contiguous()
    mm, d = dY.shape
    if mm != m:
        raise ValueError("dY must have m rows")
    code = _dtype_code(dY)
    dX = out if out is not None else torch.empty((n, d), dtype=dY.dtype, device=dY.device)
    if dX.shape != (n, d) or dX.stride(1) != 1:
        raise ValueError("out must be n x d with unit column stride")
    opts = L.make_opts(L.CG_PREC_NATIVE, L.CG_SX_AUTO, 0, _stream(dY.device), None, 0, row_offset)
    nbytes = ctypes.c_size_t(0)
    L.check(lib.cg_workspace_bytes(L.CG_KIND_ADJOINT, code, n, d, m, B, 0, ctypes.byref(opts),
                                   ctypes.byref(nbytes)), "cg_workspace_bytes")
    buf, addr, size = _workspace(nbytes.value, dY.device)
    opts.workspace, opts.workspace_bytes = addr, size
    L.check(lib.cg_sketch_adjoint(_ptr(dY), code, n, d, m, B, ctypes.c_uint64(seed & (2 ** 64 - 1)),
                                  _ptr(dX), dX.stride(0), ctypes.byref(opts)), "cg_sketch_adjoint")
    del buf
    return dX


def sketch_adjoint_csr(X, dY, m, B, seed, row_offset=0):
    """Gradient of <dY, T X> with respect to the stored values of CSR X."""
    lib = L.load()
    csr = _as_csr(X)
    _require_cuda(dY, csr.row_ptr)
    dY = dY.contiguous()
    code = _dtype_code(dY)
    dvals = torch.empty(csr.nnz, dtype=dY.dtype, device=dY.device)
    opts = L.make_opts(L.CG_PREC_NATIVE, L.CG_SX_AUTO, 0, _stream(dY.device), None, 0, row_offset)
    nbytes = ctypes.c_size_t(0)
    L.check(lib.cg_workspace_bytes(L.CG_KIND_ADJOINT_CSR, code, csr.n, csr.d, m, B, csr.nnz,
                                   ctypes.byref(opts), ctypes.byref(nbytes)), "cg_workspace_bytes")
    buf, addr, size = _workspace(nbytes.value, dY.device)
    opts.workspace, opts.workspace_bytes = addr, size
    L.check(lib.cg_sketch_adjoint_csr(_ptr(csr.row_ptr), _ptr(csr.col_idx), csr.nnz, _ptr(dY),
                                      code, csr.n, csr.d, m, B,
                                      ctypes.c_uint64(seed & (2 ** 64 - 1)), _ptr(dvals),
                                      ctypes.byref(opts)), "cg_sketch_adjoint_csr")
    del buf
    return dvals


class CountGaussFn(torch.autograd.Function):
    """Y = T X with the adjoint T^T dY as backward (dense X).  m, B, seed
    and the options are not differentiable."""

    @staticmethod
    def forward(ctx, X, m, B, seed, row_offset=0):
        ctx.shape = X.shape
        ctx.m, ctx.B, ctx.seed, ctx.row_offset = m, B, seed, row_offset
        return sketch(X, m, B, seed, row_offset=row_offset)

    @staticmethod
    def backward(ctx, dY):
        dX = sketch_adjoint(dY, ctx.shape[0], ctx.m, ctx.B, ctx.seed, ctx.row_offset)
        return dX, None, None, None, None


class CountGaussCsrFn(torch.autograd.Function):
    """Y = T X for CSR X as a function of its stored values: backward is
    dvals[k] = sigma(r) (G^T dY)[h(r), col_idx[k]] for the entry k of row r
    (T is linear, so this is <dY, T X>'s gradient).  The sparsity pattern,
    m, B, seed and row_offset are not differentiable."""

    @staticmethod
    def forward(ctx, vals, row_ptr, col_idx, n, d, m, B, seed, row_offset=0):
        X = CsrMatrix(row_ptr, col_idx, vals, n, d)
        ctx.save_for_backward(row_ptr, col_idx)
        ctx.n, ctx.d, ctx.m, ctx.B, ctx.seed, ctx.row_offset = n, d, m, B, seed, row_offset
        return sketch(X, m, B, seed, row_offset=row_offset)

    @staticmethod
    def backward(ctx, dY):
        row_ptr, col_idx = ctx.saved_tensors
        X = CsrMatrix(row_ptr, col_idx, dY.new_empty(0), ctx.n, ctx.d)
        dvals = sketch_adjoint_csr(X, dY, ctx.m, ctx.B, ctx.seed, ctx.row_offset)
        return dvals, None, None, None, None, None, None, None, None


def countgauss(X, m, B, seed, row_offset=0):
    """Differentiable T X (autograd through CountGaussFn for dense X; for
    CSR X -- a CsrMatrix or torch.sparse_csr tensor -- through
    CountGaussCsrFn, with respect to the stored values)."""
    csr = _as_csr(X)
    if csr is not None:
        return CountGaussCsrFn.apply(csr.vals, csr.row_ptr, csr.col_idx, csr.n, csr.d, m, B, seed,
                                     row_offset)
    return CountGaussFn.apply(X, m, B, seed, row_offset)


def sketch_csr_noalloc(X, m, B, seed, row_offset=0, out=None):
    """Y = T X for CSR X through cg_sketch_csr_noalloc: the library's static
    device scratch replaces the workspace, so the call allocates nothing
    beyond Y (none at all when `out`, an m x d tensor of X's dtype, is
    given).  Calls that can overlap on one GPU race on that scratch."""
    lib = L.load()
    csr = _as_csr(X)
    if csr is None:
        raise TypeError("sketch_csr_noalloc takes a CSR matrix")
    _require_cuda(csr.row_ptr, csr.col_idx, csr.vals)
    code = _dtype_code(csr.vals)
    Y = out if out is not None else torch.empty((m, csr.d), dtype=csr.vals.dtype,
                                                device=csr.vals.device)
    if Y.shape != (m, csr.d) or Y.dtype != csr.vals.dtype or not Y.is_contiguous():
        raise ValueError("out must be a contiguous m x d tensor of X's dtype")
    opts = L.make_opts(L.CG_PREC_NATIVE, L.CG_SX_AUTO, 0, _stream(csr.vals.device), None, 0,
                       row_offset)
    L.check(lib.cg_sketch_csr_noalloc(_ptr(csr.row_ptr), _ptr(csr.col_idx), _ptr(csr.vals), code,
                                      csr.n, csr.d, csr.nnz, m, B,
                                      ctypes.c_uint64(seed & (2 ** 64 - 1)), _ptr(Y),
                                      ctypes.byref(opts)), "cg_sketch_csr_noalloc")
    return Y


# ---- test access to the random source ----------------------------------
def debug_philox(seed, ctr):
    """Philox4x32-10 of each row of ctr (int32/uint32-valued tensor k x 4)."""
    lib = L.load()
    _require_cuda(ctr)
    ctr = ctr.contiguous()
    k = ctr.shape[0]
    out = torch.empty((k, 4), dtype=torch.int32, device=ctr.device)
    L.check(lib.cg_debug_philox(ctypes.c_uint64(seed & (2 ** 64 - 1)), _ptr(ctr), k, _ptr(out),
                                _stream(ctr.device)), "cg_debug_philox")
    return out


def debug_hash(seed, B, row0, count, device="cuda"):
    lib = L.load()
    h = torch.empty(count, dtype=torch.int32, device=device)
    s = torch.empty(count, dtype=torch.int8, device=device)
    L.check(lib.cg_debug_hash(ctypes.c_uint64(seed & (2 ** 64 - 1)), B, ctypes.c_uint64(row0),
                              count, _ptr(h), _ptr(s), _stream(torch.device(device))),
            "cg_debug_hash")
    return h, s


def debug_gaussian(seed, m, b0, nb, dtype=torch.float32, device="cuda"):
    lib = L.load()
    G = torch.empty((m, nb), dtype=dtype, device=device)
    code = _dtype_code(G)
    L.check(lib.cg_debug_gaussian(ctypes.c_uint64(seed & (2 ** 64 - 1)), m, b0, nb, code, _ptr(G),
                                  _stream(torch.device(device))), "cg_debug_gaussian")
    return G


def debug_normals(seed, m, B, device="cuda"):
    """Per-thread sums of the m x B normals of G (the generator-only probe
    behind the contraction rooflines): a float tensor of CG_NORMALS_SINK."""
    lib = L.load()
    sink = torch.empty(L.CG_NORMALS_SINK, dtype=torch.float32, device=device)
    L.check(lib.cg_debug_normals(ctypes.c_uint64(seed & (2 ** 64 - 1)), m, B, _ptr(sink),
                                 _stream(torch.device(device))), "cg_debug_normals")
    return sink


class SketchPlan:
    """A forward call with every buffer allocated up front: Y, optional S X
    and the workspace.  run() only queues the library's kernels on the
    current stream (no allocation), so it can sit in a timed loop.

    stage_events: optional list of CG_STAGE_EVENTS raw hipEvent_t handles
    (ints) that the library records at its stage boundaries; a None entry
    skips its boundary."""

    def __init__(self, X, m, B, seed, precision="native", algo="auto", row_offset=0, kc=0,
                 keep_sx=False):
        self.lib = L.load()
        self.csr = _as_csr(X)
        if self.csr is not None:
            c = self.csr
            _require_cuda(c.row_ptr, c.col_idx, c.vals)
            if c.row_ptr.dtype != torch.int32 or c.col_idx.dtype != torch.int32:
                raise TypeError("CSR indices must be int32")
            self.device, dt, self.n, self.d = c.vals.device, c.vals.dtype, c.n, c.d
            self.nnz = c.nnz
        else:
            _require_cuda(X)
            if X.dim() != 2:
                raise TypeError("X must be 2-D")
            if X.stride(1) != 1:
                X = X.contiguous()
            self.device, dt, (self.n, self.d) = X.device, X.dtype, X.shape
            self.nnz = self.n * self.d
        self.X = X
        self.m, self.B, self.seed = m, B, seed & (2 ** 64 - 1)
        self.code = _dtype_code(torch.empty(0, dtype=dt))
        self.Y = torch.empty((m, self.d), dtype=dt, device=self.device)
        self.SX = torch.empty((B, self.d), dtype=dt, device=self.device) if keep_sx else None
        self._events = None
        self.opts = L.make_opts(_PREC[precision], _ALGO[algo], kc, None, None, 0, row_offset,
                                _ptr(self.SX) if keep_sx else None)
        nbytes = ctypes.c_size_t(0)
        kind = L.CG_KIND_CSR if self.csr is not None else L.CG_KIND_DENSE
        L.check(self.lib.cg_workspace_bytes(kind, self.code, self.n, self.d, m, B,
                                            self.nnz if self.csr is not None else 0,
                                            ctypes.byref(self.opts), ctypes.byref(nbytes)),
                "cg_workspace_bytes")
        self._ws, addr, size = _workspace(nbytes.value, self.device)
        self.opts.workspace, self.opts.workspace_bytes = addr, size
        self.workspace_bytes = size

    def set_stage_events(self, handles):
        if handles is None:
            self._events = None
            self.opts.stage_events = None
            return
        if len(handles) != L.CG_STAGE_EVENTS:
            raise ValueError(f"need {L.CG_STAGE_EVENTS} event handles")
        self._events = (ctypes.c_void_p * L.CG_STAGE_EVENTS)(*[h or None for h in handles])
        self.opts.stage_events = ctypes.cast(self._events, ctypes.c_void_p)

    def run(self):
        self.opts.stream = _stream(self.device)
        seed = ctypes.c_uint64(self.seed)
        if self.csr is not None:
            c = self.csr
            st = self.lib.cg_sketch_csr(_ptr(c.row_ptr), _ptr(c.col_idx), _ptr(c.vals), self.code,
                                        self.n, self.d, self.nnz, self.m, self.B, seed,
                                        _ptr(self.Y), ctypes.byref(self.opts))
            L.check(st, "cg_sketch_csr")
        else:
            st = self.lib.cg_sketch_dense(_ptr(self.X), self.X.stride(0), self.code, self.n,
                                          self.d, self.m, self.B, seed, _ptr(self.Y),
                                          ctypes.byref(self.opts))
            L.check(st, "cg_sketch_dense")
        return self.Y

    def capture(self):
        """A HIP graph of one run(): its kernels, recorded once on a side
        stream (no stage events, which are host-side records).  Replaying it
        (graph.replay()) recomputes Y from the current contents of X, with
        one launch for the whole forward call.  The forward path issues no
        memset or copy, so the graph holds kernel nodes only."""
        if self._events is not None:
            raise RuntimeError("stage events cannot be recorded into a graph")
        self.run()                      # warm: first-use attributes set outside capture
        torch.cuda.synchronize(self.device)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.run()
        return graph


# ---------------------------------------------------------------- batched
class BatchedSketch:
    """Many independent CSR transforms computed together (cg_sketch_batched).

    items: sequence of (X, m, B, seed) or (X, m, B, seed, row_offset) with X
    an FP32 CsrMatrix / torch.sparse_csr on the GPU.  The plan (tile shapes
    from the current tuning table, work items, workspace) is made once;
    run() queues the whole batch on the current stream and returns the list
    of Y (m x d) tensors, overwritten by each run."""

    def __init__(self, items):
        lib = L.load()
        self.count = len(items)
        if self.count < 1:
            raise ValueError("a batch needs at least one instance")
        self._table = (L.CgInstance * self.count)()
        self._inputs = []
        self.Y = []
        device = None
        for i, it in enumerate(items):
            X, m, B, seed = it[:4]
            row_offset = it[4] if len(it) > 4 else 0
            csr = _as_csr(X)
            if csr is None:
                raise TypeError(f"instance {i}: X must be a CSR matrix")
            _require_cuda(csr.row_ptr, csr.col_idx, csr.vals)
            if csr.vals.dtype != torch.float32:
                raise TypeError(f"instance {i}: batched instances are FP32")
            if csr.row_ptr.dtype != torch.int32 or csr.col_idx.dtype != torch.int32:
                raise TypeError(f"instance {i}: CSR indices must be int32")
            if device is None:
                device = csr.vals.device
            elif csr.vals.device != device:
                raise ValueError("all instances must be on one device")
            Y = torch.empty((m, csr.d), dtype=torch.float32, device=device)
            c = self._table[i]
            c.row_ptr = csr.row_ptr.data_ptr()
            c.col_idx = csr.col_idx.data_ptr() if csr.nnz else None
            c.vals = csr.vals.data_ptr() if csr.nnz else None
            c.Y = Y.data_ptr()
            c.n, c.d, c.nnz, c.m, c.B = csr.n, csr.d, csr.nnz, m, B
            c.seed = seed & (2 ** 64 - 1)
            c.row_offset = row_offset
            self._inputs.append(csr)
            self.Y.append(Y)
        self.device = device
        nbytes = ctypes.c_size_t(0)
        L.check(lib.cg_batched_plan(self._table, self.count, None, ctypes.byref(nbytes)),
                "cg_batched_plan")
        self._buf, self._ws, self.workspace_bytes = _workspace(nbytes.value, device)

    def plan_fields(self, i):
        """The planned fields of instance i (tile rows, tiles, ranges, kc, ...)."""
        c = self._table[i]
        return {k: getattr(c, k) for k in ("ws_off", "tile_rows", "tiles", "ranges", "bp_shift",
                                           "kc", "parts", "gsx_items", "red_items", "route")}

    def run(self):
        lib = L.load()
        opts = L.make_opts(stream=_stream(self.device), workspace=self._ws,
                           workspace_bytes=self.workspace_bytes)
        L.check(lib.cg_sketch_batched(self._table, self.count, ctypes.byref(opts)),
                "cg_sketch_batched")
        return self.Y


def sketch_batched(items):
    """Y_i = T_i X_i for every (X, m, B, seed[, row_offset]) in items, as one
    batch.  Each returned Y keeps the batch's host table and workspace
    alive, so they outlive the queued work."""
    plan = BatchedSketch(items)
    Ys = plan.run()
    for Y in Ys:
        Y._cg_batch = plan
    return Ys


def set_tuning(rows_per_item=None, kc_per_item=None):
    """Set the batched planner's tuning table (one entry per d class
    ceil(log2 d) = 0 .. 10; shorter lists set the first classes).  Both None
    restores the built-in table."""
    lib = L.load()
    if rows_per_item is None and kc_per_item is None:
        L.check(lib.cg_set_tuning(None, None, 0), "cg_set_tuning")
        return
    k = len(rows_per_item if rows_per_item is not None else kc_per_item)
    arr = lambda v: (ctypes.c_int32 * k)(*v) if v is not None else None  # noqa: E731
    L.check(lib.cg_set_tuning(arr(rows_per_item), arr(kc_per_item), k), "cg_set_tuning")


def get_tuning():
    """(rows_per_item, kc_per_item) lists of the current tuning table."""
    lib = L.load()
    k = L.CG_TUNING_CLASSES
    rows, kc = (ctypes.c_int32 * k)(), (ctypes.c_int32 * k)()
    L.check(lib.cg_get_tuning(rows, kc, k), "cg_get_tuning")
    return list(rows), list(kc)
