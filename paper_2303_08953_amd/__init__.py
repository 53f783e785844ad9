"""Adaptive s-step GMRES on AMD MI355X (gfx950): Python binding.

A thin ctypes layer over the C ABI in include/sgm.h.  PyTorch provides
device memory and the HIP stream; every arithmetic step of the solver runs
in the library's HIP kernels.  The binding refuses to run without the
compiled library (libsgm.so next to this file) -- there is no fallback.

Method: Xu, Alonso, Darve, "A numerically stable communication avoiding
s-step GMRES algorithm" (arXiv 2303.08953), Alg. 4 with the scaled Newton
basis (Sec. 3.4) and the initial step-size estimator (Sec. 3.5).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgm.so")

# status codes
OK, NOT_CONVERGED, EINVAL, EHIP, ENOMEM, ENUMERIC = 0, 1, -1, -2, -3, -4
BASIS = {"scaled_newton": 0, "newton": 1, "monomial": 2}
PRECOND = {"none": 0, "jacobi": 1, "ilu0": 2}
PRECISION = {"fp64": 0, "fp32_ir": 1}
PREPHASE = {"cgs2": 0, "monomial": 1}
ORTH = {"bcgs2": 0, "bcgs2_pyth": 1}


class SgmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sgm status {status}: {msg}")
        self.status = status


class Opts(C.Structure):
    _fields_ = [
        ("s_max", C.c_int32), ("restart", C.c_int32),
        ("max_restarts", C.c_int32), ("tol", C.c_double),
        ("precond", C.c_int), ("basis", C.c_int), ("precision", C.c_int),
        ("omega", C.c_double), ("omega_est", C.c_double),
        ("use_estimator", C.c_int32), ("transpose", C.c_int32),
        ("inner_tol", C.c_double), ("max_outer", C.c_int32),
        ("ritz_reuse", C.c_int32),
        ("shifts_host", C.POINTER(C.c_double)), ("n_shifts", C.c_int32),
        ("prephase", C.c_int), ("prephase_s", C.c_int32),
        ("orth", C.c_int), ("mpk_depth", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("restarts", C.c_int32),
        ("outer_iters", C.c_int32), ("s0_est", C.c_int32),
        ("s_init", C.c_int32), ("n_hist", C.c_int32),
        ("n_blocks", C.c_int32), ("n_shifts", C.c_int32),
        ("gamma_guard_hits", C.c_int32),
        ("rel_res_true", C.c_double), ("rel_res_est", C.c_double),
        ("t_phase_ms", C.c_double * 8),
        ("n_spmv", C.c_int64), ("t_spmv_ms", C.c_double),
        ("mpk_depth", C.c_int32), ("mpk_slab_rows", C.c_int64),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "t_phase_ms"}
        d["t_phase_ms"] = list(self.t_phase_ms)
        return d


_lib = None

# (name, restype, argtypes) of every C ABI symbol declared in include/sgm.h
_P = C.c_void_p
_SIGS = [
    ("sgm_matrix_create", C.c_int,
     [C.c_int64, C.c_int64, _P, _P, _P, _P, C.POINTER(_P)]),
    ("sgm_matrix_update_values", C.c_int, [_P, _P, _P]),
    ("sgm_matrix_destroy", C.c_int, [_P]),
    ("sgm_matrix_info", C.c_int,
     [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
      C.POINTER(C.c_int32)]),
    ("sgm_matrix_ilu0", C.c_int, [_P, _P, C.POINTER(C.c_int32)]),
    ("sgm_ilu0_apply", C.c_int, [_P, _P, _P, _P]),
    ("sgm_ilu0_factors", C.c_int, [_P, _P, _P]),
    ("sgm_spmv", C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P]),
    ("sgm_opts_default", None, [C.POINTER(Opts)]),
    ("sgm_workspace_size", C.c_int, [_P, C.POINTER(Opts), C.POINTER(C.c_size_t)]),
    ("sgm_solve", C.c_int,
     [_P, _P, _P, _P, C.POINTER(Opts), _P, C.c_size_t, _P,
      C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32), C.c_int32,
      C.POINTER(Info)]),
    ("sgm_grad_vals", C.c_int, [_P, _P, _P, _P, _P]),
    ("sgm_mpk", C.c_int,
     [_P, C.c_int, C.c_int, _P, C.c_int64, C.c_int32, C.c_int32, _P,
      C.c_int32, _P]),
    ("sgm_mpk_norms", C.c_int,
     [_P, C.c_int, C.c_int, _P, C.c_int64, C.c_int32, C.c_int32, _P,
      C.c_int32, _P, _P, C.c_int64, _P]),
    ("sgm_mpk_fused", C.c_int,
     [_P, C.c_int, C.c_int, _P, C.c_int64, C.c_int32, C.c_int32, _P,
      C.c_int32, C.c_int32, _P, C.POINTER(C.c_int64)]),
    ("sgm_block_ws_size", C.c_size_t, [C.c_int64, C.c_int32, C.c_int32]),
    ("sgm_block_orth", C.c_int,
     [C.c_int, C.c_int64, _P, C.c_int64, C.c_int32, C.c_int32, C.c_double,
      C.c_int, _P, C.c_size_t, _P, C.POINTER(C.c_int32),
      C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("sgm_block_orth_noalloc", C.c_int,
     [C.c_int, C.c_int64, _P, C.c_int64, C.c_int32, C.c_int32, C.c_double,
      C.c_int, _P, C.POINTER(C.c_int32), C.POINTER(C.c_double),
      C.POINTER(C.c_double)]),
    ("sgm_shifts_ws_size", C.c_size_t, [C.c_int32]),
    ("sgm_shifts", C.c_int,
     [_P, C.c_int32, C.c_int32, C.c_int, C.c_double, C.c_double, _P,
      C.c_size_t, _P, C.POINTER(C.c_double), C.POINTER(C.c_double),
      C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("sgm_status_string", C.c_char_p, [C.c_int]),
    ("sgm_last_error", C.c_char_p, []),
    ("sgm_device_ok", C.c_int, []),
]
SYMBOLS = [s[0] for s in _SIGS]


def lib():
    """Load libsgm.so (built by paper_2303_08953_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2303_08953_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st < 0:
        msg = lib().sgm_last_error().decode(errors="replace")
        raise SgmError(st, msg)
    return st


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a ROCm GPU is required (torch.cuda unavailable)")
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(a, dtype, device="cuda"):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


class Matrix:
    """An analysed CSR matrix on the GPU (sgm_matrix_create)."""

    def __init__(self, n, row_ptr, col, val, stream=None):
        torch = _torch()
        self.n = int(n)
        self.row_ptr = _dev(row_ptr, torch.int32)
        self.col = _dev(col, torch.int32)
        self.val = _dev(val, torch.float64)
        self.nnz = int(self.col.numel())
        # bumped by every update_values: the autograd node compares it with
        # the version its forward solve ran on
        self.version = 0
        h = C.c_void_p()
        _check(lib().sgm_matrix_create(self.n, self.nnz, _ptr(self.row_ptr),
                                       _ptr(self.col), _ptr(self.val),
                                       _stream(stream), C.byref(h)))
        self._h = h

    @classmethod
    def from_csr(cls, A, stream=None):
        """From any object with n, row_ptr, col, val (e.g. workloads.Csr)."""
        return cls(A.n, A.row_ptr, A.col, A.val, stream)

    @property
    def handle(self):
        return self._h

    def update_values(self, val, stream=None):
        torch = _torch()
        self.val = _dev(val, torch.float64)
        _check(lib().sgm_matrix_update_values(self._h, _ptr(self.val),
                                              _stream(stream)))
        self.version += 1

    def ilu0(self, stream=None):
        """sgm_matrix_ilu0: ILU(0) factors for precond="ilu0"; returns the
        level counts of the forward and backward substitutions."""
        lv = (C.c_int32 * 2)()
        _check(lib().sgm_matrix_ilu0(self._h, _stream(stream), lv))
        self.ilu_levels = (lv[0], lv[1])
        return self.ilu_levels

    def ilu0_apply(self, r, out=None, stream=None):
        """z = M^{-1} r with the ILU(0) factors (sgm_ilu0_apply)."""
        torch = _torch()
        r = _dev(r, torch.float64)
        z = out if out is not None else torch.empty_like(r)
        _check(lib().sgm_ilu0_apply(self._h, _ptr(r), _ptr(z),
                                    _stream(stream)))
        return z

    def ilu0_factors(self, stream=None):
        """The ILU(0) factor values in the CSR order of A (sgm_ilu0_factors)."""
        torch = _torch()
        lu = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        _check(lib().sgm_ilu0_factors(self._h, _ptr(lu), _stream(stream)))
        return lu

    def info(self):
        n, nnz, snnz = C.c_int64(), C.c_int64(), C.c_int64()
        ib = (C.c_int32 * 2)()
        _check(lib().sgm_matrix_info(self._h, C.byref(n), C.byref(nnz),
                                     C.byref(snnz), ib))
        return dict(n=n.value, nnz=nnz.value, sell_nnz=snnz.value,
                    index_bytes=ib[0], index_bytes_t=ib[1])

    def spmv(self, x, transpose=False, precision="fp64", out=None,
             stream=None):
        torch = _torch()
        dt = torch.float64 if precision == "fp64" else torch.float32
        x = _dev(x, dt)
        y = out if out is not None else torch.empty_like(x)
        _check(lib().sgm_spmv(self._h, int(transpose), PRECISION[precision],
                              _ptr(x), _ptr(y), _stream(stream)))
        return y

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().sgm_matrix_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_opts(s_max=8, restart=64, max_restarts=100, tol=1e-10,
              precond="none", basis="scaled_newton", precision="fp64",
              omega=0.0, omega_est=0.0, use_estimator=True, transpose=False,
              inner_tol=1e-6, max_outer=200, ritz_reuse=True, shifts=None,
              prephase="cgs2", prephase_s=8, orth="bcgs2", mpk_depth=1):
    o = Opts()
    lib().sgm_opts_default(C.byref(o))
    o.s_max, o.restart, o.max_restarts, o.tol = s_max, restart, max_restarts, tol
    o.precond = PRECOND[precond]
    o.basis = BASIS[basis]
    o.precision = PRECISION[precision]
    o.omega, o.omega_est = omega, omega_est
    o.use_estimator = int(bool(use_estimator))
    o.transpose = int(bool(transpose))
    o.inner_tol, o.max_outer = inner_tol, max_outer
    o.ritz_reuse = int(bool(ritz_reuse))
    o.prephase = PREPHASE[prephase]
    o.prephase_s = int(prephase_s)
    o.orth = ORTH[orth]
    o.mpk_depth = int(mpk_depth)
    keep = None
    if shifts is not None:
        z = np.asarray(shifts, dtype=np.complex128).ravel()
        keep = np.ascontiguousarray(np.stack([z.real, z.imag], 1).ravel())
        o.shifts_host = keep.ctypes.data_as(C.POINTER(C.c_double))
        o.n_shifts = z.size
    return o, keep


def workspace_size(A: Matrix, **opts):
    o, _keep = make_opts(**opts)
    nb = C.c_size_t()
    _check(lib().sgm_workspace_size(A.handle, C.byref(o), C.byref(nb)))
    return nb.value


class Workspace:
    """A reusable device workspace (a torch uint8 tensor)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        return self.buf


@dataclass
class SolveResult:
    x: object
    status: int
    res_hist: np.ndarray
    s_hist: np.ndarray
    info: dict


def solve(A: Matrix, b, x0=None, out=None, workspace: Workspace | None = None,
          stream=None, hist_cap=200000, **opts) -> SolveResult:
    """sgm_solve: adaptive s-step GMRES(m) on the GPU (Alg. 4).  With
    precond="ilu0" the matrix's ILU(0) factors are built first if it has
    none (sgm_matrix_ilu0)."""
    torch = _torch()
    if opts.get("precond") == "ilu0" and getattr(A, "ilu_levels", None) is None:
        A.ilu0(stream)
    o, keep = make_opts(**opts)
    nb = C.c_size_t()
    _check(lib().sgm_workspace_size(A.handle, C.byref(o), C.byref(nb)))
    ws = (workspace or Workspace()).get(nb.value)
    b = _dev(b, torch.float64)
    x0 = _dev(x0, torch.float64) if x0 is not None else None
    x = out if out is not None else torch.empty(A.n, dtype=torch.float64,
                                                device="cuda")
    rh = np.zeros(hist_cap, dtype=np.float64)
    sh = np.zeros(hist_cap, dtype=np.int32)
    info = Info()
    st = lib().sgm_solve(
        A.handle, _ptr(b), _ptr(x0) if x0 is not None else None, _ptr(x),
        C.byref(o), _ptr(ws), C.c_size_t(ws.numel()), _stream(stream),
        rh.ctypes.data_as(C.POINTER(C.c_double)), hist_cap,
        sh.ctypes.data_as(C.POINTER(C.c_int32)), hist_cap, C.byref(info))
    _check(st)
    del keep
    d = info.as_dict()
    return SolveResult(x, st, rh[:min(info.n_hist, hist_cap)].copy(),
                       sh[:min(info.n_blocks, hist_cap)].copy(), d)


def grad_vals(A: Matrix, lam, x, out=None, stream=None):
    torch = _torch()
    g = out if out is not None else torch.empty(A.nnz, dtype=torch.float64,
                                                device="cuda")
    _check(lib().sgm_grad_vals(A.handle, _ptr(lam), _ptr(x), _ptr(g),
                               _stream(stream)))
    return g


def mpk(A: Matrix, Q, ldq, c, s, records, transpose=False, precision="fp64",
        stream=None):
    """sgm_mpk on a column-major Q given as a flat device tensor."""
    torch = _torch()
    rec = _dev(np.asarray(records, dtype=np.float64).ravel(), torch.float64)
    _check(lib().sgm_mpk(A.handle, int(transpose), PRECISION[precision],
                         _ptr(Q), int(ldq), int(c), int(s), _ptr(rec),
                         rec.numel() // 3, _stream(stream)))
    torch.cuda.current_stream().synchronize()


def mpk_norms(A: Matrix, Q, ldq, c, s, records, transpose=False,
              precision="fp64", stream=None):
    """sgm_mpk_norms: sgm_mpk with the fused square-sum epilogue.  Returns
    the float64 sums of squares of the s new columns (numpy)."""
    torch = _torch()
    rec = _dev(np.asarray(records, dtype=np.float64).ravel(), torch.float64)
    norms2 = torch.zeros(max(1, int(s)), dtype=torch.float64, device="cuda")
    work = torch.empty((A.n + 255) // 256, dtype=torch.float64,
                       device="cuda")
    _check(lib().sgm_mpk_norms(A.handle, int(transpose), PRECISION[precision],
                               _ptr(Q), int(ldq), int(c), int(s), _ptr(rec),
                               rec.numel() // 3, _ptr(norms2), _ptr(work),
                               work.numel(), _stream(stream)))
    torch.cuda.current_stream().synchronize()
    return norms2[:int(s)].cpu().numpy()


def mpk_fused(A: Matrix, Q, ldq, c, s, records, depth, transpose=False,
              precision="fp64", stream=None):
    """sgm_mpk_fused (temporal blocking, `depth` steps per pass) on a
    column-major Q given as a flat device tensor.  Returns the slab height
    in rows (0 when it ran one step per launch)."""
    torch = _torch()
    rec = _dev(np.asarray(records, dtype=np.float64).ravel(), torch.float64)
    slab = C.c_int64()
    _check(lib().sgm_mpk_fused(A.handle, int(transpose), PRECISION[precision],
                               _ptr(Q), int(ldq), int(c), int(s), _ptr(rec),
                               rec.numel() // 3, int(depth), _stream(stream),
                               C.byref(slab)))
    torch.cuda.current_stream().synchronize()
    return slab.value


def block_orth(Q, n_rows, ldq, i, s, omega=0.0, precision="fp64",
               stream=None, orth="bcgs2"):
    """sgm_block_orth on a flat column-major device tensor Q (in place).
    Returns (p, R_top (i x s), R_kk (s x s)) as numpy arrays."""
    torch = _torch()
    L = lib()
    nbytes = L.sgm_block_ws_size(int(n_rows), int(i), int(s))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    p = C.c_int32()
    Rt = np.zeros(i * s, dtype=np.float64)
    Rk = np.zeros(s * s, dtype=np.float64)
    _check(L.sgm_block_orth(PRECISION[precision], int(n_rows), _ptr(Q),
                            int(ldq), int(i), int(s), float(omega),
                            ORTH[orth], _ptr(ws),
                            C.c_size_t(nbytes), _stream(stream), C.byref(p),
                            Rt.ctypes.data_as(C.POINTER(C.c_double)),
                            Rk.ctypes.data_as(C.POINTER(C.c_double))))
    return p.value, Rt.reshape(s, i).T.copy(), Rk.reshape(s, s).T.copy()


def block_orth_noalloc(Q, n_rows, ldq, i, s, omega=0.0, precision="fp64",
                       stream=None, orth="bcgs2"):
    """sgm_block_orth_noalloc: block_orth with the library's static device
    scratch instead of a workspace (no device allocation in the call;
    s <= 64, i + s <= 256).  Returns (p, R_top (i x s), R_kk (s x s))."""
    p = C.c_int32()
    Rt = np.zeros(i * s, dtype=np.float64)
    Rk = np.zeros(s * s, dtype=np.float64)
    _check(lib().sgm_block_orth_noalloc(
        PRECISION[precision], int(n_rows), _ptr(Q), int(ldq), int(i), int(s),
        float(omega), ORTH[orth], _stream(stream), C.byref(p),
        Rt.ctypes.data_as(C.POINTER(C.c_double)),
        Rk.ctypes.data_as(C.POINTER(C.c_double))))
    return p.value, Rt.reshape(s, i).T.copy(), Rk.reshape(s, s).T.copy()


def shifts(H, m0, basis="scaled_newton", eps=2.0 ** -53, omega_est=0.0,
           stream=None):
    """sgm_shifts: Ritz values (Leja order), records and s0* of the leading
    m0 x m0 block of a Hessenberg matrix H (numpy or device, square)."""
    torch = _torch()
    Hd = _dev(np.asfortranarray(np.asarray(H, dtype=np.float64)).ravel(order="F")
              if not isinstance(H, torch.Tensor) else H, torch.float64)
    ldh = int(np.asarray(H).shape[0]) if not isinstance(H, torch.Tensor) else m0
    L = lib()
    nbytes = L.sgm_shifts_ws_size(int(m0))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    re = np.zeros(m0)
    im = np.zeros(m0)
    rec = np.zeros(3 * m0)
    s0 = C.c_int32()
    hits = C.c_int32()
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    _check(L.sgm_shifts(_ptr(Hd), ldh, int(m0), BASIS[basis], float(eps),
                        float(omega_est), _ptr(ws), C.c_size_t(nbytes),
                        _stream(stream), dp(re), dp(im), dp(rec),
                        C.byref(s0), C.byref(hits)))
    return re + 1j * im, rec.reshape(m0, 3), s0.value, hits.value


# ------------------------------------------------------------------ autograd

def _autograd_function():
    import torch

    class SStepSolve(torch.autograd.Function):
        """x = A(vals)^{-1} b with gradients w.r.t. vals and b.

        Backward solves A^T lambda = dL/dx with the same s-step kernels on
        the transposed SELL structure; grad_b = lambda and
        grad_vals[k] = -lambda[row(k)] x[col(k)] (one fused kernel).

        The forward keeps a copy of vals and the matrix version it solved
        with; if the shared Matrix was given other values since (another
        forward, update_values), backward puts these back before the
        adjoint solve and the gradient.  A solve that stops short of its
        tolerance raises SgmError unless allow_not_converged is set."""

        @staticmethod
        def forward(ctx, vals, b, A: Matrix, opts: dict, allow, trace):
            vsave = vals.detach().clone()
            A.update_values(vsave)
            r = solve(A, b.detach(), **opts)
            if r.status != OK and not allow:
                raise SgmError(r.status, "forward solve did not converge "
                               f"(relative residual {r.info['rel_res_true']:.3e})")
            if trace is not None:
                trace.append(("forward", r))
            ctx.A = A
            ctx.opts = opts
            ctx.allow = allow
            ctx.trace = trace
            ctx.version = A.version
            ctx.save_for_backward(r.x, vsave)
            return r.x

        @staticmethod
        def backward(ctx, gx):
            x, vsave = ctx.saved_tensors
            A = ctx.A
            if A.version != ctx.version:
                A.update_values(vsave)
                ctx.version = A.version
            o = dict(ctx.opts)
            o["transpose"] = not o.get("transpose", False)
            r = solve(A, gx.detach().contiguous(), **o)
            if r.status != OK and not ctx.allow:
                raise SgmError(r.status, "adjoint solve did not converge "
                               f"(relative residual {r.info['rel_res_true']:.3e})")
            if ctx.trace is not None:
                ctx.trace.append(("adjoint", r))
            lam = r.x
            gv = grad_vals(A, lam, x) if ctx.needs_input_grad[0] else None
            gb = lam if ctx.needs_input_grad[1] else None
            return gv, gb, None, None, None, None

    return SStepSolve


def sstep_solve(vals, b, A: Matrix, allow_not_converged=False, trace=None,
                **opts):
    """Differentiable solve: x = A(vals)^{-1} b (see SStepSolve).

    trace: an optional list; the forward and adjoint SolveResults are
    appended to it as ("forward", r) and ("adjoint", r)."""
    global SStepSolve
    if SStepSolve is None:
        SStepSolve = _autograd_function()
    return SStepSolve.apply(vals, b, A, opts, bool(allow_not_converged),
                            trace)


SStepSolve = None
