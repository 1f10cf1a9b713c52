"""Python binding of libsmg.so (argument marshalling only).

Every name mirrors an entry point of ``include/smg.h``.  PyTorch provides the
device memory (the workspace and every vector are torch CUDA tensors) and the
current stream; all computation runs in the library's HIP kernels.  There is
no fallback: if the shared library is missing or fails to load, this module
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmg.so")

SMG_OK, SMG_NOT_CONVERGED = 0, 1
PREC = {"f64": 0, "f32": 1, "bf16": 2}
PRECOND = {"smg": 0, "none": 1}
KERNELS = {"line_relax": 0, "restrict2": 1, "prolong2": 2, "resid3": 3, "correct3": 4, "restrict3": 5,
           "prolong3": 6, "down2": 7, "coarse2": 8, "chain2": 9, "up2": 10, "chain3": 11}


class SMGError(RuntimeError):
    pass


class smg_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("cx", C.c_double), ("cy", C.c_double), ("cz", C.c_double)]


class smg_opts(C.Structure):
    _fields_ = [("pre", C.c_int32), ("post", C.c_int32), ("inner_pre", C.c_int32),
                ("inner_post", C.c_int32), ("order", C.c_int32), ("precision", C.c_int32),
                ("kernel_mode", C.c_int32)]


class krylov_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("precond", C.c_int32),
                ("x0_zero", C.c_int32), ("stop_norm", C.c_int32),
                ("history", C.POINTER(C.c_double)), ("history_c", C.POINTER(C.c_double)),
                ("xstar", C.c_void_p), ("diag_work", C.c_void_p),
                ("err_a", C.POINTER(C.c_double)), ("sin_angle", C.POINTER(C.c_double))]


class krylov_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("solve_seconds", C.c_double), ("rel_res_c", C.c_double)]


STOP = {"2": 0, "c": 1}


class smg_tune_info(C.Structure):
    _fields_ = [("candidates", C.c_int32), ("l0", C.c_int32), ("s_down", C.c_int32), ("s_up", C.c_int32),
                ("march_waves", C.c_int32), ("reserved", C.c_int32),
                ("coarse_lds", C.c_int64), ("default_ms", C.c_double), ("best_ms", C.c_double)]


class lobpcg_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("precond", C.c_int32),
                ("guard", C.c_int32), ("reserved", C.c_int32)]


class lobpcg_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("nconv", C.c_int32), ("status", C.c_int32),
                ("reserved", C.c_int32), ("seconds", C.c_double)]


class net_solve_info(C.Structure):
    _fields_ = [("fallback_iter", C.c_int32), ("fallback_reason", C.c_int32)]


NET_PREC = {"bf16": 0, "f64": 1}
NET_LOSS = {"mse": 0, "energy": 1}
NET_NPARAMS = 14737
FALLBACK = {0: "none", 1: "sr", 2: "nonfinite", 3: "stagnation"}

_lib = None


def lib():
    """Load libsmg.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SMGError(f"{LIB_PATH} is not built; run paper_1212_6680_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        p, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.smg_workspace_bytes.argtypes = [C.POINTER(smg_grid), C.POINTER(smg_opts), i32, C.POINTER(C.c_size_t)]
        L.smg_setup.argtypes = [C.POINTER(smg_grid), C.POINTER(smg_opts), i32, p, C.c_size_t, p,
                                C.POINTER(p)]
        L.smg_apply.argtypes = [p, p, p, i32, i64, p]
        L.smg_apply_static.argtypes = [C.POINTER(smg_grid), C.POINTER(smg_opts), p, p, i32, i64, p]
        L.smg_matvec.argtypes = [p, p, p, i32, i64, p]
        for f in (L.pcg_solve, L.fpcg_solve, L.psd_solve):
            f.argtypes = [p, p, p, C.POINTER(krylov_opts), C.POINTER(krylov_info), p]
        L.smg_destroy.argtypes = [p]
        L.smg_strerror.argtypes = [C.c_int]
        L.smg_strerror.restype = C.c_char_p
        L.smg_profile_kernel.argtypes = [p, i32, p, p, i32, p, C.POINTER(i32), C.POINTER(d), C.POINTER(d)]
        L.smg_profile_levels.argtypes = [p, i32, p, p, i32, p, i32, C.POINTER(i32), p, p, p]
        if hasattr(L, "lobpcg_solve"):
            L.lobpcg_workspace_bytes.argtypes = [p, i32, C.POINTER(C.c_size_t)]
            L.lobpcg_profile_gram.argtypes = [p, i32, i32, p, C.c_size_t, i32, p, C.POINTER(d)]
            L.lobpcg_solve.argtypes = [p, i32, p, p, p, p, C.c_size_t,
                                       C.POINTER(lobpcg_opts), C.POINTER(lobpcg_info), p]
        L.smg_autotune.argtypes = [p, p, p, i32, p, C.POINTER(smg_tune_info)]
        L.smgv_workspace_bytes.argtypes = [i32, i32, i32, C.POINTER(smg_opts), i32, i32, C.POINTER(C.c_size_t)]
        L.smgv_setup.argtypes = [i32, i32, i32, p, p, p, p, i32, C.POINTER(smg_opts), i32, p, C.c_size_t, p,
                                 C.POINTER(p)]
        L.smgv_levels.argtypes = [p, C.POINTER(i32), C.POINTER(i32)]
        L.smgv_export.argtypes = [p, i32, i32, p, p]
        L.smg_delta.argtypes = [p, p, d, p, i32, p, C.POINTER(d), p]
        L.smg_delta_min.argtypes = [p, p, d, d, d, p, i32, p, C.POINTER(d), C.POINTER(d), p]
        L.smg_spectrum.argtypes = [p, p, i32, p, C.POINTER(d), C.POINTER(d), p]
        L.smg_get_schedule.argtypes = [p, C.POINTER(smg_tune_info)]
        L.smg_set_march.argtypes = [p, i32]
        L.smg_batch_workspace_bytes.argtypes = [p, i32, C.POINTER(C.c_size_t)]
        L.smg_batch_create.argtypes = [p, i32, p, p, p, C.c_size_t, i32, p, C.POINTER(p)]
        L.smg_batch_fpcg.argtypes = [p, C.POINTER(krylov_opts), p, p]
        L.smg_batch_destroy.argtypes = [p]
        L.smg_batch_stats.argtypes = [p, C.POINTER(i32), C.POINTER(i32)]
        L.net_workspace_bytes.argtypes = [i64, i32, i32, C.POINTER(C.c_size_t)]
        L.net_setup.argtypes = [i64, i32, i32, p, C.c_size_t, p, C.POINTER(p)]
        L.net_destroy.argtypes = [p]
        L.net_set_params.argtypes = [p, p, p]
        L.net_get_params.argtypes = [p, p, p]
        L.net_layer_forward.argtypes = [p, i32, i32, i32, i32, p, p, p]
        L.net_loss_grad.argtypes = [p, i32, i32, i32, p, p, i32, p, p, p]
        L.net_adam_step.argtypes = [p, d, p]
        L.net_train.argtypes = [p, i32, i32, i32, p, p, i32, i32, p, p, i32, p, p]
        L.net_correct.argtypes = [p, p, p, p, p, p, p]
        L.net_make_pairs.argtypes = [p, p, p, i32, C.c_uint64, d, i32, p, p, p, p]
        L.fpcg_learned_solve.argtypes = [p, p, p, p, C.POINTER(krylov_opts), C.POINTER(krylov_info),
                                         C.POINTER(net_solve_info), p]
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().smg_strerror(code).decode()


def _check(code: int, what: str, ok=(SMG_OK,)):
    if code not in ok:
        raise SMGError(f"{what}: {strerror(code)} ({code})")
    return code


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t: torch.Tensor, n: int | None = None):
    """Device pointer of a contiguous float64 CUDA tensor of exactly n elements (when n is given)."""
    if n is not None and t.numel() != n:
        raise SMGError(f"expected {n} elements, got a tensor of shape {tuple(t.shape)}")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise SMGError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _block(t: torch.Tensor, n: int, max_cols: int | None = None):
    """(nrhs, ld) of a block of vectors of length n: a 1-D tensor of n elements,
    or a 2-D (nrhs, n) tensor with unit column stride and row stride ld >= n.
    Checked before anything reaches the device."""
    if t.dim() == 1:
        if t.shape[0] != n:
            raise SMGError(f"expected a vector of {n} elements, got shape {tuple(t.shape)}")
        nrhs, ld = 1, n
    elif t.dim() == 2:
        if t.shape[1] != n or t.shape[0] < 1:
            raise SMGError(f"expected an (nrhs, {n}) block, got shape {tuple(t.shape)}")
        if t.stride(1) != 1 or (t.shape[0] > 1 and t.stride(0) < n):
            raise SMGError("block rows must be contiguous with a row stride >= n")
        nrhs, ld = t.shape[0], (t.stride(0) if t.shape[0] > 1 else n)
    else:
        raise SMGError(f"expected a 1-D or 2-D tensor, got shape {tuple(t.shape)}")
    if max_cols is not None and nrhs > max_cols:
        raise SMGError(f"{nrhs} right-hand sides exceed max_nrhs = {max_cols}")
    return nrhs, ld


def _on_device(*ts: torch.Tensor):
    for t in ts:
        if not t.is_cuda or t.dtype != torch.float64:
            raise SMGError("expected a float64 CUDA tensor")


def _like(t: torch.Tensor) -> torch.Tensor:
    """An output with t's shape and strides (the library uses one leading dimension for both)."""
    return torch.empty_strided(t.shape, t.stride(), dtype=t.dtype, device=t.device)


def _same_layout(a: torch.Tensor, b: torch.Tensor):
    if a.shape != b.shape or (a.dim() == 2 and a.shape[0] > 1 and a.stride() != b.stride()):
        raise SMGError(f"output shape/strides {tuple(b.shape)}/{b.stride()} differ from the input's "
                       f"{tuple(a.shape)}/{a.stride()}")
    if b.dtype != a.dtype or b.device != a.device:
        raise SMGError("output dtype/device differ from the input's")


class Info(dict):
    __getattr__ = dict.__getitem__


def apply_static(shape, r: torch.Tensor, s: torch.Tensor | None = None, c=(1.0, 1.0, 1.0), pre=1, post=1,
                 inner_pre=-1, inner_post=-1, order=0, precision="f64", kernel_mode=0) -> torch.Tensor:
    """s = T r through smg_apply_static: no handle, no workspace, no device
    allocation by the library (the hierarchy lives in its static scratch)."""
    shape = tuple(int(v) for v in shape)
    n = shape[0] * shape[1] * shape[2]
    nrhs, ld = _block(r, n)
    if s is None:
        s = _like(r)
    _same_layout(r, s)
    _on_device(r, s)
    grid = smg_grid(*shape, *[float(v) for v in c])
    opts = smg_opts(pre, post, inner_pre, inner_post, order, PREC[precision], kernel_mode)
    _check(lib().smg_apply_static(C.byref(grid), C.byref(opts), C.c_void_p(r.data_ptr()), C.c_void_p(s.data_ptr()),
                                  nrhs, ld, _stream()), "smg_apply_static")
    return s


class SMG:
    """One SMG hierarchy on the GPU for an (nx, ny, nz) brick with coefficients c."""

    def __init__(self, shape, c=(1.0, 1.0, 1.0), pre=1, post=1, inner_pre=-1, inner_post=-1, order=0,
                 precision="f64", max_nrhs=1, device="cuda", kernel_mode=0, ws_fill=None):
        L = lib()
        self.shape = tuple(int(v) for v in shape)
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        self.grid = smg_grid(*self.shape, *[float(v) for v in c])
        self.opts = smg_opts(pre, post, inner_pre, inner_post, order, PREC[precision], kernel_mode)
        self.max_nrhs = int(max_nrhs)
        nbytes = C.c_size_t(0)
        _check(L.smg_workspace_bytes(C.byref(self.grid), C.byref(self.opts), self.max_nrhs,
                                     C.byref(nbytes)), "smg_workspace_bytes")
        self.ws_bytes = nbytes.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        if ws_fill is not None:             # byte pattern left in the workspace before setup
            self.ws.fill_(int(ws_fill))
        h = C.c_void_p()
        _check(L.smg_setup(C.byref(self.grid), C.byref(self.opts), self.max_nrhs,
                           C.c_void_p(self.ws.data_ptr()), self.ws_bytes, _stream(), C.byref(h)),
               "smg_setup")
        self.h = h

    @classmethod
    def variable(cls, shape, diag, ax, ay, az, pre=1, post=1, inner_pre=-1, inner_post=-1, order=0,
                 interp="operator", max_nrhs=1, device="cuda"):
        """SMG for the variable-coefficient 7-point operator (A x)_p = diag[p] x_p
        - sum_e (a_e[p] x_{p+e} + a_e[p-e] x_{p-e}) (smgv_setup); diag, ax, ay, az
        are float64 tensors (or arrays) of nx*ny*nz values, x fastest.
        interp: "linear" or "operator" (operator-dependent) prolongation weights."""
        L = lib()
        G = object.__new__(cls)
        G.shape = tuple(int(v) for v in shape)
        G.n = G.shape[0] * G.shape[1] * G.shape[2]
        G.grid = smg_grid(*G.shape, 1.0, 1.0, 1.0)
        G.opts = smg_opts(pre, post, inner_pre, inner_post, order, PREC["f64"], 0)
        G.max_nrhs = int(max_nrhs)
        G.variable_coefficients = True
        coef = []
        for a in (diag, ax, ay, az):
            t = torch.as_tensor(a, dtype=torch.float64).to(device).contiguous().reshape(-1)
            if t.numel() != G.n:
                raise SMGError(f"coefficient arrays need {G.n} values, got {t.numel()}")
            coef.append(t)
        ip = {"linear": 0, "operator": 1}[interp]
        nbytes = C.c_size_t(0)
        _check(L.smgv_workspace_bytes(*G.shape, C.byref(G.opts), ip, G.max_nrhs, C.byref(nbytes)),
               "smgv_workspace_bytes")
        G.ws_bytes = nbytes.value
        G.ws = torch.empty(G.ws_bytes, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(L.smgv_setup(*G.shape, *[C.c_void_p(t.data_ptr()) for t in coef], ip, C.byref(G.opts), G.max_nrhs,
                            C.c_void_p(G.ws.data_ptr()), G.ws_bytes, _stream(), C.byref(h)), "smgv_setup")
        G.h = h
        return G

    def levels(self):
        """(3D levels, 2D levels per plane) of a variable-coefficient hierarchy."""
        a, b = C.c_int32(0), C.c_int32(0)
        _check(lib().smgv_levels(self.h, C.byref(a), C.byref(b)), "smgv_levels")
        return a.value, b.value

    def export(self, level: int, level2: int = -1, nz_l: int | None = None, ny_l2: int | None = None):
        """The stored operator of a variable-coefficient hierarchy (smgv_export) as a
        float64 CPU tensor: (8, nz_l, ny, nx) for a 3D level, (5, nz_l, ny_l2, nx) for
        the 2D level `level2` of its planes."""
        nx, ny, _ = self.shape
        narr = 8 if level2 < 0 else 5
        rows = ny if level2 < 0 else ny_l2
        out = torch.empty(narr * nz_l * rows * nx, dtype=torch.float64, device=self.ws.device)
        _check(lib().smgv_export(self.h, int(level), int(level2), C.c_void_p(out.data_ptr()), _stream()),
               "smgv_export")
        return out.cpu().reshape(narr, nz_l, rows, nx)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.smg_destroy(h)
            self.h = None

    def apply(self, r: torch.Tensor, s: torch.Tensor | None = None) -> torch.Tensor:
        """s = T r; r is (n,) or (nrhs, n) (one vector per row, row stride >= n)."""
        nrhs, ld = _block(r, self.n, self.max_nrhs)
        if s is None:
            s = _like(r)
        _same_layout(r, s)
        _on_device(r, s)
        _check(lib().smg_apply(self.h, C.c_void_p(r.data_ptr()), C.c_void_p(s.data_ptr()), nrhs, ld, _stream()),
               "smg_apply")
        return s

    def matvec(self, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        """y = A x; x is (n,) or (nrhs, n) (one vector per row, row stride >= n)."""
        nrhs, ld = _block(x, self.n)
        if y is None:
            y = _like(x)
        _same_layout(x, y)
        _on_device(x, y)
        _check(lib().smg_matvec(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nrhs, ld, _stream()),
               "smg_matvec")
        return y

    def _solve(self, fn, b, x, rtol, max_iter, precond, history, zero_x0, net=None, stop="2", xstar=None):
        vecs = [t for t in (b, x, xstar) if t is not None]
        for t in vecs:                      # sizes first, then the device
            if t.numel() != self.n:
                raise SMGError(f"expected {self.n} elements, got a tensor of shape {tuple(t.shape)}")
        for t in vecs:
            _dptr(t, self.n)
        if max_iter < 0:
            raise SMGError("max_iter must be >= 0")
        if x is None:
            x = torch.empty_like(b)
            x0_zero = 1
        else:
            x0_zero = 1 if zero_x0 else 0
        dbl = C.POINTER(C.c_double)
        hist = (C.c_double * (max_iter + 1))() if history else None
        histc = (C.c_double * max(max_iter, 1))() if history else None
        erra = (C.c_double * (max_iter + 1))() if xstar is not None else None
        sina = (C.c_double * max(max_iter, 1))() if xstar is not None else None
        work = torch.empty(2 * self.n, dtype=torch.float64, device=b.device) if xstar is not None else None
        o = krylov_opts(rtol, max_iter, PRECOND[precond], x0_zero, STOP[stop],
                        C.cast(hist, dbl) if history else None, C.cast(histc, dbl) if history else None,
                        C.c_void_p(xstar.data_ptr()) if xstar is not None else None,
                        C.c_void_p(work.data_ptr()) if work is not None else None,
                        C.cast(erra, dbl) if erra is not None else None,
                        C.cast(sina, dbl) if sina is not None else None)
        info = krylov_info()
        if net is None:
            code = fn(self.h, _dptr(b, self.n), _dptr(x, self.n), C.byref(o), C.byref(info), _stream())
        else:
            ninfo = net_solve_info()
            code = fn(self.h, net.h, _dptr(b, self.n), _dptr(x, self.n), C.byref(o), C.byref(info),
                      C.byref(ninfo), _stream())
        _check(code, fn.__name__, ok=(SMG_OK, SMG_NOT_CONVERGED))
        out = Info(iters=info.iters, status=info.status, rel_res=info.rel_res,
                   true_rel_res=info.true_rel_res, seconds=info.solve_seconds, rel_res_c=info.rel_res_c)
        if net is not None:
            out["fallback_iter"] = ninfo.fallback_iter
            out["fallback_reason"] = FALLBACK[ninfo.fallback_reason]
        if history:
            out["history"] = list(hist[:info.iters + 1])
            nc = info.iters + (1 if stop == "c" and info.status == SMG_OK else 0)
            out["history_c"] = list(histc[:min(nc, max_iter)])
        if xstar is not None:
            out["err_a"] = list(erra[:info.iters + 1])
            out["sin_angle"] = list(sina[:info.iters])
        return x, out

    def pcg(self, b, x=None, rtol=1e-8, max_iter=500, precond="smg", history=False, zero_x0=False, stop="2",
            xstar=None):
        """Algorithm 1 with beta from equation (1); stop "2" (||r||/||b||) or "c" (C-norm ratio); xstar: exact
        solution for the per-step Section 5 diagnostics (err_a, sin_angle)."""
        return self._solve(lib().pcg_solve, b, x, rtol, max_iter, precond, history, zero_x0, stop=stop,
                           xstar=xstar)

    def fpcg(self, b, x=None, rtol=1e-8, max_iter=500, precond="smg", history=False, zero_x0=False, stop="2",
            xstar=None):
        """Algorithm 1 with beta from equation (2); stop "2" (||r||/||b||) or "c" (C-norm ratio); xstar: exact
        solution for the per-step Section 5 diagnostics (err_a, sin_angle)."""
        return self._solve(lib().fpcg_solve, b, x, rtol, max_iter, precond, history, zero_x0, stop=stop,
                           xstar=xstar)

    def psd(self, b, x=None, rtol=1e-8, max_iter=500, precond="smg", history=False, zero_x0=False, stop="2",
            xstar=None):
        """Algorithm 1 with beta = 0; stop "2" (||r||/||b||) or "c" (C-norm ratio); xstar: exact
        solution for the per-step Section 5 diagnostics (err_a, sin_angle)."""
        return self._solve(lib().psd_solve, b, x, rtol, max_iter, precond, history, zero_x0, stop=stop,
                           xstar=xstar)

    def fpcg_learned(self, net, b, x=None, rtol=1e-8, max_iter=500, history=False, zero_x0=False):
        """Flexible PCG with the V-cycle followed by the learned correction of `net` (with fallback)."""
        if net.max_voxels < self.n:
            raise SMGError(f"network workspace holds {net.max_voxels} voxels, the grid has {self.n}")
        return self._solve(lib().fpcg_learned_solve, b, x, rtol, max_iter, "smg", history, zero_x0, net=net)

    def lobpcg(self, X0: torch.Tensor, rtol=1e-8, max_iter=500, precond="smg", guard=0):
        """LOBPCG for the m smallest eigenpairs; X0 is (m + guard, n), one initial vector per row.

        Returns (Ritz values (m + guard,) as a NumPy array, Ritz vectors (m + guard, n), info);
        convergence is required of the first m."""
        if X0.dim() != 2 or X0.shape[1] != self.n:
            raise SMGError(f"X0 must be (m + guard, {self.n}), got shape {tuple(X0.shape)}")
        mb = X0.shape[0]
        m = mb - guard
        if guard < 0 or m < 1:
            raise SMGError(f"need at least one wanted column (block {mb}, guard {guard})")
        if precond == "smg" and mb > self.max_nrhs:
            raise SMGError(f"block of {mb} columns exceeds max_nrhs = {self.max_nrhs}")
        if not X0.is_cuda or X0.dtype != torch.float64:
            raise SMGError("X0 must be a float64 CUDA tensor")
        nbytes = C.c_size_t(0)
        _check(lib().lobpcg_workspace_bytes(self.h, mb, C.byref(nbytes)), "lobpcg_workspace_bytes")
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=X0.device)
        X = X0.clone().contiguous()
        lam = (C.c_double * mb)()
        res = (C.c_double * mb)()
        o = lobpcg_opts(rtol, max_iter, PRECOND[precond], guard, 0)
        info = lobpcg_info()
        code = lib().lobpcg_solve(self.h, m, _dptr(X), C.cast(lam, C.c_void_p), C.cast(res, C.c_void_p),
                                  C.c_void_p(ws.data_ptr()), nbytes.value, C.byref(o), C.byref(info), _stream())
        _check(code, "lobpcg_solve", ok=(SMG_OK, SMG_NOT_CONVERGED))
        import numpy as np
        out = Info(iters=info.iters, nconv=info.nconv, status=info.status, seconds=info.seconds,
                   resnorms=np.array(res[:]))
        return np.array(lam[:]), X, out

    def _theory_args(self, ht, v0, nwork):
        if ht is not None and ht.n != self.n:
            raise SMGError("the transposed preconditioner must be on the same grid")
        _dptr(v0, self.n)
        return torch.empty(nwork * self.n, dtype=torch.float64, device=v0.device)

    def delta(self, c: float, v0: torch.Tensor, iters: int = 50, transpose: "SMG | None" = None) -> float:
        """Power-iteration estimate of ||I - c A T||_{A^{-1}} (Section 5, assumption (4));
        transpose: a handle of T's transpose (pre and post swapped), self when omitted."""
        ht = self if transpose is None else transpose
        work = self._theory_args(ht, v0, 5)
        out = C.c_double(0)
        _check(lib().smg_delta(self.h, ht.h, float(c), _dptr(v0, self.n), int(iters), C.c_void_p(work.data_ptr()),
                               C.byref(out), _stream()), "smg_delta")
        return out.value

    def delta_min(self, v0: torch.Tensor, c_lo=0.5, c_hi=2.0, tol=1e-3, iters: int = 50,
                  transpose: "SMG | None" = None):
        """(c, min_c ||I - c A T||_{A^{-1}}) by golden-section search over [c_lo, c_hi]."""
        ht = self if transpose is None else transpose
        work = self._theory_args(ht, v0, 5)
        cb, out = C.c_double(0), C.c_double(0)
        _check(lib().smg_delta_min(self.h, ht.h, float(c_lo), float(c_hi), float(tol), _dptr(v0, self.n), int(iters),
                                   C.c_void_p(work.data_ptr()), C.byref(cb), C.byref(out), _stream()),
               "smg_delta_min")
        return cb.value, out.value

    def spectrum(self, v0: torch.Tensor, iters: int = 50):
        """(lambda_min, lambda_max) of T A for an SPD T (pre = post) by power iteration."""
        work = self._theory_args(None, v0, 3)
        lo, hi = C.c_double(0), C.c_double(0)
        _check(lib().smg_spectrum(self.h, _dptr(v0, self.n), int(iters), C.c_void_p(work.data_ptr()), C.byref(lo),
                                  C.byref(hi), _stream()), "smg_spectrum")
        return lo.value, hi.value

    def autotune(self, r: torch.Tensor, reps: int = 5):
        """Times the candidate fused schedules on r and keeps the fastest; returns the tuning info."""
        s = torch.empty_like(r)
        info = smg_tune_info()
        _check(lib().smg_autotune(self.h, _dptr(r, self.n), _dptr(s, self.n), reps, _stream(), C.byref(info)),
               "smg_autotune")
        return Info(candidates=info.candidates, l0=info.l0, s_down=info.s_down, s_up=info.s_up,
                    march_waves=info.march_waves, coarse_lds=info.coarse_lds, default_ms=info.default_ms,
                    best_ms=info.best_ms)

    def schedule(self):
        """(l0, coarse kernel LDS bytes, marching threshold) of the fused 2D-cycle schedule in use."""
        info = smg_tune_info()
        _check(lib().smg_get_schedule(self.h, C.byref(info)), "smg_get_schedule")
        return info.l0, info.coarse_lds, info.march_waves

    def set_march(self, march_waves: int):
        """Marching threshold of the register-only pre-smoothing kernels (0: never march)."""
        _check(lib().smg_set_march(self.h, int(march_waves)), "smg_set_march")

    def profile_gram(self, m: int, k: int, reps: int = 5) -> float:
        """ms of one LOBPCG Gram product S^T S for an n x k block (k <= 3m)."""
        nbytes = C.c_size_t(0)
        _check(lib().lobpcg_workspace_bytes(self.h, m, C.byref(nbytes)), "lobpcg_workspace_bytes")
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        ms = C.c_double(0)
        _check(lib().lobpcg_profile_gram(self.h, m, k, C.c_void_p(ws.data_ptr()), nbytes.value, reps, _stream(),
                                         C.byref(ms)), "lobpcg_profile_gram")
        return ms.value

    def profile_kernel(self, family: str, r: torch.Tensor, reps: int = 3):
        """(launches per V-cycle, kernel ms per V-cycle, algorithmic bytes per V-cycle) of one kernel family."""
        if family not in KERNELS:
            raise SMGError(f"unknown kernel family {family!r}")
        rp = _dptr(r, self.n)
        s = torch.empty_like(r)
        nl, ms, by = C.c_int32(0), C.c_double(0), C.c_double(0)
        _check(lib().smg_profile_kernel(self.h, KERNELS[family], rp, _dptr(s, self.n), reps, _stream(),
                                        C.byref(nl), C.byref(ms), C.byref(by)), "smg_profile_kernel")
        return nl.value, ms.value, by.value

    def profile_levels(self, r: torch.Tensor, reps: int = 3, family: str | None = None):
        """Per 3D level (finest first, then the prolongation chain spanning every
        level): (launches, kernel ms, algorithmic bytes) per V-cycle, of every
        launch or of one kernel family."""
        if family is not None and family not in KERNELS:
            raise SMGError(f"unknown kernel family {family!r}")
        rp = _dptr(r, self.n)
        s = torch.empty_like(r)
        rows = 64
        nl = (C.c_int32 * rows)()
        ms = (C.c_double * rows)()
        by = (C.c_double * rows)()
        nr = C.c_int32(0)
        fam = -1 if family is None else KERNELS[family]
        _check(lib().smg_profile_levels(self.h, fam, rp, _dptr(s, self.n), reps, _stream(), rows, C.byref(nr),
                                        C.cast(nl, C.c_void_p), C.cast(ms, C.c_void_p), C.cast(by, C.c_void_p)),
               "smg_profile_levels")
        return [(nl[i], ms[i], by[i]) for i in range(nr.value)]


def _tptr(t: torch.Tensor, dtype, n: int | None = None):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise SMGError(f"expected a contiguous {dtype} CUDA tensor")
    if n is not None and t.numel() < n:
        raise SMGError("tensor too small")
    return C.c_void_p(t.data_ptr())


class Net:
    """The learned post-smoother network (include/smg_net.h) in the caller's device workspace."""

    def __init__(self, max_voxels: int, precision="bf16", train=False, device="cuda"):
        L = lib()
        self.precision = precision
        self.storage = torch.bfloat16 if precision == "bf16" else torch.float64
        self.accum = torch.float32 if precision == "bf16" else torch.float64
        self.max_voxels = int(max_voxels)
        self.train_mode = 1 if train else 0
        nbytes = C.c_size_t(0)
        _check(L.net_workspace_bytes(self.max_voxels, NET_PREC[precision], self.train_mode, C.byref(nbytes)),
               "net_workspace_bytes")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(L.net_setup(self.max_voxels, NET_PREC[precision], self.train_mode, C.c_void_p(self.ws.data_ptr()),
                           nbytes.value, _stream(), C.byref(h)), "net_setup")
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.net_destroy(h)
            self.h = None

    def set_params(self, params):
        import numpy as np
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        if a.size != NET_NPARAMS:
            raise SMGError("wrong parameter count")
        _check(lib().net_set_params(self.h, C.c_void_p(a.ctypes.data), _stream()), "net_set_params")

    def get_params(self):
        import numpy as np
        a = np.empty(NET_NPARAMS, dtype=np.float64)
        _check(lib().net_get_params(self.h, C.c_void_p(a.ctypes.data), _stream()), "net_get_params")
        return a

    def layer_forward(self, layer: int, shape, inp: torch.Tensor) -> torch.Tensor:
        nx, ny, nz = shape
        n = nx * ny * nz
        cin = 1 if layer == 0 else 16
        if layer == 3:
            out = torch.empty(n, dtype=self.accum, device=inp.device)
        else:
            out = torch.empty(n * 16, dtype=self.storage, device=inp.device)
        _check(lib().net_layer_forward(self.h, layer, nx, ny, nz, _tptr(inp, self.storage, n * cin),
                                       C.c_void_p(out.data_ptr()), _stream()), "net_layer_forward")
        return out

    def loss_grad(self, shape, inp: torch.Tensor, target: torch.Tensor, loss="mse"):
        import numpy as np
        nx, ny, nz = shape
        n = nx * ny * nz
        val = C.c_double(0)
        g = np.empty(NET_NPARAMS, dtype=np.float64)
        _check(lib().net_loss_grad(self.h, nx, ny, nz, _tptr(inp, self.storage, n), _tptr(target, self.accum, n),
                                   NET_LOSS[loss], C.byref(val), C.c_void_p(g.ctypes.data), _stream()),
               "net_loss_grad")
        return val.value, g

    def adam_step(self, lr: float):
        _check(lib().net_adam_step(self.h, float(lr), _stream()), "net_adam_step")

    def train(self, shape, inputs: torch.Tensor, targets: torch.Tensor, order, lr, loss="mse"):
        """Adam steps on pairs order[k] with learning rates lr[k]; returns the loss history."""
        import numpy as np
        nx, ny, nz = shape
        n = nx * ny * nz
        npairs = inputs.numel() // n
        o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
        r = np.ascontiguousarray(np.asarray(lr, dtype=np.float64))
        if o.size != r.size:
            raise SMGError("order and lr must have the same length")
        hist = np.empty(max(o.size, 1), dtype=np.float64)
        _check(lib().net_train(self.h, nx, ny, nz, _tptr(inputs, self.storage, npairs * n),
                               _tptr(targets, self.accum, npairs * n), npairs, o.size, C.c_void_p(o.ctypes.data),
                               C.c_void_p(r.ctypes.data), NET_LOSS[loss], C.c_void_p(hist.ctypes.data), _stream()),
               "net_train")
        return hist[:o.size]

    def correct(self, smg: "SMG", r: torch.Tensor, s: torch.Tensor, out: torch.Tensor | None = None):
        """out = s + sigma N(r'/(cbar sigma)), r' = r - A s; returns (out, sigma)."""
        if out is None:
            out = torch.empty_like(s)
        sig = C.c_double(0)
        _check(lib().net_correct(self.h, smg.h, _dptr(r, smg.n), _dptr(s, smg.n), _dptr(out, smg.n),
                                 C.byref(sig), _stream()), "net_correct")
        return out, sig.value

    def make_pairs(self, smg_pre: "SMG", smg_exact: "SMG", npairs: int, seed0: int, exact_rtol=1e-13,
                   exact_max_iter=200):
        """Training pairs on smg_pre's grid: (inputs, targets, sigmas)."""
        import numpy as np
        n = smg_pre.n
        inputs = torch.empty(npairs * n, dtype=self.storage, device=self.ws.device)
        targets = torch.empty(npairs * n, dtype=self.accum, device=self.ws.device)
        sig = np.empty(npairs, dtype=np.float64)
        _check(lib().net_make_pairs(self.h, smg_pre.h, smg_exact.h, npairs, int(seed0), float(exact_rtol),
                                    int(exact_max_iter), C.c_void_p(inputs.data_ptr()),
                                    C.c_void_p(targets.data_ptr()), C.c_void_p(sig.ctypes.data), _stream()),
               "net_make_pairs")
        return inputs, targets, sig


class SMGBatch:
    """Batched flexible PCG over independent boxes (smg_batch_* in include/smg.h).

    smgs: list of FP64 SMG handles (one per box); b, x: lists of device vectors
    bound to the batch.  use_graph: replay one captured iteration per step."""

    def __init__(self, smgs, b, x, use_graph=True):
        L = lib()
        n = len(smgs)
        if not (len(b) == len(x) == n) or n < 1:
            raise SMGError("need one b and one x per box")
        self.smgs, self.b, self.x = list(smgs), list(b), list(x)
        for G, bi, xi in zip(self.smgs, self.b, self.x):
            _dptr(bi, G.n)
            _dptr(xi, G.n)
        self._hs = (C.c_void_p * n)(*[G.h.value for G in self.smgs])
        self._bp = (C.c_void_p * n)(*[bi.data_ptr() for bi in self.b])
        self._xp = (C.c_void_p * n)(*[xi.data_ptr() for xi in self.x])
        nbytes = C.c_size_t(0)
        _check(L.smg_batch_workspace_bytes(C.cast(self._hs, C.c_void_p), n, C.byref(nbytes)),
               "smg_batch_workspace_bytes")
        self.ws = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=self.b[0].device)
        h = C.c_void_p()
        _check(L.smg_batch_create(C.cast(self._hs, C.c_void_p), n, C.cast(self._bp, C.c_void_p),
                                  C.cast(self._xp, C.c_void_p), C.c_void_p(self.ws.data_ptr()), nbytes.value,
                                  1 if use_graph else 0, _stream(), C.byref(h)), "smg_batch_create")
        self.h = h
        self.nbox = n

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.smg_batch_destroy(h)
            self.h = None

    def stats(self):
        """(grouped launches per iteration, per-box launches they replace)."""
        a, b = C.c_int32(0), C.c_int32(0)
        _check(lib().smg_batch_stats(self.h, C.byref(a), C.byref(b)), "smg_batch_stats")
        return a.value, b.value

    def fpcg(self, rtol=1e-8, max_iter=500, zero_x0=True):
        """Solves every box; returns one Info per box (status, iters, rel_res, true_rel_res, seconds)."""
        o = krylov_opts(rtol, max_iter, PRECOND["smg"], 1 if zero_x0 else 0, 0, None, None)
        infos = (krylov_info * self.nbox)()
        code = lib().smg_batch_fpcg(self.h, C.byref(o), C.cast(infos, C.c_void_p), _stream())
        if code < 0 and code != -4 and code != -5:
            _check(code, "smg_batch_fpcg")
        return [Info(iters=i.iters, status=i.status, rel_res=i.rel_res, true_rel_res=i.true_rel_res,
                     seconds=i.solve_seconds) for i in infos]
