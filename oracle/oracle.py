"""ctypes wrapper of the FP64 C oracle (``smg_oracle.c``).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never does.

Functions mirror the paper's objects: the 7-point model operator (Section 2),
the SMG V-cycle preconditioner (Section 3; internals as read in the C file's
header) and Algorithm 1 with beta from equation (1), equation (2) or zero.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PCG, FPCG, PSD = 0, 1, 2
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        d, i, p = C.c_double, C.c_int, C.c_void_p
        L.oracle_matvec.argtypes = [i, i, i, d, d, d, p, p]
        L.oracle_line_solve.argtypes = [i, d, d, p, p, p]
        L.oracle_smg_create.argtypes = [i, i, i, d, d, d, i, i, i, i, i]
        L.oracle_smg_create.restype = p
        L.oracle_smg_destroy.argtypes = [p]
        L.oracle_smg_apply.argtypes = [p, p, p]
        L.oracle_smg_nlevels.argtypes = [p]
        L.oracle_smg_level_nz.argtypes = [p, i]
        L.oracle_smg_plane_coef.argtypes = [p, i, i, p]
        L.oracle_smg_plane_nlevels.argtypes = [p, i, i]
        L.oracle_smg_plane_level_ny.argtypes = [p, i, i, i]
        L.oracle_smg_line_coef.argtypes = [p, i, i, i, i, p]
        L.oracle_smg_plane_solve.argtypes = [p, i, i, p, p]
        L.oracle_krylov.argtypes = [p, i, i, i, i, d, d, d, p, p, d, i, i, p, p,
                                    C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_krylov.restype = i
        L.oracle_num_threads.restype = i
        L.oracle_set_num_threads.argtypes = [i]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops from now on."""
    lib().oracle_set_num_threads(int(n))


def matvec(x: np.ndarray, shape, c=(1.0, 1.0, 1.0)) -> np.ndarray:
    """y = A x for the 7-point operator on an (nx, ny, nz) brick, x flattened x-fastest."""
    nx, ny, nz = shape
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    y = np.empty_like(x)
    lib().oracle_matvec(nx, ny, nz, c[0], c[1], c[2], _ptr(x), _ptr(y))
    return y


def line_solve(a: float, b: float, f: np.ndarray) -> np.ndarray:
    """Exact solve of (a*Tx + b*I) u = f, Tx = tridiag(-1, 2, -1)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    u = np.empty_like(f)
    w = np.empty_like(f)
    lib().oracle_line_solve(f.size, a, b, _ptr(f), _ptr(u), _ptr(w))
    return u


class SMG:
    """The oracle's SMG V-cycle preconditioner B on one brick."""

    def __init__(self, shape, c=(1.0, 1.0, 1.0), pre=1, post=1, ipre=-1, ipost=-1, order=0):
        self.shape = tuple(int(v) for v in shape)
        self.c = tuple(float(v) for v in c)
        nx, ny, nz = self.shape
        self.h = lib().oracle_smg_create(nx, ny, nz, self.c[0], self.c[1], self.c[2],
                                         pre, post, ipre, ipost, order)
        if not self.h:
            raise ValueError("invalid SMG parameters")
        self.n = nx * ny * nz

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().oracle_smg_destroy(h)
            self.h = None

    def apply(self, r: np.ndarray) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
        assert r.size == self.n
        s = np.empty_like(r)
        lib().oracle_smg_apply(self.h, _ptr(r), _ptr(s))
        return s

    def nlevels(self) -> int:
        return lib().oracle_smg_nlevels(self.h)

    def level_nz(self, l: int) -> int:
        return lib().oracle_smg_level_nz(self.h, l)

    def plane_coef(self, l: int, K: int) -> np.ndarray:
        """(alpha, beta, gamma, delta) of C_K = alpha*T2 + beta*I, U_K = gamma*T2 + delta*I."""
        out = np.zeros(4)
        lib().oracle_smg_plane_coef(self.h, l, K, _ptr(out))
        return out

    def plane_nlevels(self, l: int, K: int) -> int:
        return lib().oracle_smg_plane_nlevels(self.h, l, K)

    def plane_level_ny(self, l: int, K: int, l2: int) -> int:
        return lib().oracle_smg_plane_level_ny(self.h, l, K, l2)

    def line_coef(self, l: int, K: int, l2: int, j: int) -> np.ndarray:
        out = np.zeros(4)
        lib().oracle_smg_line_coef(self.h, l, K, l2, j, _ptr(out))
        return out

    def plane_solve(self, l: int, K: int, b: np.ndarray) -> np.ndarray:
        nx, ny, _ = self.shape
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
        assert b.size == nx * ny
        x = np.empty_like(b)
        lib().oracle_smg_plane_solve(self.h, l, K, _ptr(b), _ptr(x))
        return x


class KrylovResult:
    def __init__(self, status, iters, rel, true_rel, hist, histC, x):
        self.status, self.iters, self.rel, self.true_rel = status, iters, rel, true_rel
        self.hist, self.histC, self.x = hist, histC, x

    def __repr__(self):
        return (f"KrylovResult(status={self.status}, iters={self.iters}, rel={self.rel:.3e}, "
                f"true_rel={self.true_rel:.3e})")


def krylov(method: int, b: np.ndarray, shape, c=(1.0, 1.0, 1.0), smg: SMG | None = None,
           x0: np.ndarray | None = None, rtol=1e-8, max_iter=500, history=True, stop="2") -> KrylovResult:
    """Algorithm 1 with beta from (1) [PCG], (2) [FPCG] or 0 [PSD]; T = smg or identity.
    stop "2": ||r_k||_2 <= rtol ||b||_2; stop "c": sqrt|(T r_k, r_k)| <= rtol sqrt|(T b, b)|."""
    nx, ny, nz = shape
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64).reshape(-1)
    hist = np.full(max_iter + 1, np.nan) if history else None
    histC = np.full(max_iter + 1, np.nan) if history else None
    it, rel, trel = C.c_int(0), C.c_double(0), C.c_double(0)
    stop_c = 1 if stop == "c" else 0
    st = lib().oracle_krylov(smg.h if smg is not None else None, method, nx, ny, nz,
                             c[0], c[1], c[2], _ptr(b), _ptr(x), rtol, stop_c, max_iter,
                             _ptr(hist) if history else None, _ptr(histC) if history else None,
                             C.byref(it), C.byref(rel), C.byref(trel))
    k = it.value
    nc = k + (1 if stop_c and st == 0 else 0)
    return KrylovResult(st, k, rel.value, trel.value,
                        hist[:k + 1] if history else None,
                        histC[:nc] if history else None, x)
