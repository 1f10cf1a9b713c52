"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no arithmetic of the method: it only turns (seed, index)
counters into pseudo-random numbers, so that the CPU oracle and the GPU
library can be fed bit-identical right-hand sides and initial blocks.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-style: the value with index
``i`` under seed ``s`` is ``mix(s + (i + 1) * 0x9E3779B97F4A7C15)`` with the
published two-round xor-shift-multiply finaliser.  Uniforms take the top 53
bits; Gaussians use the Box-Muller transform of two consecutive uniforms.

The paper only says its initial approximations are pseudo-random (Section 2
model problem); the distributions used here are the workload recipe of the
benchmarks (uniform [-1, 1) right-hand sides, standard normal LOBPCG blocks).
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Raw 64-bit outputs with indices start .. start+count-1 (uint64 array)."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits."""
    z = splitmix64(seed, start, count)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_pm1(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Doubles in [-1, 1): the right-hand-side distribution of the workloads."""
    return 2.0 * uniform01(seed, count, start) - 1.0


def gaussian(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Standard normal doubles by Box-Muller on uniform pairs (2i, 2i+1)."""
    z = splitmix64(seed, 2 * start, 2 * count)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    u1 = 1.0 - u[0::2]          # (0, 1]: keeps log finite
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def rhs(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """Right-hand side b ~ U[-1, 1), flattened with x fastest (index i + nx*(j + ny*k))."""
    return uniform_pm1(seed, nx * ny * nz)


def block(n: int, m: int, seed: int) -> np.ndarray:
    """Initial LOBPCG block, n rows by m columns, column-major (column c is entries c*n .. c*n+n-1).

    Returned as an (m, n) C-contiguous array, i.e. one row per column vector.
    """
    return gaussian(seed, n * m).reshape(m, n)


def box_dims(count: int, lo: int, hi: int, seed: int) -> list:
    """``count`` boxes with nx, ny, nz drawn uniformly from the integers lo..hi inclusive."""
    u = uniform01(seed, 3 * count)
    d = lo + np.floor(u * (hi - lo + 1)).astype(np.int64)
    d = np.minimum(d, hi)
    return [tuple(int(v) for v in d[3 * i:3 * i + 3]) for i in range(count)]


NET_CHANNELS = (1, 16, 16, 16, 1)


def he_init(seed: int) -> np.ndarray:
    """Initial parameters of the learned post-smoother in the library's flat
    order (per layer W[3][3][3][cin][cout], then b): weights normal with
    variance 2/(27 cin) (He et al. 2015), biases normal with deviation 0.01,
    from the Gaussian stream of `seed`."""
    out, pos = [], 0
    for ci, co in zip(NET_CHANNELS[:-1], NET_CHANNELS[1:]):
        nw = 27 * ci * co
        out.append(gaussian(seed, nw, pos) * np.sqrt(2.0 / (27 * ci)))
        pos += nw
        out.append(0.01 * gaussian(seed, co, pos))
        pos += co
    return np.concatenate(out)


# --- variable-coefficient problems -----------------------------------------
# A diffusion problem -div(kappa grad u) on the brick, discretised like the
# model problem (one unknown per grid point, neighbours outside the brick are
# zero): the coupling across the face between two neighbours is the axis
# factor times the harmonic mean of their conductivities (kappa itself across a
# boundary face), and the diagonal is the sum of the six face couplings.  With
# kappa = 1 this is the model operator with coefficients c.

def conductivity(shape, kind: str, seed: int, contrast: float = 1e3):
    """Per-point conductivities (kx, ky, kz) of a named test field, x fastest:
    "const": 1 everywhere;
    "layers": z-layers of 2..9 planes, alternately 1 and `contrast`;
    "aniso_layers": the same layers, with kx = 100 ky inside every other layer;
    "lognormal": exp(1.5 g), g standard normal i.i.d. per point."""
    nx, ny, nz = shape
    n = nx * ny * nz
    one = np.ones(n)
    if kind == "const":
        return one, one.copy(), one.copy()
    if kind in ("layers", "aniso_layers"):
        u = uniform01(seed, nz)
        kz_plane, ax_plane = np.empty(nz), np.ones(nz)
        k, layer = 0, 0
        while k < nz:
            t = 2 + int(u[k] * 8)
            kz_plane[k:k + t] = contrast if layer % 2 else 1.0
            if kind == "aniso_layers" and layer % 2 == 0:
                ax_plane[k:k + t] = 100.0
            k += t
            layer += 1
        kap = np.repeat(kz_plane, nx * ny)
        return kap * np.repeat(ax_plane, nx * ny), kap.copy(), kap.copy()
    if kind == "lognormal":
        kap = np.exp(1.5 * gaussian(seed, n))
        return kap, kap.copy(), kap.copy()
    raise ValueError(kind)


def diffusion_stencil(shape, kx, ky, kz, c=(1.0, 1.0, 1.0)):
    """(diag, ax, ay, az) of the 7-point operator: A[p, p+e] = -a_e[p] for the
    neighbour p+e along each axis (a_e = 0 where p+e is outside the brick) and
    A[p, p] = diag[p]."""
    nx, ny, nz = shape
    shp = (nz, ny, nx)
    K = [np.asarray(v, dtype=np.float64).reshape(shp) for v in (kx, ky, kz)]
    diag = np.zeros(shp)
    out = []
    for axis, (Kx, cc) in enumerate(zip(K, c)):
        ax3 = 2 - axis                       # array axis of this grid axis (z, y, x order)
        a = np.zeros(shp)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax3] = slice(0, -1)
        hi[ax3] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        a[lo] = cc * 2.0 * Kx[lo] * Kx[hi] / (Kx[lo] + Kx[hi])
        diag += a
        diag[hi] += a[lo]
        # the two boundary faces along this axis couple to zero values outside
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[ax3] = 0
        last[ax3] = -1
        diag[tuple(first)] += cc * Kx[tuple(first)]
        diag[tuple(last)] += cc * Kx[tuple(last)]
        out.append(a.reshape(-1))
    return diag.reshape(-1), out[0], out[1], out[2]
