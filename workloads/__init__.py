"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This module only assembles matrices and right-hand sides.  It holds none of
the solver's arithmetic, and it imports neither the oracle nor the GPU
package: both sides read the very same arrays from here.

Every matrix is returned as CSR with int32 row pointers / column indices and
float64 values (`Csr` below).  Random draws use numpy's PCG64
(`default_rng(seed)`) and are taken in a fixed order (coefficients, then b,
then x*), so every input is reproducible from its seed.

The workloads stand in for the paper's test matrices, which are not
available here (Matrix Market E20R5000 and the SuiteSparse set of the
stability study, Table "Properties of test matrices"; the 3D Laplace
matrices of the scaling study, Sec. 5).  Their shapes, nonzero counts per row
and spectra are chosen to match that class of PDE problems.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np


@dataclass
class Csr:
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        np.add.at(d, (rows, self.col), self.val)
        return d


def _from_coo(n, rows, cols, vals, name):
    """Sorted, duplicate-free CSR from COO triplets (rows/cols int64)."""
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    if rp[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 indexing")
    return Csr(n, rp.astype(np.int32), cols.astype(np.int32),
               np.ascontiguousarray(vals, dtype=np.float64), name)


def _stencil(shape, offsets_vals):
    """Assemble a constant-coefficient stencil on a Dirichlet box grid.

    shape: grid dims (slowest first); offsets_vals: list of (offset tuple,
    value or per-cell array).  Neighbours outside the box are dropped
    (homogeneous Dirichlet boundary).
    """
    dims = tuple(shape)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64).reshape(dims)
    rows_l, cols_l, vals_l = [], [], []
    for off, v in offsets_vals:
        src = [slice(None)] * len(dims)
        dst = [slice(None)] * len(dims)
        ok = True
        for d, o in enumerate(off):
            if o > 0:
                src[d] = slice(0, dims[d] - o)
                dst[d] = slice(o, dims[d])
            elif o < 0:
                src[d] = slice(-o, dims[d])
                dst[d] = slice(0, dims[d] + o)
            if dims[d] - abs(o) <= 0:
                ok = False
        if not ok:
            continue
        r = idx[tuple(src)].ravel()
        c = idx[tuple(dst)].ravel()
        if np.isscalar(v):
            vv = np.full(r.shape, float(v))
        else:
            vv = np.asarray(v)[tuple(src)].ravel()
        rows_l.append(r)
        cols_l.append(c)
        vals_l.append(vv)
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    vals = np.concatenate(vals_l)
    return n, rows, cols, vals


# --------------------------------------------------------------------------
# The five solver workloads
# --------------------------------------------------------------------------

def conv_diff_2d(nx: int = 64, peclet: float = 10.0) -> Csr:
    """2D convection-diffusion, 5-point first-order upwind, flow along (1,1).

    Rows are scaled by h^2: centre 4+2P, west/south -(1+P), east/north -1,
    with P the cell Peclet number in each direction.  Dirichlet boundary.
    """
    P = float(peclet)
    n, r, c, v = _stencil((nx, nx), [
        ((0, 0), 4.0 + 2.0 * P),
        ((0, -1), -(1.0 + P)), ((-1, 0), -(1.0 + P)),
        ((0, 1), -1.0), ((1, 0), -1.0)])
    return _from_coo(n, r, c, v, f"convdiff2d_{nx}_pe{peclet:g}")


def poisson_3d(nx: int = 128) -> Csr:
    """3D Poisson, 7-point (6, -1) on an nx^3 interior grid, Dirichlet."""
    A = poisson_3d_box((nx, nx, nx))
    A.name = f"poisson3d_{nx}"
    return A


def poisson_3d_box(shape) -> Csr:
    """3D Poisson, 7-point (6, -1) on a box grid of the given shape (slowest
    axis first), Dirichlet.  The couplings across the slowest axis lie one
    plane (shape[1] * shape[2] rows) from the diagonal."""
    offs = [((0, 0, 0), 6.0)]
    for d in range(3):
        for s in (-1, 1):
            o = [0, 0, 0]
            o[d] = s
            offs.append((tuple(o), -1.0))
    n, r, c, v = _stencil(tuple(shape), offs)
    return _from_coo(n, r, c, v, "poisson3d_" + "x".join(map(str, shape)))


def laplace_2d(nx: int) -> Csr:
    """2D Laplace, 5-point (4, -1), Dirichlet (the paper's Test 2 matrix)."""
    n, r, c, v = _stencil((nx, nx), [
        ((0, 0), 4.0), ((0, -1), -1.0), ((0, 1), -1.0),
        ((-1, 0), -1.0), ((1, 0), -1.0)])
    return _from_coo(n, r, c, v, f"laplace2d_{nx}")


def var_conv_diff_3d(nx: int = 192, seed: int = 3,
                     velocity=(20.0, 10.0, 5.0)) -> Csr:
    """3D variable-coefficient convection-diffusion, 7-point, upwind.

    Cell diffusion coefficients k ~ lognormal(0,1) (seeded).  The coefficient
    on an interior face is the harmonic mean of its two cells; a boundary face
    uses its cell's value.  Velocity components are positive, so first-order
    upwinding takes the lower neighbour in every direction.  Rows are scaled
    by h^2 with h = 1/(nx+1).
    """
    rng = np.random.default_rng(seed)
    k = rng.lognormal(0.0, 1.0, size=(nx, nx, nx))
    h = 1.0 / (nx + 1)
    n = nx ** 3
    idx = np.arange(n, dtype=np.int64).reshape(nx, nx, nx)
    diag = np.zeros((nx, nx, nx))
    rows_l, cols_l, vals_l = [], [], []
    # axis order (z, y, x) slowest first; velocity given as (x, y, z)
    vel = {2: velocity[0], 1: velocity[1], 0: velocity[2]}
    for d in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[d] = slice(0, nx - 1)
        hi[d] = slice(1, nx)
        lo, hi = tuple(lo), tuple(hi)
        kf = 2.0 * k[lo] * k[hi] / (k[lo] + k[hi])  # interior faces
        w = vel[d] * h
        # face between cell a=lo and b=hi: diffusion couples both ways
        diag[lo] += kf
        diag[hi] += kf
        # boundary faces (Dirichlet): low side of first cell, high side of last
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[d] = slice(0, 1)
        last[d] = slice(nx - 1, nx)
        diag[tuple(first)] += k[tuple(first)]
        diag[tuple(last)] += k[tuple(last)]
        # upwind convection (w > 0): + w (u_c - u_lower)
        diag += w
        # hi row gets -kf - w from its lower neighbour (lo)
        rows_l.append(idx[hi].ravel())
        cols_l.append(idx[lo].ravel())
        vals_l.append((-kf - w).ravel())
        # lo row gets -kf from its upper neighbour (hi)
        rows_l.append(idx[lo].ravel())
        cols_l.append(idx[hi].ravel())
        vals_l.append((-kf).ravel())
    rows_l.append(idx.ravel())
    cols_l.append(idx.ravel())
    vals_l.append(diag.ravel())
    return _from_coo(n, np.concatenate(rows_l), np.concatenate(cols_l),
                     np.concatenate(vals_l), f"varcd3d_{nx}")


def banded_random(n: int = 1_000_000, band: int = 1000, offdiag: int = 26,
                  seed: int = 4, diag_factor: float = 1.2) -> Csr:
    """Random banded nonsymmetric matrix.

    Every row i gets `offdiag` distinct off-diagonal columns drawn uniformly
    from [i-band, i+band] intersected with [0, n) minus {i}; values U(-1,1);
    the diagonal is diag_factor * (sum of |off-diagonal| in the row).
    """
    rng = np.random.default_rng(seed)
    if n - 1 < offdiag:
        raise ValueError("n too small for the requested row count")
    cols_all = np.empty((n, offdiag), dtype=np.int64)
    chunk = 65536
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        rows = np.arange(r0, r1)
        lo = np.maximum(rows - band, 0)
        hi = np.minimum(rows + band, n - 1)
        width = hi - lo  # number of admissible columns (window minus i)
        todo = np.arange(r1 - r0)
        out = np.empty((r1 - r0, offdiag), dtype=np.int64)
        draws = 2 * offdiag + 8
        while todo.size:
            u = rng.integers(0, 2**62, size=(todo.size, draws))
            t = u % width[todo, None]
            c = lo[todo, None] + t
            c = c + (c >= rows[todo, None])  # skip the diagonal
            # keep first occurrence of each value, in draw order
            order = np.argsort(c, axis=1, kind="stable")
            cs = np.take_along_axis(c, order, axis=1)
            dup_sorted = np.zeros_like(cs, dtype=bool)
            dup_sorted[:, 1:] = cs[:, 1:] == cs[:, :-1]
            dup = np.empty_like(dup_sorted)
            np.put_along_axis(dup, order, dup_sorted, axis=1)
            keep_rank = np.cumsum(~dup, axis=1)
            enough = keep_rank[:, -1] >= offdiag
            sel = (~dup) & (keep_rank <= offdiag)
            ok_rows = np.nonzero(enough)[0]
            for_rows = c[ok_rows][sel[ok_rows]].reshape(ok_rows.size, offdiag)
            out[todo[ok_rows]] = for_rows
            todo = todo[~enough]
        cols_all[r0:r1] = out
    vals = rng.uniform(-1.0, 1.0, size=(n, offdiag))
    d = diag_factor * np.abs(vals).sum(axis=1)
    rows = np.repeat(np.arange(n, dtype=np.int64), offdiag + 1)
    cols = np.concatenate([cols_all, np.arange(n)[:, None]], axis=1).ravel()
    allv = np.concatenate([vals, d[:, None]], axis=1).ravel()
    return _from_coo(n, rows, cols, allv, f"banded_{n}_{band}")


def aniso_diffusion_2d(nx: int = 4096, ratio: float = 1e-3,
                       angle_deg: float = 30.0) -> Csr:
    """2D anisotropic diffusion, 5-point, Dirichlet.

    The tensor is R(angle) diag(1, ratio) R(angle)^T; a 5-point stencil keeps
    only its K_xx and K_yy entries (centre 2(Kxx+Kyy), x-neighbours -Kxx,
    y-neighbours -Kyy).  Dropping K_xy removes most of the rotated tensor's
    anisotropy: at the default 30 degrees K_xx = 0.75025, K_yy = 0.25075, an
    axis ratio of 0.334; angle_deg = 0 keeps the full ratio along the axes.
    """
    a = math.radians(angle_deg)
    c, s = math.cos(a), math.sin(a)
    kxx = c * c + ratio * s * s
    kyy = s * s + ratio * c * c
    n, r, cc, v = _stencil((nx, nx), [
        ((0, 0), 2.0 * (kxx + kyy)),
        ((0, -1), -kxx), ((0, 1), -kxx),
        ((-1, 0), -kyy), ((1, 0), -kyy)])
    return _from_coo(n, r, cc, v, f"aniso2d_{nx}")


def diagonal(lams) -> Csr:
    """Diagonal matrix with the given eigenvalues (the paper's Tests 1, 3, 8)."""
    lams = np.asarray(lams, dtype=np.float64)
    n = lams.size
    return Csr(n, np.arange(n + 1, dtype=np.int32),
               np.arange(n, dtype=np.int32), lams.copy(), f"diag_{n}")


def rhs(n: int, seed: int) -> np.ndarray:
    """b ~ N(0,1), seeded."""
    return np.random.default_rng(seed).standard_normal(n)


def banded_problem(n: int, seed: int = 4, band: int = 1000):
    """Adjoint workload: matrix, b and target x* (drawn in that order)."""
    A = banded_random(n, band=min(band, n - 1), seed=seed)
    rng = np.random.default_rng(seed + 1000)
    b = rng.standard_normal(n)
    xstar = rng.standard_normal(n)
    return A, b, xstar


# --------------------------------------------------------------------------
# Named configurations (the solver settings travel with the workload)
# --------------------------------------------------------------------------

CONFIGS = {
    "convdiff2d_64": dict(make=lambda: conv_diff_2d(64, 10.0), seed=1,
                          s_max=8, restart=64, tol=1e-10, precond="none"),
    "poisson3d_128": dict(make=lambda: poisson_3d(128), seed=2,
                          s_max=32, restart=128, tol=1e-10, precond="none"),
    "varcd3d_192": dict(make=lambda: var_conv_diff_3d(192, 3), seed=3,
                        s_max=128, restart=256, tol=1e-10, precond="jacobi"),
    "banded_1m": dict(make=lambda: banded_random(1_000_000, 1000, 26, 4),
                      seed=4, s_max=8, restart=128, tol=1e-12,
                      precond="none"),
    "aniso2d_4096": dict(make=lambda: aniso_diffusion_2d(4096), seed=5,
                         s_max=200, restart=400, tol=1e-10, precond="none"),
}
