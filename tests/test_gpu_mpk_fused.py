"""The depth-k matrix powers kernel (temporal blocking over row slabs,
sgm_mpk_fused and the mpk_depth solve option) against the one-step kernel:
bitwise equal vectors and solves, in float64 and float32.

Every row of the fused kernel is computed by the same arithmetic as the
one-step SpMV, only in a different launch order, so the comparison is exact.
The matrices are large enough for at least three row slabs of the default
plan (about 8 MB of matrix and at least 1024 slices of 64 rows, or the
matrix bandwidth if larger), with a
ragged last slab, and include a 3D stencil, a 2D stencil and a banded
matrix; the recurrence records include complex conjugate pairs (the
delta term reads the vector two steps back).
"""
import numpy as np
import pytest

import workloads as W
from oracle import sstep_gmres as o

pytestmark = pytest.mark.gpu

MATS = [
    ("poisson3d_90", lambda: W.poisson_3d(90)),          # 729,000 rows, h 8,100
    ("laplace2d_800", lambda: W.laplace_2d(800)),        # 640,000 rows, h 800
    ("banded_200k", lambda: W.banded_random(200_003, band=1000, seed=3)),
]


def _records(s, seed):
    rng = np.random.default_rng(seed)
    ritz = []
    while len(ritz) < s:
        if len(ritz) + 2 <= s and rng.random() < 0.4:
            z = complex(rng.uniform(0.5, 8), rng.uniform(0.2, 2))
            ritz += [z, z.conjugate()]
        else:
            ritz.append(rng.uniform(0.5, 8))
    sh = o.newton_shifts(o.leja_order(np.array(ritz)), scaled=True)
    return np.stack([sh.theta, sh.gamma, sh.delta], 1), sh


@pytest.mark.parametrize("name,mk", MATS, ids=[m[0] for m in MATS])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_mpk_fused_bitwise_equal(lib, name, mk, precision):
    import torch
    A = mk()
    G = lib.Matrix.from_csr(A)
    n = A.n
    ld = ((n + 63) // 64) * 64
    s = 11
    rec, sh = _records(s, 5)
    assert np.count_nonzero(sh.delta) >= 1
    dt = np.float64 if precision == "fp64" else np.float32
    q = np.random.default_rng(2).standard_normal(n)
    q = (q / np.linalg.norm(q)).astype(dt)
    buf = np.zeros((s + 1, ld), dtype=dt)
    buf[0, :n] = q
    ref = torch.tensor(buf.ravel(), device="cuda")
    lib.mpk(G, ref, ld, 0, s, rec, precision=precision)
    ref_h = ref.cpu().numpy()
    assert np.all(np.isfinite(ref_h))
    for depth in (2, 3, 4):
        Qd = torch.tensor(buf.ravel(), device="cuda")
        slab = lib.mpk_fused(G, Qd, ld, 0, s, rec, depth, precision=precision)
        assert slab >= 64 * 1024 and (n + slab - 1) // slab >= 3, slab
        assert n % slab != 0                   # ragged last slab
        assert np.array_equal(Qd.cpu().numpy(), ref_h), (name, depth)


def test_mpk_fused_transpose_bitwise_equal(lib):
    import torch
    A = W.banded_random(200_003, band=1000, seed=3)
    G = lib.Matrix.from_csr(A)
    n, ld, s = A.n, ((A.n + 63) // 64) * 64, 8
    rec, _ = _records(s, 9)
    buf = np.zeros((s + 1, ld))
    buf[0, :n] = np.random.default_rng(4).standard_normal(n) / np.sqrt(n)
    ref = torch.tensor(buf.ravel(), device="cuda")
    lib.mpk(G, ref, ld, 0, s, rec, transpose=True)
    Qd = torch.tensor(buf.ravel(), device="cuda")
    lib.mpk_fused(G, Qd, ld, 0, s, rec, 4, transpose=True)
    assert np.array_equal(Qd.cpu().numpy(), ref.cpu().numpy())


def test_mpk_fused_small_matrix_runs_one_step_per_launch(lib):
    """Fewer than three slabs: the plan falls back to depth 1 (reported as
    slab height 0 and info mpk_depth 1) and the result is still the
    one-step kernel's."""
    import torch
    A = W.conv_diff_2d(64, 10.0)
    G = lib.Matrix.from_csr(A)
    n, ld, s = A.n, ((A.n + 63) // 64) * 64, 6
    rec, _ = _records(s, 1)
    buf = np.zeros((s + 1, ld))
    buf[0, :n] = 1.0 / np.sqrt(n)
    ref = torch.tensor(buf.ravel(), device="cuda")
    lib.mpk(G, ref, ld, 0, s, rec)
    Qd = torch.tensor(buf.ravel(), device="cuda")
    assert lib.mpk_fused(G, Qd, ld, 0, s, rec, 4) == 0
    assert np.array_equal(Qd.cpu().numpy(), ref.cpu().numpy())
    r = lib.solve(G, W.rhs(n, 1), s_max=8, restart=64, tol=1e-10,
                  mpk_depth=4)
    assert r.status == lib.OK and r.info["mpk_depth"] == 1


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_solve_with_fused_mpk_bitwise_equal(lib, precision):
    """Whole solves (s_max 16, restart 64, scaled Newton blocks after the
    pre-phase) with mpk_depth 1, 2 and 4: identical iterates, block sizes
    and residual histories."""
    A = W.poisson_3d(90)
    G = lib.Matrix.from_csr(A)
    b = W.rhs(A.n, 6)
    kw = dict(s_max=16, restart=64, tol=1e-10, precision=precision,
              max_restarts=100, max_outer=50)
    base = lib.solve(G, b, mpk_depth=1, **kw)
    assert base.status == lib.OK and max(base.s_hist) > 1
    xb = base.x.cpu().numpy()
    for depth in (2, 4):
        r = lib.solve(G, b, mpk_depth=depth, **kw)
        assert r.info["mpk_depth"] == depth and r.info["mpk_slab_rows"] > 0
        assert list(r.s_hist) == list(base.s_hist)
        assert np.array_equal(np.asarray(r.res_hist), np.asarray(base.res_hist))
        assert np.array_equal(r.x.cpu().numpy(), xb)


def test_mpk_depth_option_rejected_outside_range(lib):
    A = W.conv_diff_2d(16, 1.0)
    G = lib.Matrix.from_csr(A)
    for d in (0, 5):
        with pytest.raises(lib.SgmError, match="mpk_depth"):
            lib.solve(G, W.rhs(A.n, 1), mpk_depth=d)
