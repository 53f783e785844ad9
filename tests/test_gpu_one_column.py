"""GPU parity of one-column blocks (the column-wise Ritz pre-phase: CGS2
with the 1 x 1 partial Cholesky of Alg. 3) against the oracle's
block_orth, in float64 and float32.

Up to 256 prior columns the first update and the second projection share
one pass over Q: one wavefront per panel with 4-, 8-, 16- and 32-column
register tiles up to 32 columns, then 2 to 8 wavefronts per panel with 32
columns each; beyond 256 they are two passes.  The cases reach every tile
width, every wavefront count's edges and the two-pass path, on a ragged
row count, and include a vector almost inside span(Q), where the second
projection carries the re-orthogonalisation.
"""
import numpy as np
import pytest

from oracle import sstep_gmres as o

pytestmark = pytest.mark.gpu


def flat_cols(torch, M, ld, dtype):
    n, k = M.shape
    buf = np.zeros((k, ld), dtype=dtype)
    buf[:, :n] = M.T
    return torch.tensor(buf.ravel(), device="cuda")


def cols_of(t, n, ld, k):
    return t.cpu().numpy().reshape(k, ld)[:, :n].T


def _block(n, i, seed, delta=1.0):
    rng = np.random.default_rng(seed)
    Qi, _ = np.linalg.qr(rng.standard_normal((n, i)))
    v = Qi @ rng.standard_normal((i, 1)) + delta * rng.standard_normal((n, 1))
    return Qi, v


def _run(lib, Qi, v, precision):
    import torch
    n, i = Qi.shape
    ld = ((n + 63) // 64) * 64
    f32 = precision == "fp32_ir"
    wd = np.float32 if f32 else np.float64
    om = o.default_omega(o.U32 if f32 else o.U64)
    Qw, vw = Qi.astype(wd), v.astype(wd)
    ref = o.block_orth(np.asfortranarray(Qw.copy()), i, vw.copy(), om,
                       work_dtype=wd)
    Qd = flat_cols(torch, np.concatenate([Qw, vw], 1), ld, wd)
    p, Rt, Rk = lib.block_orth(Qd, n, ld, i, 1, omega=om, precision=precision)
    return p, Rt, Rk, cols_of(Qd, n, ld, i + 1).astype(np.float64), ref


@pytest.mark.parametrize("i", [1, 33, 64, 65, 129, 200, 256, 257])
def test_one_column_fp64(lib, i):
    n = 9001
    Qi, v = _block(n, i, seed=600 + i)
    p, Rt, Rk, Qg, ref = _run(lib, Qi, v, "fp64")
    assert p == ref.p == 1
    assert np.abs(Qg[:, i] - ref.Qk[:, 0]).max() <= 1e-12
    assert np.abs(Rt[:, 0] - ref.R_top[:, 0]).max() <= 1e-12 * np.abs(ref.R_top).max()
    assert abs(Rk[0, 0] - ref.R_kk[0, 0]) <= 1e-12 * abs(ref.R_kk[0, 0])
    assert o.loo(Qg[:, :i + 1]) <= 1e-13


@pytest.mark.parametrize("i", [3, 8, 12, 20, 32, 33, 47, 100, 256, 257])
def test_one_column_fp32(lib, i):
    n = 9001
    Qi, v = _block(n, i, seed=500 + i)
    p, Rt, Rk, Qg, ref = _run(lib, Qi, v, "fp32_ir")
    assert p == ref.p == 1
    # float32 rounding of the projections: a few units of 2^-24 per
    # prior column on unit-norm columns
    assert np.abs(Qg[:, i] - ref.Qk[:, 0]).max() <= 2e-6
    assert np.abs(Rt[:, 0] - ref.R_top[:, 0]).max() <= 1e-5 * np.abs(ref.R_top).max()
    assert abs(Rk[0, 0] - ref.R_kk[0, 0]) <= 1e-5 * abs(ref.R_kk[0, 0])
    assert o.loo(Qg[:, :i + 1]) <= 1e-5


@pytest.mark.parametrize("precision,i,tol_loo",
                         [("fp64", 32, 1e-13), ("fp64", 40, 1e-13),
                          ("fp64", 200, 1e-13), ("fp32_ir", 32, 1e-5),
                          ("fp32_ir", 100, 1e-5)])
def test_one_column_near_span(lib, precision, i, tol_loo):
    """v = Q c + 1e-6 N in float64 (1e-3 N in float32): the first pass
    leaves components along Q of about u / delta relative to the result,
    which only the second projection removes."""
    f32 = precision == "fp32_ir"
    Qi, v = _block(4000, i, seed=77 + i, delta=1e-3 if f32 else 1e-6)
    p, Rt, Rk, Qg, ref = _run(lib, Qi, v, precision)
    assert p == ref.p == 1
    assert o.loo(Qg[:, :i + 1]) <= tol_loo
    # v = Q R_top + q R_kk to the working precision
    rec = Qi @ Rt[:, :1] + Qg[:, i:i + 1] * Rk[0, 0]
    eps = 1e-5 if f32 else 1e-13
    assert np.linalg.norm(rec - v) <= eps * np.linalg.norm(v)
    assert np.abs(Qg[:, i] - ref.Qk[:, 0]).max() <= (1e-3 if f32 else 1e-8)
