"""GPU parity of the Pythagorean BCGS2 variant (orth="bcgs2_pyth") against
the oracle's block_orth(pythagorean=True) and solve(orth="bcgs2_pyth").

Block shapes reach every kernel path of the variant's second pass, in
float64 and float32:
- up to 64 new columns: the triangular solve with the Gram of its result
  in the same pass, then the projection; beyond 64, the triangular solve,
  then [Q Q_1]^T Q_1 as one wider product;
- the fused update + triangular solve for 1..4 column tiles, and the
  two-pass fallback beyond 64 columns;
- a truncating Krylov block (p < s) and a block almost inside span(Q),
  where the second pass has real work to do.
"""
import numpy as np
import pytest

import workloads as W
from oracle import sstep_gmres as o

pytestmark = pytest.mark.gpu


def csr(A):
    return o.csr_matrix(A.n, A.row_ptr, A.col, A.val)


def flat_cols(torch, M, ld, dtype):
    n, k = M.shape
    buf = np.zeros((k, ld), dtype=dtype)
    buf[:, :n] = M.T
    return torch.tensor(buf.ravel(), device="cuda")


def cols_of(t, n, ld, k):
    return t.cpu().numpy().reshape(k, ld)[:, :n].T


def _run_block(lib, Qi, V, precision="fp64", omega=None):
    import torch
    n, i = Qi.shape
    s = V.shape[1]
    ld = ((n + 63) // 64) * 64
    f32 = precision == "fp32_ir"
    wd = np.float32 if f32 else np.float64
    om = o.default_omega(o.U32 if f32 else o.U64) if omega is None else omega
    Qi_w = Qi.astype(wd)
    V_w = V.astype(wd)
    ref = o.block_orth(np.asfortranarray(Qi_w.copy()), i, V_w.copy(), om,
                       work_dtype=wd, pythagorean=True)
    Qd = flat_cols(torch, np.concatenate([Qi_w, V_w], 1), ld, wd)
    p, Rt, Rk = lib.block_orth(Qd, n, ld, i, s, omega=om, precision=precision,
                               orth="bcgs2_pyth")
    Qg = cols_of(Qd, n, ld, i + s).astype(np.float64)
    return p, Rt, Rk, Qg, ref


def _random_block(n, i, s, seed, delta=1.0):
    rng = np.random.default_rng(seed)
    Qi, _ = np.linalg.qr(rng.standard_normal((n, i)))
    V = Qi @ rng.standard_normal((i, s)) + delta * rng.standard_normal((n, s))
    return Qi, V


@pytest.mark.parametrize("i,s", [(1, 2), (1, 16), (33, 32), (64, 17),
                                 (65, 32), (97, 48), (40, 64), (7, 100),
                                 (129, 128)])
def test_block_orth_pyth_fp64(lib, i, s):
    n = 21 ** 3  # 9261: ragged last panel
    Qi, V = _random_block(n, i, s, seed=300 + i + s)
    p, Rt, Rk, Qg, ref = _run_block(lib, Qi, V)
    assert p == ref.p == s
    assert np.abs(Qg[:, i:i + p] - ref.Qk).max() <= 1e-10
    assert np.abs(Rt[:, :p] - ref.R_top).max() <= 1e-10 * np.abs(ref.R_top).max()
    assert (np.abs(np.triu(Rk[:p, :p]) - ref.R_kk).max()
            <= 1e-10 * np.abs(ref.R_kk).max())
    assert o.loo(Qg[:, :i + p]) <= 1e-12


@pytest.mark.parametrize("i,s", [(1, 8), (33, 32), (97, 32), (20, 80)])
def test_block_orth_pyth_fp32(lib, i, s):
    n = 9001
    Qi, V = _random_block(n, i, s, seed=400 + i + s)
    p, Rt, Rk, Qg, ref = _run_block(lib, Qi, V, precision="fp32_ir")
    assert p == ref.p == s
    assert np.abs(Qg[:, i:i + p] - ref.Qk).max() <= 2e-5
    assert np.abs(Rt[:, :p] - ref.R_top).max() <= 1e-5 * np.abs(ref.R_top).max()
    assert o.loo(Qg[:, :i + p]) <= 1e-4


def test_block_orth_pyth_near_span(lib):
    """V = Q_i C + 1e-12 N: the first pass leaves R2 ~ 1e-4, the
    Pythagorean Gram's R2^T R2 term is what keeps the result orthonormal."""
    Qi, V = _random_block(3000, 20, 12, seed=11, delta=1e-12)
    p, Rt, Rk, Qg, ref = _run_block(lib, Qi, V)
    assert p == ref.p == 12
    assert o.loo(Qg[:, :32]) <= 1e-12
    rec = Qi @ Rt[:, :p] + Qg[:, 20:32] @ np.triu(Rk[:p, :p])
    assert np.linalg.norm(rec - V) <= 1e-13 * np.linalg.norm(V)
    # the direction of the tiny residual is fixed to u * kappa ~ 1e-4 only
    assert np.abs(Qg[:, 20:32] - ref.Qk).max() <= 1e-3


@pytest.mark.parametrize("s", [32, 128])
def test_block_orth_pyth_truncating_krylov(lib, s):
    """A scaled Newton block with 8 shifts reused cyclically: partial
    CholQR keeps p < s columns, as the oracle does."""
    A = W.conv_diff_2d(64, 10.0)
    M = csr(A)
    b = W.rhs(A.n, 2)
    i = 33
    r = o.solve(M, b, opts=o.Options(s_max=8, restart=i - 1, max_restarts=0,
                                     tol=1e-300, record=True))
    Qi = r.trace["Q_first_cycle"][:, :i]
    V = o._Engine(M, o.Options()).mpk(Qi[:, i - 1], r.shifts, s)
    p, Rt, Rk, Qg, ref = _run_block(lib, Qi, V)
    assert p == ref.p and 1 <= p < s
    assert np.abs(Qg[:, i:i + p] - ref.Qk).max() <= 1e-9
    assert o.loo(Qg[:, :i + p]) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_solve_pyth_matches_oracle(lib, precision):
    """Whole solves with the variant: the same blocks as the oracle's model
    of it, residual history and solution to the usual tolerances, and the
    same solution as the paper's BCGS2."""
    A = W.poisson_3d(27)
    M = csr(A)
    b = W.rhs(A.n, 3)
    kw = dict(s_max=16, restart=48, tol=1e-10)
    G = lib.Matrix.from_csr(A)
    if precision == "fp64":
        ref = o.solve(M, b, opts=o.Options(max_restarts=50, orth="bcgs2_pyth",
                                           **kw))
        gpu = lib.solve(G, b, max_restarts=50, orth="bcgs2_pyth", **kw)
        assert gpu.status == lib.OK and ref.status == "ok"
        assert list(gpu.s_hist) == ref.s_hist
        h, hr = np.array(gpu.res_hist), np.array(ref.res_hist)
        assert h.size == hr.size
        assert np.all(np.abs(h - hr) <= 1e-6 * hr + 1e-13)
        x = gpu.x.cpu().numpy()
        assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
    else:
        ir = o.solve_ir(M, b, opts=o.Options(orth="bcgs2_pyth", **kw),
                        inner_tol=1e-6, max_outer=50)
        gpu = lib.solve(G, b, precision="fp32_ir", inner_tol=1e-6,
                        max_outer=50, orth="bcgs2_pyth", **kw)
        assert gpu.status == lib.OK and ir.status == "ok"
        assert abs(gpu.info["outer_iters"] - ir.outer) <= 1
        x = gpu.x.cpu().numpy()
        assert np.linalg.norm(b - M @ x) <= 1e-10 * np.linalg.norm(b)
    base = lib.solve(G, b, max_restarts=50, **kw)
    xb = base.x.cpu().numpy()
    assert np.linalg.norm(gpu.x.cpu().numpy() - xb) <= 1e-8 * np.linalg.norm(xb)


def test_solve_pyth_large_block_given_shifts(lib):
    """s_max 128 with 128 given Ritz values: the first block's second pass
    runs the two-pass fallback (more than 64 columns) and truncates."""
    A = W.conv_diff_2d(64, 10.0)
    M = csr(A)
    b = W.rhs(A.n, 1)
    r0 = o.solve(M, b, opts=o.Options(s_max=1, restart=128, max_restarts=0,
                                      tol=1e-300, basis="monomial",
                                      record=True))
    ritz = np.linalg.eigvals(r0.trace["H_first_cycle"][:128, :128])
    kw = dict(s_max=128, restart=256, tol=1e-10, shifts=ritz,
              use_estimator=False, orth="bcgs2_pyth")
    ref = o.solve(M, b, opts=o.Options(max_restarts=20, **kw))
    gpu = lib.solve(lib.Matrix.from_csr(A), b, max_restarts=20, **kw)
    assert gpu.status == lib.OK and ref.status == "ok"
    assert list(gpu.s_hist) == ref.s_hist and ref.s_hist[0] > 64
    x = gpu.x.cpu().numpy()
    assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
