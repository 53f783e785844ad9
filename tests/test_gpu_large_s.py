"""GPU parity at large block sizes (s = 64 .. 256) against the CPU oracle.

These are the code paths the 192^3 (s <= 128) and 4096^2 (s <= 200)
workloads take: wide tall-skinny kernels (up to 16 column tiles), the
partial Cholesky and block tail with their working sets in global scratch,
long matrix powers runs with cyclically reused shifts.  The matrices are
small enough for the oracle to finish in seconds; n is not a multiple of
64 where the generator allows it.
"""
import numpy as np
import pytest

import workloads as W
from oracle import sstep_gmres as o

pytestmark = pytest.mark.gpu


def csr(A):
    return o.csr_matrix(A.n, A.row_ptr, A.col, A.val)


def flat_cols(torch, M, ld):
    n, k = M.shape
    buf = np.zeros((k, ld), dtype=M.dtype)
    buf[:, :n] = M.T
    return torch.tensor(buf.ravel(), device="cuda")


def cols_of(t, n, ld, k):
    return t.cpu().numpy().reshape(k, ld)[:, :n].T


def _sensitivity(Qi, V, om, ref, trials=3):
    """How far the oracle's own Q_k, R_top and R_kk move when V is perturbed
    by one unit roundoff (relative, random): the rounding-level spread a
    different summation order may show.  None if the accepted size moves."""
    rng = np.random.default_rng(11)
    dq = dt = dk = 0.0
    for _ in range(trials):
        Vp = V * (1 + 2.0 ** -53 * rng.standard_normal(V.shape))
        rp = o.block_orth(np.asfortranarray(Qi.copy()), Qi.shape[1], Vp, om)
        if rp.p != ref.p:
            return None
        dq = max(dq, np.abs(rp.Qk - ref.Qk).max())
        dt = max(dt, np.abs(rp.R_top - ref.R_top).max())
        dk = max(dk, np.abs(rp.R_kk - ref.R_kk).max())
    return dq, dt, dk


def _check_block(lib, Qi, V, omega=None, spread=None):
    """block_orth on [Qi, V] (GPU, in place) against the oracle.  With
    spread = (dq, dt, dk) from _sensitivity, Q_k and R may differ by up to
    100x the oracle's own response to a one-roundoff perturbation of V (for
    ill-conditioned blocks, where rounding alone moves the last columns);
    the accepted size and the orthogonality are checked exactly as always."""
    import torch
    n, i = Qi.shape
    s = V.shape[1]
    ld = ((n + 63) // 64) * 64
    om = o.default_omega(o.U64) if omega is None else omega
    ref = o.block_orth(np.asfortranarray(Qi.copy()), i, V.copy(), om)
    Qd = flat_cols(torch, np.concatenate([Qi, V], 1), ld)
    p, Rt, Rk = lib.block_orth(Qd, n, ld, i, s, omega=om)
    assert p == ref.p, (p, ref.p)
    Qg = cols_of(Qd, n, ld, i + s)
    dq, dt, dk = spread if spread is not None else (0.0, 0.0, 0.0)
    if p > 0:
        assert np.abs(Qg[:, i:i + p] - ref.Qk).max() <= max(1e-9, 100 * dq)
        assert (np.abs(Rt[:, :p] - ref.R_top).max()
                <= max(1e-9 * max(1.0, np.abs(ref.R_top).max()), 100 * dt))
        assert (np.abs(np.triu(Rk[:p, :p]) - ref.R_kk).max()
                <= max(1e-9 * np.abs(ref.R_kk).max(), 100 * dk))
        assert o.loo(Qg[:, :i + p]) <= 1e-12
    return p, ref


@pytest.mark.parametrize("i,s", [(1, 64), (40, 100), (129, 128), (7, 200),
                                 (64, 256), (150, 100), (200, 200),
                                 (208, 113)])
def test_block_orth_wide_full_rank(lib, i, s):
    """A well-conditioned block: every column is accepted (p = s), so every
    column tile of the update, triangular solve and Gram products is live.
    (129, 128) runs the LDS-shared projection kernel on one 144 x 128
    output block; (150, 100), (200, 200) and (208, 113) the kernel that
    holds all 145 to 208 rows per workgroup, on one, two and two (7 + 1
    column tiles) blocks."""
    rng = np.random.default_rng(100 + s)
    n = 21 ** 3   # 9261, ragged
    Qi, _ = np.linalg.qr(rng.standard_normal((n, i)))
    V = rng.standard_normal((n, s)) + 0.1 * (Qi @ rng.standard_normal((i, s)))
    p, _ = _check_block(lib, Qi, V)
    assert p == s


@pytest.mark.parametrize("i,s", [(33, 128), (33, 200), (129, 128),
                                 (129, 200)])
def test_block_orth_wide_krylov_truncates(lib, i, s):
    """A long scaled Newton MPK block with the 8 shifts of a short pre-phase
    reused cyclically: the basis becomes ill-conditioned and partial
    CholQR truncates it; the GPU keeps the same number of columns.  With
    129 prior columns the second projection runs the LDS-shared kernel
    with its output columns masked to the first pass's accepted count."""
    A = W.conv_diff_2d(64, 10.0)
    M = csr(A)
    b = W.rhs(A.n, 2)
    r = o.solve(M, b, opts=o.Options(s_max=8, restart=i - 1, max_restarts=0,
                                     tol=1e-300, record=True))
    Qi = r.trace["Q_first_cycle"][:, :i]
    V = o._Engine(M, o.Options()).mpk(Qi[:, i - 1], r.shifts, s)
    assert np.all(np.isfinite(V))
    om = o.default_omega(o.U64)
    ref0 = o.block_orth(np.asfortranarray(Qi.copy()), i, V.copy(), om)
    spread = _sensitivity(Qi, V, om, ref0)
    assert spread is not None   # the accepted size is not on a knife edge
    p, ref = _check_block(lib, Qi, V, spread=spread)
    assert 1 <= p < s


def _ritz(M, b, m0):
    r0 = o.solve(M, b, opts=o.Options(s_max=1, restart=m0, max_restarts=0,
                                      tol=1e-300, basis="monomial",
                                      record=True))
    return np.linalg.eigvals(r0.trace["H_first_cycle"][:m0, :m0])


@pytest.mark.parametrize("s_max,restart", [(128, 256), (200, 400)])
def test_solve_large_blocks_given_shifts(lib, s_max, restart):
    """128 Ritz values passed in: the first block runs s_max matrix powers
    steps and partial CholQR keeps 97 of them, so the block tail works on a
    97-column block out of global scratch.  Same blocks, residual history
    and solution as the oracle."""
    A = W.conv_diff_2d(64, 10.0)
    M = csr(A)
    b = W.rhs(A.n, 1)
    ritz = _ritz(M, b, 128)
    kw = dict(s_max=s_max, restart=restart, tol=1e-10, shifts=ritz,
              use_estimator=False)
    ref = o.solve(M, b, opts=o.Options(max_restarts=20, **kw))
    G = lib.Matrix.from_csr(A)
    gpu = lib.solve(G, b, max_restarts=20, **kw)
    assert gpu.status == lib.OK and ref.status == "ok"
    assert list(gpu.s_hist) == ref.s_hist
    assert ref.s_hist[0] > 64
    h, hr = np.array(gpu.res_hist), np.array(ref.res_hist)
    assert h.size == hr.size
    assert np.all(np.abs(h - hr) <= 1e-6 * hr + 1e-13)
    x = gpu.x.cpu().numpy()
    assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_solve_given_shifts_use_the_estimator(lib):
    """Given shifts stand in for the pre-phase: the estimator picks the
    initial step size from them on both sides."""
    A = W.conv_diff_2d(48, 10.0)
    M = csr(A)
    b = W.rhs(A.n, 4)
    ritz = _ritz(M, b, 64)
    kw = dict(s_max=128, restart=256, tol=1e-10, shifts=ritz)
    ref = o.solve(M, b, opts=o.Options(max_restarts=20, **kw))
    gpu = lib.solve(lib.Matrix.from_csr(A), b, max_restarts=20, **kw)
    assert 0 < ref.s0_est <= 64          # s0* never exceeds the shift count
    assert gpu.info["s0_est"] == ref.s0_est
    assert gpu.info["s_init"] == ref.s0_est
    assert ref.s_hist[0] <= ref.s0_est
    assert list(gpu.s_hist) == ref.s_hist


def aniso2d_kappa(nx, ratio=1e-3, angle_deg=30.0):
    """2-norm condition number of the 5-point anisotropic operator of
    workloads.aniso_diffusion_2d on an nx^2 Dirichlet grid, from its
    closed-form eigenvalues 2 Kxx (1 - cos a) + 2 Kyy (1 - cos b)."""
    a = np.radians(angle_deg)
    kxx = np.cos(a) ** 2 + ratio * np.sin(a) ** 2
    kyy = np.sin(a) ** 2 + ratio * np.cos(a) ** 2
    c1, cn = np.cos(np.pi / (nx + 1)), np.cos(nx * np.pi / (nx + 1))
    return (2 * (kxx + kyy) * (1 - cn)) / (2 * (kxx + kyy) * (1 - c1))


def test_solve_anisotropic_s200_one_cycle(lib):
    """The 4096^2 workload's shape at 64^2: 200 pre-phase steps, then the
    estimator's step size (200) with partial CholQR truncation, restart 400;
    one cycle, compared block by block with the oracle."""
    A = W.aniso_diffusion_2d(64)
    M = csr(A)
    b = W.rhs(A.n, 5)
    kw = dict(s_max=200, restart=400, tol=1e-10)
    ref = o.solve(M, b, opts=o.Options(max_restarts=0, **kw))
    gpu = lib.solve(lib.Matrix.from_csr(A), b, max_restarts=0, **kw)
    assert gpu.info["s0_est"] == ref.s0_est
    assert list(gpu.s_hist) == ref.s_hist
    assert max(ref.s_hist) > 100
    h, hr = np.array(gpu.res_hist), np.array(ref.res_hist)
    assert np.all(np.abs(h - hr) <= 1e-6 * hr + 1e-13)
    x = gpu.x.cpu().numpy()
    assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_fp32_ir_anisotropic_s200(lib):
    """Float32 inner cycles (s up to 200, restart 400) inside float64
    refinement reach 1e-10 on the anisotropic problem; the outer step count
    matches the float32 oracle model within one and the solution matches
    the float64 oracle."""
    A = W.aniso_diffusion_2d(64)
    M = csr(A)
    b = W.rhs(A.n, 5)
    kw = dict(s_max=200, restart=400, tol=1e-10)
    ref = o.solve(M, b, opts=o.Options(max_restarts=50, **kw))
    ir = o.solve_ir(M, b, opts=o.Options(**kw), inner_tol=1e-6, max_outer=50)
    gpu = lib.solve(lib.Matrix.from_csr(A), b, precision="fp32_ir",
                    inner_tol=1e-6, max_outer=50, **kw)
    x = gpu.x.cpu().numpy()
    assert gpu.status == lib.OK and ir.status == "ok"
    assert np.linalg.norm(b - M @ x) <= 1e-10 * np.linalg.norm(b)
    assert abs(gpu.info["outer_iters"] - ir.outer) <= 1
    # both iterates have true residuals <= 1e-10, so each lies within
    # kappa(A) times its residual of the exact solution (kappa from the
    # closed-form eigenvalues of the 5-point operator, 1.7e3)
    true = np.linalg.norm(b - M @ x) / np.linalg.norm(b)
    bound = aniso2d_kappa(64) * (true + ref.rel_res_true)
    assert np.linalg.norm(x - ref.x) <= bound * np.linalg.norm(ref.x)
