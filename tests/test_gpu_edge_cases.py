"""GPU edge cases against the CPU oracle: degenerate sizes and right-hand
sides, the smallest and largest block and restart settings, tolerances
that cannot be met, and rejected options."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import sstep_gmres as o

pytestmark = pytest.mark.gpu


class Csr:
    def __init__(self, A):
        A = A.tocsr()
        A.sort_indices()
        self.n = A.shape[0]
        self.row_ptr = A.indptr.astype(np.int32)
        self.col = A.indices.astype(np.int32)
        self.val = A.data.astype(np.float64)
        self.nnz = A.nnz


def small_random(n, seed=3):
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=0.1, random_state=rng, format="csr")
    return (A + sp.eye(n) * 4).tocsr(), rng.standard_normal(n)


def gpu_solve(lib, A, b, x0=None, **kw):
    return lib.solve(lib.Matrix.from_csr(Csr(A)), b, x0=x0, **kw)


def test_one_by_one_system(lib):
    A = sp.csr_matrix([[2.0]])
    r = gpu_solve(lib, A, np.array([4.0]), s_max=8, restart=8, tol=1e-12)
    assert r.status == lib.OK
    assert r.x.cpu().numpy()[0] == 2.0


def test_smaller_than_one_slice(lib):
    """n = 63: a single, partly filled 64-row slice and panel."""
    A, b = small_random(63)
    kw = dict(s_max=8, restart=16, tol=1e-12, max_restarts=50)
    ref = o.solve(A, b, opts=o.Options(**kw))
    r = gpu_solve(lib, A, b, **kw)
    assert r.status == lib.OK and ref.status == "ok"
    assert list(r.s_hist) == ref.s_hist
    assert np.linalg.norm(r.x.cpu().numpy() - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


def test_zero_rhs_and_exact_start(lib):
    """b = 0 returns x = 0 at once.  An exact x0 leaves a residual at
    rounding level; the tolerance is relative to it (Sec. 4), so the solve
    runs to its restart cap and must keep x at the solution."""
    A, b = small_random(200)
    r = gpu_solve(lib, A, np.zeros(200), s_max=8, restart=16, tol=1e-12)
    assert r.status == lib.OK and r.info["iters"] == 0
    assert np.all(r.x.cpu().numpy() == 0.0)
    xs = np.linalg.solve(A.toarray(), b)
    r = gpu_solve(lib, A, b, x0=xs, s_max=8, restart=16, tol=1e-12,
                  max_restarts=2)
    assert r.status in (lib.OK, lib.NOT_CONVERGED)
    assert np.linalg.norm(r.x.cpu().numpy() - xs) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("s_max,restart", [(1, 1), (16, 8)])
def test_smallest_blocks_and_short_restarts(lib, s_max, restart):
    """GMRES(1), and a restart length below s_max (the pre-phase and the
    blocks are cut at m)."""
    A, b = small_random(300, seed=5)
    kw = dict(s_max=s_max, restart=restart, tol=1e-10, max_restarts=500)
    ref = o.solve(A, b, opts=o.Options(**kw))
    r = gpu_solve(lib, A, b, **kw)
    assert r.status == lib.OK and ref.status == "ok"
    assert abs(r.info["iters"] - ref.iters) <= s_max
    assert np.linalg.norm(r.x.cpu().numpy() - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_unreachable_tolerance(lib):
    """tol = 1e-18 cannot be met in float64: the restart cap ends the solve
    with SGM_NOT_CONVERGED and the last iterate, as accurate as the
    oracle's."""
    A, b = small_random(300, seed=6)
    kw = dict(s_max=8, restart=16, tol=1e-18, max_restarts=3)
    ref = o.solve(A, b, opts=o.Options(**kw))
    r = gpu_solve(lib, A, b, **kw)
    assert r.status == lib.NOT_CONVERGED and ref.status == "not_converged"
    assert r.info["restarts"] == 3 and r.info["iters"] == ref.iters
    assert list(r.s_hist) == ref.s_hist
    x = r.x.cpu().numpy()
    true, true_ref = (np.linalg.norm(b - A @ y) / np.linalg.norm(b)
                      for y in (x, ref.x))
    assert abs(true - true_ref) <= 1e-6 * true_ref
    assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


def test_largest_block(lib):
    """s_max = 256 (the largest allowed) with 256 given shifts: the first
    block keeps all 256 columns (partial Cholesky, block tail and the wide
    tall-skinny kernels at their largest), restart 512."""
    A = W.aniso_diffusion_2d(64)
    M = o.csr_matrix(A.n, A.row_ptr, A.col, A.val)
    b = W.rhs(A.n, 5)
    r0 = o.solve(M, b, opts=o.Options(s_max=1, restart=256, max_restarts=0,
                                      tol=1e-300, basis="monomial",
                                      record=True))
    ritz = np.linalg.eigvals(r0.trace["H_first_cycle"][:256, :256])
    kw = dict(s_max=256, restart=512, tol=1e-10, shifts=ritz,
              use_estimator=False, max_restarts=5)
    ref = o.solve(M, b, opts=o.Options(**kw))
    r = lib.solve(lib.Matrix.from_csr(A), b, **kw)
    assert r.status == lib.OK and ref.status == "ok"
    assert ref.s_hist[0] == 256
    assert list(r.s_hist) == ref.s_hist
    x = r.x.cpu().numpy()
    assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("bad", [dict(s_max=0), dict(s_max=257),
                                 dict(restart=0), dict(tol=0.0),
                                 dict(tol=-1.0), dict(prephase_s=0),
                                 dict(precision="fp32_ir", inner_tol=1.5)])
def test_invalid_options_rejected(lib, bad):
    A, b = small_random(100)
    kw = dict(s_max=8, restart=16, tol=1e-10)
    kw.update(bad)
    with pytest.raises(lib.SgmError) as e:
        gpu_solve(lib, A, b, **kw)
    assert e.value.status == lib.EINVAL


@pytest.mark.parametrize("shift", [2.5, 3.0])
def test_converges_inside_queued_prephase(lib, shift):
    """s_max 100: the column-wise pre-phase (100 steps) is queued in batches
    of 32 without per-step synchronisation, and the solve converges inside
    it (42 or 62 iterations, the second batch).  Iterations, residual
    history and solution match the oracle; the steps queued past
    convergence change nothing."""
    rng = np.random.default_rng(7)
    n = 3000
    A = sp.random(n, n, density=0.003, random_state=rng, format="csr")
    A = (A + sp.eye(n) * shift).tocsr()
    b = rng.standard_normal(n)
    kw = dict(s_max=100, restart=128, tol=1e-10, max_restarts=5)
    ref = o.solve(A, b, opts=o.Options(**kw))
    r = gpu_solve(lib, A, b, **kw)
    assert r.status == lib.OK and ref.status == "ok"
    assert 32 < ref.iters <= 64
    assert r.info["iters"] == ref.iters
    assert list(r.s_hist) == ref.s_hist
    h, hr = np.array(r.res_hist), np.array(ref.res_hist)
    assert np.all(np.abs(h - hr) <= 1e-6 * hr)
    x = r.x.cpu().numpy()
    assert np.linalg.norm(x - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("cap", [0, 5])
def test_short_history_buffers(lib, cap):
    """History buffers shorter than the histories: sgm_solve writes the
    first cap entries and reports the full lengths in info (n_hist,
    n_blocks); the solution is unaffected."""
    A = W.conv_diff_2d(64, 10.0)
    b = W.rhs(A.n, 1)
    G = lib.Matrix.from_csr(A)
    full = lib.solve(G, b, s_max=8, restart=64, tol=1e-10)
    short = lib.solve(G, b, s_max=8, restart=64, tol=1e-10, hist_cap=cap)
    assert full.info["n_hist"] == len(full.res_hist) > cap
    assert full.info["n_blocks"] == len(full.s_hist) > cap
    assert short.info["n_hist"] == full.info["n_hist"]
    assert short.info["n_blocks"] == full.info["n_blocks"]
    assert len(short.res_hist) == cap and len(short.s_hist) == cap
    assert np.array_equal(short.res_hist, full.res_hist[:cap])
    assert np.array_equal(short.s_hist, full.s_hist[:cap])
    assert np.array_equal(short.x.cpu().numpy(), full.x.cpu().numpy())


def test_solve_on_a_side_stream(lib):
    """All work is enqueued on the caller's stream: a solve under a
    non-default torch stream, whose right-hand side is produced on that
    stream just before the call, gives bitwise the default-stream result."""
    import torch
    A = W.conv_diff_2d(64, 10.0)
    b = W.rhs(A.n, 1)
    G = lib.Matrix.from_csr(A)
    ref = lib.solve(G, b, s_max=8, restart=64, tol=1e-10)
    bd = torch.tensor(b, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b2 = bd * 2.0
        b2.mul_(0.5)
        r = lib.solve(G, b2, s_max=8, restart=64, tol=1e-10)
        x = r.x.clone()
    side.synchronize()
    assert r.status == lib.OK
    assert np.array_equal(x.cpu().numpy(), ref.x.cpu().numpy())
    assert list(r.s_hist) == list(ref.s_hist)


def test_non_finite_matrix_ends_the_solve(lib):
    """A NaN in the matrix ends the solve with the numerical-breakdown
    status inside the first block, which (with the shifts given, no
    pre-phase) already has the next block's matrix powers steps queued
    behind it; they are gated off on the device and the call returns
    after them, so the same workspace then serves a clean solve that is
    bitwise a fresh one."""
    A = W.conv_diff_2d(64, 10.0)
    b = W.rhs(A.n, 1)
    shifts = np.linspace(0.2, 7.8, 8)
    kw = dict(s_max=8, restart=64, tol=1e-10, shifts=shifts,
              use_estimator=False)
    val = np.array(A.val, dtype=np.float64)
    val[val.size // 2] = np.nan
    ws = lib.Workspace()
    G = lib.Matrix(A.n, A.row_ptr, A.col, val)
    with pytest.raises(lib.SgmError) as e:
        lib.solve(G, b, workspace=ws, **kw)
    assert e.value.status == lib.ENUMERIC
    G.update_values(np.array(A.val, dtype=np.float64))
    r = lib.solve(G, b, workspace=ws, **kw)
    ref = lib.solve(lib.Matrix.from_csr(A), b, **kw)
    assert r.status == lib.OK and ref.status == lib.OK
    assert np.array_equal(r.x.cpu().numpy(), ref.x.cpu().numpy())
    assert list(r.s_hist) == list(ref.s_hist)
