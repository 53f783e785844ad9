"""GPU parity of the float32 inner path, step by step, against the
oracle's float32 model (the mixed-precision variant: basis vectors, SpMV and
tall-skinny products in float32, every small matrix in float64).

- the classical BCGS2 block (Alg. 4, both partial CholQR passes taking
  their Gram matrix from the updated block) at the block shapes of the
  solver: one to 200 new columns after 1 to 129 prior ones, full-rank and
  truncating;
- the matrix powers kernel with a complex conjugate pair (Eq.
  (newtonrecurrence) with the pair recurrence);
- one float32 inner cycle of the refinement loop: block sizes identical,
  Givens residual estimates within 1e-4 relative.

Tolerances are float32-scaled: the two sides sum in different orders, so
basis entries differ by O(sqrt(n) u32) and R entries by O(u32) relative;
accepted block sizes are compared exactly where the condition estimates at
the cut lie well away from Omega = 409.6 (checked in the test).
"""
import numpy as np
import pytest

import workloads as W
from oracle import sstep_gmres as o

pytestmark = pytest.mark.gpu

OM32 = o.default_omega(o.U32)


def csr(A):
    return o.csr_matrix(A.n, A.row_ptr, A.col, A.val)


def flat_cols(torch, M, ld, dtype):
    n, k = M.shape
    buf = np.zeros((k, ld), dtype=dtype)
    buf[:, :n] = M.T
    return torch.tensor(buf.ravel(), device="cuda")


def cols_of(t, n, ld, k):
    return t.cpu().numpy().reshape(k, ld)[:, :n].T


def _run_fp32_block(lib, Qi, V):
    import torch
    n, i = Qi.shape
    s = V.shape[1]
    ld = ((n + 63) // 64) * 64
    Qi32, V32 = Qi.astype(np.float32), V.astype(np.float32)
    ref = o.block_orth(np.asfortranarray(Qi32.copy()), i, V32.copy(), OM32,
                       work_dtype=np.float32)
    Qd = flat_cols(torch, np.concatenate([Qi32, V32], 1), ld, np.float32)
    p, Rt, Rk = lib.block_orth(Qd, n, ld, i, s, omega=OM32,
                               precision="fp32_ir")
    Qg = cols_of(Qd, n, ld, i + s).astype(np.float64)
    return p, Rt, Rk, Qg, ref


def _random_block(n, i, s, seed):
    rng = np.random.default_rng(seed)
    Qi, _ = np.linalg.qr(rng.standard_normal((n, i)))
    V = Qi @ rng.standard_normal((i, s)) + rng.standard_normal((n, s))
    return Qi, V


@pytest.mark.parametrize("i,s", [(1, 8), (33, 32), (97, 32), (129, 128),
                                 (7, 200), (201, 200)])
def test_block_orth_classical_fp32(lib, i, s):
    """Full-rank blocks (kappa about 1.4): p = s on both sides; the new
    basis vectors, R(1:i, k) and R(k, k) agree to float32 accuracy.
    (201, 200) updates in column groups (its 201 x 200 coefficient matrix
    does not fit in LDS whole) and forms its Gram with the LDS-shared
    kernel."""
    n = 9001   # ragged last panel
    Qi, V = _random_block(n, i, s, seed=500 + i + s)
    p, Rt, Rk, Qg, ref = _run_fp32_block(lib, Qi, V)
    assert p == ref.p == s
    assert np.abs(Qg[:, i:i + p] - ref.Qk).max() <= 2e-5
    assert np.abs(Rt[:, :p] - ref.R_top).max() <= 1e-5 * np.abs(ref.R_top).max()
    assert (np.abs(np.triu(Rk[:p, :p]) - ref.R_kk).max()
            <= 1e-5 * np.abs(ref.R_kk).max())
    assert o.loo(Qg[:, :i + p]) <= 1e-4


@pytest.mark.parametrize("i,s", [(9, 16), (33, 32)])
def test_block_orth_classical_fp32_truncating(lib, i, s):
    """A float32 scaled Newton Krylov block with 8 shifts reused
    cyclically: the float32 condition bound 409.6 cuts it (p < s) at the
    same column on both sides."""
    A = W.conv_diff_2d(64, 10.0)
    M = csr(A)
    b = W.rhs(A.n, 2)
    r = o.solve(M, b, opts=o.Options(s_max=8, restart=i - 1, max_restarts=0,
                                     tol=1e-300, record=True))
    Qi = r.trace["Q_first_cycle"][:, :i]
    eng = o._Engine(M, o.Options(work_dtype=np.float32))
    V = eng.mpk(Qi[:, i - 1].astype(np.float32), r.shifts, s)
    p, Rt, Rk, Qg, ref = _run_fp32_block(lib, Qi, V.astype(np.float64))
    # the cut is decided away from the bound: the two sides' float32 Gram
    # matrices differ by O(sqrt(s) u32) relative, which moves these
    # condition estimates by far less than the 2% margin
    k1 = ref.kappas1
    assert ref.p1 < s and k1[ref.p1] > 1.02 * OM32
    assert k1[ref.p1 - 1] < OM32 / 1.02
    assert p == ref.p and 1 <= p < s
    assert np.abs(Qg[:, i:i + p] - ref.Qk).max() <= 1e-4
    assert np.abs(Rt[:, :p] - ref.R_top).max() <= 1e-4 * np.abs(ref.R_top).max()
    assert o.loo(Qg[:, :i + p]) <= 1e-4


def test_mpk_fp32_with_complex_pair(lib):
    """Float32 matrix powers kernel: scaled Newton records with two complex
    conjugate pairs, against the oracle's float32 recurrence."""
    import torch
    A = W.conv_diff_2d(40, 10.0)
    M = csr(A)
    n, ld, s = A.n, ((A.n + 63) // 64) * 64, 9
    rng = np.random.default_rng(1)
    q = rng.standard_normal(n)
    q = (q / np.linalg.norm(q)).astype(np.float32)
    ritz = np.array([7.5, 2.0 + 1.0j, 2.0 - 1.0j, 0.5, 5.0, 3.0 + 0.25j,
                     3.0 - 0.25j, 1.0, 6.0])
    sh = o.newton_shifts(o.leja_order(ritz), scaled=True)
    assert np.count_nonzero(sh.delta) == 2
    eng = o._Engine(M, o.Options(work_dtype=np.float32))
    V = eng.mpk(q, sh, s).astype(np.float64)
    rec = np.stack([sh.theta, sh.gamma, sh.delta], 1)
    Q0 = np.zeros((n, s + 1), dtype=np.float32)
    Q0[:, 0] = q
    Qd = flat_cols(torch, Q0, ld, np.float32)
    lib.mpk(lib.Matrix.from_csr(A), Qd, ld, 0, s, rec, precision="fp32_ir")
    Vg = cols_of(Qd, n, ld, s + 1)[:, 1:].astype(np.float64)
    for j in range(s):
        err = np.linalg.norm(Vg[:, j] - V[:, j]) / np.linalg.norm(V[:, j])
        assert err <= 2e-6 * (j + 1), (j, err)


@pytest.mark.parametrize("mk,kw", [
    (lambda: W.poisson_3d(27), dict(s_max=16, restart=48)),
    # the 4096^2 workload's family at 64^2: blocks truncated by the float32
    # condition bound after a 64-column pre-phase
    (lambda: W.aniso_diffusion_2d(64), dict(s_max=64, restart=400))],
    ids=["poisson3d_27", "aniso2d_64"])
def test_fp32_inner_cycle_matches_oracle(lib, mk, kw):
    """One float32 inner cycle (max_outer = 1) against the first cycle of the
    oracle's refinement: the same block sizes (pre-phase steps and
    blocks), Givens estimates within 1e-4 relative, and the refined iterate
    within 1e-4 relative."""
    A = mk()
    M = csr(A)
    b = W.rhs(A.n, 3)
    ir = o.solve_ir(M, b, opts=o.Options(tol=1e-10, **kw), inner_tol=1e-6,
                    max_outer=1)
    rel, s_ref, res_ref = ir.inner[0]
    assert rel == 1.0 and max(s_ref) > 1
    G = lib.Matrix.from_csr(A)
    gpu = lib.solve(G, b, tol=1e-10, precision="fp32_ir", inner_tol=1e-6,
                    max_outer=1, **kw)
    assert gpu.info["outer_iters"] == 1
    assert list(gpu.s_hist) == s_ref
    h, hr = np.asarray(gpu.res_hist), np.asarray(res_ref)
    assert h.shape == hr.shape
    assert np.all(np.abs(h - hr) <= 1e-4 * hr)
    x = gpu.x.cpu().numpy()
    assert np.linalg.norm(x - ir.x) <= 1e-4 * np.linalg.norm(ir.x)
