"""GPU parity of the ILU(0) right preconditioner (the preconditioner of the
paper's 2D Laplace test with an ILU preconditioner, Sec. 4.3) against the
oracle's ILU0 and its preconditioned solves.

- factors: the GPU factorisation (levels of the forward substitution, IKJ
  elimination on the pattern) against the oracle's L and U at every stored
  entry, on 2D and 3D stencils, a random nonsymmetric pattern whose rows
  hold more than eight entries on one side of the diagonal, and a matrix
  whose second level depends on rows more than 16384 positions back (the
  solve's global-memory path); the level counts against the closed forms
  2N - 1 (N x N grid) and 3N - 2 (N^3);
- M^{-1} r against the oracle's two triangular solves, also in place;
- invalid input: no stored diagonal, unsorted columns, a zero pivot;
- new values through sgm_matrix_update_values refactor;
- whole preconditioned solves against the oracle: identical block sizes,
  residual estimates within 1e-6 relative, x within 1e-8 relative;
- the full-size 400^2 Laplace case of Sec. 4.3 at the library's largest
  step size (256) against the oracle's stored solve.

Tolerances: the GPU contracts a_ij - l_ik u_kj into one fused multiply-add
and sums the substitutions in another order, so factors and M^{-1} r agree
to a few units of roundoff (1e-12 relative, the factors' growth is small on
these diagonally dominant matrices).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import sstep_gmres as o

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def csr(A):
    return o.csr_matrix(A.n, A.row_ptr, A.col, A.val)


class _Csr:
    def __init__(self, M):
        M = sp.csr_matrix(M)
        M.sort_indices()
        self.n = M.shape[0]
        self.row_ptr = M.indptr.astype(np.int32)
        self.col = M.indices.astype(np.int32)
        self.val = M.data.astype(np.float64)


def _random_pattern(n=3000, seed=11, per_row=24):
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=per_row / n, random_state=rng, format="csr")
    A = A - 0.5 * A.sign()
    d = np.asarray(abs(A).sum(axis=1)).ravel() + 1.0
    return (A + sp.diags(d)).tocsr()


def _two_levels(n=40000):
    """4 I with -1 couplings n/2 apart: two levels of n/2 rows each, so the
    second level depends on positions more than 16384 back (read from
    global memory, with the full barrier between levels)."""
    h = n // 2
    return sp.diags([-np.ones(h), 4.0 * np.ones(n), -np.ones(h)],
                    [-h, 0, h]).tocsr()


CASES = [
    ("laplace2d_40", lambda: csr(W.laplace_2d(40)), (79, 79)),
    ("two_levels_40000", _two_levels, (2, 2)),
    ("convdiff2d_33", lambda: csr(W.conv_diff_2d(33, 10.0)), (65, 65)),
    ("poisson3d_11", lambda: csr(W.poisson_3d(11)), (31, 31)),
    # levels of up to about 1200 rows: the 1024-thread solve
    ("poisson3d_40", lambda: csr(W.poisson_3d(40)), (118, 118)),
    ("random_3000", lambda: _random_pattern(), None),
]


@pytest.mark.parametrize("name,mk,levels", CASES, ids=[c[0] for c in CASES])
def test_ilu0_factors_and_apply_match_oracle(lib, name, mk, levels):
    M = mk()
    ref = o.ILU0(M)
    G = lib.Matrix.from_csr(_Csr(M))
    lv = G.ilu0()
    if levels is not None:
        assert tuple(lv) == levels
    else:
        assert lv[0] >= 2 and lv[1] >= 2
    if name == "random_3000":
        wl = max(np.diff(sp.tril(M, -1).tocsr().indptr))
        wu = max(np.diff(sp.triu(M, 1).tocsr().indptr))
        assert wl > 8 and wu > 8      # the levels' register fallback runs
    Ms = sp.csr_matrix(M)
    Ms.sort_indices()
    lu = G.ilu0_factors().cpu().numpy()
    F = sp.csr_matrix((lu, Ms.indices, Ms.indptr), shape=M.shape)
    Lr, Ur = sp.tril(ref.L, -1).tocsr(), ref.U.tocsr()
    scale = abs(Ms).max()
    assert abs(sp.tril(F, -1) - Lr).max() <= 1e-12 * max(1.0, abs(Lr).max())
    assert abs(sp.triu(F) - Ur).max() <= 1e-12 * scale
    r = np.random.default_rng(3).standard_normal(M.shape[0])
    z = G.ilu0_apply(r).cpu().numpy()
    zr = ref.solve(r)
    assert np.abs(z - zr).max() <= 1e-12 * np.abs(zr).max()
    import torch
    t = torch.tensor(r, device="cuda")
    G.ilu0_apply(t, out=t)                      # in place
    assert np.abs(t.cpu().numpy() - zr).max() <= 1e-12 * np.abs(zr).max()


def test_ilu0_rejects_invalid_input(lib):
    # no stored diagonal in row 1
    M = sp.csr_matrix(np.array([[2.0, 1.0, 0.0], [1.0, 0.0, 1.0],
                                [0.0, 1.0, 2.0]]))
    M.eliminate_zeros()
    G = lib.Matrix.from_csr(_Csr(M))
    with pytest.raises(lib.SgmError, match="diagonal"):
        G.ilu0()
    # unsorted columns
    A = _Csr(csr(W.laplace_2d(5)))
    A.col = A.col.copy()
    A.col[[0, 1]] = A.col[[1, 0]]
    A.val = A.val.copy()
    A.val[[0, 1]] = A.val[[1, 0]]
    G2 = lib.Matrix.from_csr(A)
    with pytest.raises(lib.SgmError, match="sorted"):
        G2.ilu0()
    # a zero pivot: u_11 = 1 - 1 * 1 = 0
    Z = sp.csr_matrix(np.array([[1.0, 1.0], [1.0, 1.0]]))
    G3 = lib.Matrix.from_csr(_Csr(Z))
    with pytest.raises(lib.SgmError, match="pivot"):
        G3.ilu0()
    # a solve asking for ILU(0) on float32 inner cycles is refused
    G4 = lib.Matrix.from_csr(W.laplace_2d(8))
    with pytest.raises(lib.SgmError, match="float64"):
        lib.solve(G4, W.rhs(64, 1), precond="ilu0", precision="fp32_ir")


def test_ilu0_follows_update_values(lib):
    A = W.conv_diff_2d(20, 5.0)
    G = lib.Matrix.from_csr(A)
    G.ilu0()
    rng = np.random.default_rng(4)
    v2 = A.val * (1.0 + 0.2 * rng.random(A.val.size))
    G.update_values(v2)
    M2 = o.csr_matrix(A.n, A.row_ptr, A.col, v2)
    ref = o.ILU0(M2)
    r = rng.standard_normal(A.n)
    z = G.ilu0_apply(r).cpu().numpy()
    zr = ref.solve(r)
    assert np.abs(z - zr).max() <= 1e-12 * np.abs(zr).max()


@pytest.mark.parametrize("mk,kw", [
    (lambda: W.conv_diff_2d(64, 10.0), dict(s_max=16, restart=64)),
    (lambda: W.poisson_3d(27), dict(s_max=16, restart=48)),
    (lambda: W.laplace_2d(60), dict(s_max=32, restart=96, ritz_reuse=False)),
    (lambda: W.conv_diff_2d(48, 10.0),
     dict(s_max=16, restart=64, prephase="monomial"))],
    ids=["convdiff2d_64", "poisson3d_27", "laplace2d_60_separate_prephase",
         "convdiff2d_48_monomial_prephase"])
def test_ilu0_solve_matches_oracle(lib, mk, kw):
    A = mk()
    M = csr(A)
    b = W.rhs(A.n, 2)
    ref = o.solve(M, b, opts=o.Options(tol=1e-10, precond="ilu0", **kw))
    assert ref.status == "ok"
    G = lib.Matrix.from_csr(A)
    r = lib.solve(G, b, tol=1e-10, precond="ilu0", **kw)
    assert r.status == lib.OK
    assert list(r.s_hist) == list(ref.s_hist)
    h, hr = np.asarray(r.res_hist), np.asarray(ref.res_hist)
    assert h.shape == hr.shape
    assert np.all(np.abs(h - hr) <= 1e-6 * hr)
    x = r.x.cpu().numpy()
    assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
    assert np.linalg.norm(b - M @ x) / np.linalg.norm(b) <= 1e-10
    # fewer iterations than without the preconditioner
    r0 = lib.solve(G, b, tol=1e-10, **kw)
    assert r.info["iters"] < r0.info["iters"]


def test_laplace400_ilu0_full_size(lib):
    """Sec. 4.3's 2D Laplace 400^2 with right ILU(0) at s0 = 256 (the
    library's largest step; the paper's 400 is pinned on the oracle),
    separate 256-step pre-phase, no estimator, Omega = 1e7, m = 400,
    tol 1e-8: against the oracle's stored solve
    (tests/golden/make_laplace2d_400_ilu0_oracle.py)."""
    g = np.load(os.path.join(GOLD, "laplace2d_400_ilu0_oracle.npz"))
    A = W.laplace_2d(400)
    b = W.rhs(A.n, 1)
    G = lib.Matrix.from_csr(A)
    assert tuple(G.ilu0()) == (799, 799)
    r = lib.solve(G, b, s_max=256, restart=400, max_restarts=0, tol=1e-8,
                  omega=1e7, use_estimator=False, ritz_reuse=False,
                  precond="ilu0")
    assert r.status == lib.OK
    assert list(r.s_hist) == list(g["s_hist"])
    assert r.info["iters"] == int(g["iters"])
    h, hr = np.asarray(r.res_hist), g["res_hist"]
    assert h.shape == hr.shape and np.all(np.abs(h - hr) <= 1e-6 * hr)
    x = r.x.cpu().numpy()
    xs = g["x_samples"]
    assert (np.linalg.norm(x[g["sample_idx"]] - xs)
            <= 1e-8 * np.linalg.norm(xs))
    M = csr(A)
    assert np.linalg.norm(b - M @ x) / np.linalg.norm(b) <= 1e-8
