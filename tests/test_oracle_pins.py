"""Pins of the CPU oracle against facts fixed independently of it.

Each test checks the oracle against something other than itself: the paper's
printed values for reproducible experiments (tests/golden), closed forms,
library routines on tiny inputs, brute force, the GMRES minimisation
property, or mathematical invariants.  Together they are chosen so that a
plausible slip anywhere in the oracle (a dropped term, a wrong sign or index,
a transposed operand) fails at least one of them; test_oracle_mutations.py
plants such slips and checks that they are caught.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import sstep_gmres as o

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def csr(A):
    return o.csr_matrix(A.n, A.row_ptr, A.col, A.val)


def small_nonsym(n=120, seed=0, shift=3.0):
    """Small well-conditioned nonsymmetric sparse test matrix."""
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=6.0 / n, random_state=rng, format="csr")
    A = A + sp.eye(n) * shift + sp.diags(rng.uniform(0.5, 1.5, n))
    return A.tocsr()


# ---------------------------------------------------------------- P1, P15, P2

@pytest.mark.parametrize("basis", ["monomial", "newton", "scaled_newton"])
def test_s1_equals_mgs_gmres(basis):
    """P1: with s = 1 the method is column-wise CGS2-GMRES (Sec. 3.3), whose
    iterates equal MGS-GMRES in exact arithmetic: residual estimates agree at
    every iteration and the final iterates agree."""
    A = small_nonsym(150, 1)
    b = np.random.default_rng(2).standard_normal(150)
    xm, hm, itm = o.mgs_gmres(A, b, restart=30, tol=1e-12, max_restarts=20)
    r = o.solve(A, b, opts=o.Options(s_max=1, restart=30, tol=1e-12,
                                     max_restarts=20, basis=basis))
    assert r.status == "ok"
    assert r.iters == itm
    h1, h2 = np.array(r.res_hist), np.array(hm)
    assert np.all(np.abs(h1 - h2) <= 1e-10 * np.maximum(h2, 1e-12) + 1e-15)
    assert np.linalg.norm(r.x - xm) <= 1e-10 * np.linalg.norm(xm)


@pytest.mark.parametrize("basis", ["monomial", "newton", "scaled_newton"])
@pytest.mark.parametrize("s", [2, 3, 5])
def test_sstep_iterates_are_gmres_minimisers(basis, s):
    """P15: every basis gives the GMRES iterate, i.e. the minimiser of
    ||b - A x|| over x0 + K_k(A, r0) (the methods are mathematically
    equivalent, Sec. 1).  Checked against that definition (Householder QR of
    the Krylov matrix + least squares) after k steps of one cycle."""
    n = 60
    A = small_nonsym(n, 3, shift=4.0)
    Ad = A.toarray()
    b = np.random.default_rng(4).standard_normal(n)
    x0 = np.random.default_rng(5).standard_normal(n) * 0.1
    for k in (6, 12, 17):
        r = o.solve(A, b, x0, o.Options(s_max=s, restart=k, max_restarts=0,
                                        tol=1e-300, basis=basis,
                                        use_estimator=False, ritz_reuse=True))
        xk = o.gmres_iterates_dense(Ad, b, x0, k)
        assert r.iters == k
        assert np.linalg.norm(r.x - xk) <= 1e-8 * np.linalg.norm(xk)


def test_dense_lu_solution():
    """P2: converged solution vs a dense LU solve, error within kappa*tol*10."""
    A = W.conv_diff_2d(16, 10.0)
    b = W.rhs(A.n, 1)
    r = o.solve(csr(A), b, opts=o.Options(s_max=8, restart=32, tol=1e-12))
    Ad = A.to_dense()
    x = np.linalg.solve(Ad, b)
    kap = np.linalg.cond(Ad)
    assert r.status == "ok"
    assert np.linalg.norm(r.x - x) / np.linalg.norm(x) <= kap * 1e-12 * 10
    assert r.rel_res_true <= 1e-12


# ---------------------------------------------------------------- P3 - P6

def _conv_diff_run(**kw):
    A = W.conv_diff_2d(32, 10.0)
    b = W.rhs(A.n, 1)
    opts = dict(s_max=8, restart=64, tol=1e-10, record=True)
    opts.update(kw)
    return A, b, o.solve(csr(A), b, opts=o.Options(**opts))


def test_residual_monotone_and_true_residual():
    """P3 + P6: the Givens estimates never increase inside a cycle (minimal
    residual property), the true residuals at restarts never increase, and
    at cycle ends the estimate matches the true residual."""
    A, b, r = _conv_diff_run(max_restarts=3, tol=1e-13)
    h = np.array(r.res_hist)
    m = 64
    for c0 in range(0, len(h), m):
        seg = h[c0:c0 + m]
        assert np.all(np.diff(seg) <= 1e-14 * seg[:-1] + 1e-300)
    tr = np.array(r.true_res_restarts)
    assert np.all(np.diff(tr) <= 1e-12)
    # cycle-end estimate vs true residual
    ends = [h[min(len(h), (c + 1) * m) - 1] for c in range(len(tr))]
    for e, t in zip(ends, tr):
        if t > 1e-11:
            assert abs(e - t) <= 1e-8 * t


def test_loss_of_orthogonality():
    """P4: ||I - Q^T Q||_F stays O(eps) for BCGS2 + partial CholQR (Sec. 4)."""
    for basis in ("scaled_newton", "newton", "monomial"):
        _, _, r = _conv_diff_run(basis=basis, max_restarts=0, tol=1e-300)
        assert o.loo(r.trace["Q_first_cycle"]) <= 1e-12


def test_arnoldi_relation_and_hessenberg_structure():
    """P5: the recovered H satisfies A Q_k = Q_{k+1} H and is upper
    Hessenberg (entries below the subdiagonal vanish to rounding)."""
    A, b, r = _conv_diff_run(max_restarts=0, tol=1e-300)
    H = r.trace["H_first_cycle"]
    Q = r.trace["Q_first_cycle"]
    k = H.shape[1]
    M = csr(A)
    res = np.linalg.norm(M @ Q[:, :k] - Q @ H)
    assert res / (sp.linalg.norm(M) * math.sqrt(k)) <= 1e-12
    low = np.tril(H, -2)
    assert np.abs(low).max() <= 1e-13 * np.abs(H).max()


def test_givens_least_squares_vs_lstsq():
    """P6: the Givens least-squares solution equals numpy lstsq on a random
    Hessenberg matrix, and |g_{k+1}| is the least-squares residual."""
    rng = np.random.default_rng(7)
    m = 25
    H = np.triu(rng.standard_normal((m + 1, m)), -1)
    gv = o.Givens(m, 2.5)
    for c in range(m):
        gv.add_column(c, H[:, c])
    y = gv.solve(m)
    rhs = np.zeros(m + 1)
    rhs[0] = 2.5
    yl, *_ = np.linalg.lstsq(H, rhs, rcond=None)
    assert np.allclose(y, yl, rtol=1e-11, atol=1e-13)
    assert abs(abs(gv.g[m]) - np.linalg.norm(rhs - H @ yl)) <= 1e-12


# ---------------------------------------------------------------- P7: paper

def test_E1_monomial_step_size_six():
    """P7a, Test 1 (Sec. 4.1): diagonal N=1e4, eigenvalues evenly spaced in
    (0.1, 10), monomial basis, s0 = 10, Omega = 1e7 => adapted s = 6 in every
    block; the ICE estimate tracks the SVD condition number."""
    g = golden("paper_stability_results.json")["E1"]
    A = W.diagonal(np.linspace(0.1, 10.0, 10000))
    for b in (np.ones(A.n), W.rhs(A.n, 1)):
        r = o.solve(csr(A), b, opts=o.Options(
            s_max=10, restart=100, max_restarts=0, tol=1e-300,
            basis="monomial", omega=1e7, record=True))
        # every block that the end of the cycle does not cut short keeps
        # s = 6: the first (s_eff = 10) and the ones after it (s_eff = 6,
        # since s never grows inside a cycle)
        full = [p for (_, i, se, _, p) in r.blocks if se >= g["adapted_s"]]
        assert len(full) >= 15
        assert all(p == g["adapted_s"] for p in full)
        kice = r.trace["first_block"]["kappas"]
        r2 = o.solve(csr(A), b, opts=o.Options(
            s_max=10, restart=12, max_restarts=0, tol=1e-300,
            basis="monomial", omega=1e7, record=True, cond="svd"))
        ksvd = r2.trace["first_block"]["kappas"]
        for a, c in zip(kice, ksvd):
            assert a <= c * (1 + 1e-8) and c <= 10 * a   # P9


@pytest.mark.slow
def test_E2_laplace_monomial_step_size_six():
    """P7b, Test 2: 2D Laplace 400^2, m = 100, monomial, s0 = 10 => every
    block of the first cycle that the end of the cycle does not cut short
    keeps s = 6 (one cycle is enough to see it; the paper runs 5 restarts).
    The paper does not give b; a seeded N(0,1) vector is used.  (b = ones
    is a poor stand-in: A 1 vanishes away from the boundary, which changes
    the first block.)"""
    g = golden("paper_stability_results.json")["E2"]
    A = W.laplace_2d(400)
    b = W.rhs(A.n, 1)
    m = 100
    r = o.solve(csr(A), b, opts=o.Options(
        s_max=10, restart=m, max_restarts=0, tol=1e-300, basis="monomial",
        omega=1e7))
    ps = [p for (_, i, _, _, p) in r.blocks if i + g["adapted_s"] <= m]
    assert len(ps) >= 15 and all(p == g["adapted_s"] for p in ps)


def test_E3_scaled_newton_single_block():
    """P7c, Test 3 (Sec. 4.2): same diagonal matrix, s0 = 100, scaled Newton
    => one block of s = 100, residuals agreeing with GMRES; Newton and
    monomial adapt to smaller sizes."""
    g = golden("paper_stability_results.json")["E3"]
    A = W.diagonal(np.linspace(0.1, 10.0, 10000))
    b = np.ones(A.n)
    M = csr(A)
    _, hm, _ = o.mgs_gmres(M, b, restart=100, tol=1e-300, max_restarts=0)
    res = {}
    for basis in ("scaled_newton", "newton", "monomial"):
        r = o.solve(M, b, opts=o.Options(
            s_max=100, restart=100, max_restarts=0, tol=1e-300, basis=basis,
            omega=1e7, use_estimator=False, ritz_reuse=False))
        res[basis] = r
        assert np.allclose(r.res_hist, hm, rtol=1e-6)
    assert res["scaled_newton"].s_hist == [g["adapted_s_scaled_newton"]]
    assert max(res["newton"].s_hist) < 100
    assert max(res["monomial"].s_hist) < max(res["newton"].s_hist)


def _ritz_from_arnoldi(lam, seed):
    n = lam.size
    A = sp.diags(lam).tocsr()
    v = np.random.default_rng(seed).standard_normal(n)
    r = o.solve(A, v, opts=o.Options(s_max=1, restart=n, max_restarts=0,
                                     tol=1e-300, basis="monomial", record=True))
    H = r.trace["H_first_cycle"]
    k = H.shape[1]
    return np.linalg.eigvals(H[:k, :k])


# The oracle's s0* on the two Test 8 spectra.  The paper prints 134 and 17
# (Sec. 4.4).  Eq. (auxiliarymatrix) taken as printed gives 137 and 16, and
# so do the alternative readings tried (epsilon only above the diagonal,
# epsilon = 2^-52 or 1e-16, the 1-, 2- or max-norm of column j, the norm
# relative to column 1, argmax over all j, Omega_est = 1e7 or
# 0.1 u^{-1/2}, every Leja tie rule): none gives both printed values, and
# the value 134 is not reached for any epsilon with this spectrum.  The
# paper's Ritz values came from its own Arnoldi run, which it does not
# give.  So this is "parity unpinned" against the paper; the adopted
# (literal) values are asserted exactly, here and on the GPU.
E8_ADOPTED = {"uniform_200": 137, "max_2000": 16}


def test_E8_estimator_prediction():
    """P7d, Test 8 (Sec. 4.4): diagonal N = 200, eigenvalues 1..200 (and the
    same with the largest raised to 2000), Omega_est = 1e7.  The estimator
    is unpinned against the paper's printed s0* (see E8_ADOPTED); what is
    pinned here is the rest of the experiment: Ritz values from an Arnoldi
    run equal the eigenvalues, s0* does not depend on which of them the
    run returns first, and the float64 scaled Newton basis' condition
    number crosses 1e8 where the paper says (j = 15 for the second
    matrix, within the spread of random start vectors)."""
    g = golden("paper_stability_results.json")["E8"]
    for case in ("uniform_200", "max_2000"):
        lam = np.arange(1.0, 201.0)
        if case == "max_2000":
            lam[-1] = 2000.0
        ritz = _ritz_from_arnoldi(lam, 11)
        assert np.abs(np.sort(ritz.real) - lam).max() <= 1e-8 * lam.max()
        sh = o.newton_shifts(o.leja_order(ritz), scaled=True)
        s0, _ = o.estimator(sh.ritz, sh.gamma, o.U64, 1e7)
        assert s0 == E8_ADOPTED[case], (case, s0)
        # the same from the exact eigenvalues in reversed input order
        sx = o.newton_shifts(o.leja_order(lam[::-1].astype(complex)),
                             scaled=True)
        assert o.estimator(sx.ritz, sx.gamma, o.U64, 1e7)[0] == s0
        if case == "max_2000":
            v = np.random.default_rng(12).standard_normal(200)
            v /= np.linalg.norm(v)
            V = [v]
            for j in range(40):
                th, ga, de = sh.record(j)
                V.append((lam * V[-1] - th * V[-1]) / ga)
            V = np.array(V).T
            cross = next(j for j in range(1, 41)
                         if np.linalg.cond(V[:, :j]) > 1e8)
            assert abs(cross - g[case]["kappa_1e8_at"]) <= 3


def test_estimator_matrix_small_closed_form():
    """The estimator matrix against Eq. (auxiliarymatrix) written out by hand
    for three shifts (no logarithms), and E^L bounded while E grows."""
    th = np.array([3.0, -1.0, 0.5])
    mean = th.mean()
    ga = np.abs(mean - th)
    eps = 1e-3
    f = lambda i, k: abs(th[i] - th[k]) / ga[k]
    # Rows i = 1, 2, 3 and columns j = 1, 2, 3 of Eq. (auxiliarymatrix):
    E = np.array([
        # i=1: j=1 -> eps;  j=2 -> eps (k=2..1 empty);  j=3 -> eps*f(1,2)
        [eps, eps, eps * f(0, 1)],
        # i=2: j=1 -> 1;  j=2 -> f(2,1)*eps;  j=3 -> f(2,1)*eps (k=3..2 empty)
        [1.0, f(1, 0) * eps, f(1, 0) * eps],
        # i=3: j=1 -> 1;  j=2 -> f(3,1);  j=3 -> f(3,1)*f(3,2)*eps
        [1.0, f(2, 0), f(2, 0) * f(2, 1) * eps],
    ])
    L = o.estimator_matrix_log(th.astype(complex), ga, eps)
    assert np.allclose(np.exp(L), E, rtol=1e-13)
    s0, lg = o.estimator(th.astype(complex), ga, eps, 10.0)
    nrm = np.linalg.norm(E, axis=0)
    assert np.allclose(10 ** lg, nrm, rtol=1e-12)
    first = next((j for j in range(3) if nrm[j] >= 10.0), 3)
    assert s0 == max(1, first)


# ---------------------------------------------------------------- P8

@pytest.mark.parametrize("k", [-3, 3])
def test_scaled_newton_scale_invariance(k):
    """P8 (Sec. 4.3, equilibration): scaled Newton polynomials are insensitive
    to scalar scaling.  With A -> 2^k A and b -> 2^k b every operation is
    scaled exactly, so s history, residual history and x are bit-identical."""
    A = W.conv_diff_2d(24, 10.0)
    b = W.rhs(A.n, 1)
    M = csr(A)
    # The Ritz values come from a library eigensolver, which is not bitwise
    # scale-equivariant; give both runs the same (exactly scaled) values.
    ritz = o.solve(M, b, opts=o.Options(s_max=8, restart=40, tol=1e-11,
                                        max_restarts=0)).shifts.ritz
    opts = o.Options(s_max=8, restart=40, tol=1e-11, shifts=ritz)
    r1 = o.solve(M, b, opts=opts)
    opts2 = o.Options(s_max=8, restart=40, tol=1e-11, shifts=ritz * 2.0 ** k)
    r2 = o.solve((M * 2.0 ** k).tocsr(), b * 2.0 ** k, opts=opts2)
    assert r1.status == "ok" and len(set(r1.s_hist)) >= 1
    assert r1.s_hist == r2.s_hist
    assert r1.res_hist == r2.res_hist
    assert np.array_equal(r1.x, r2.x)


def test_newton_under_scaling_matches_constant_gamma():
    """Sec. 4.3: standard Newton on alpha*A equals scaled Newton-type
    recurrence with the constant coefficient gamma = alpha: the basis vectors
    differ only by powers of alpha, so the adapted sizes match when alpha is
    a power of two."""
    A = W.conv_diff_2d(20, 10.0)
    b = W.rhs(A.n, 3)
    M = csr(A)
    alpha = 2.0 ** -4
    rN = o.solve((M * alpha).tocsr(), b, opts=o.Options(
        s_max=6, restart=30, tol=1e-300, max_restarts=0, basis="newton"))
    assert rN.iters == 30
    # GMRES iterates are basis-independent: compare with MGS
    _, hm, _ = o.mgs_gmres((M * alpha).tocsr(), b, restart=30, tol=1e-300,
                           max_restarts=0)
    assert np.allclose(rN.res_hist, hm, rtol=1e-8)


# ---------------------------------------------------------------- P9-P13

def test_ice_brackets_true_condition():
    """P9: ICE's estimates lie inside [sigma_min, sigma_max] (so kappa_ICE <=
    kappa) and are usually within a factor of 10 (Sec. 3.2)."""
    rng = np.random.default_rng(0)
    ratios = []
    for t in range(40):
        m = 12
        R = np.triu(rng.standard_normal((m, m)))
        R[np.diag_indices(m)] = np.abs(R[np.diag_indices(m)]) + 0.1
        ice = o.ICE()
        for j in range(m):
            kap = ice.add_column(R[:j, j], R[j, j])
            sv = np.linalg.svd(R[:j + 1, :j + 1], compute_uv=False)
            assert kap <= sv[0] / sv[-1] * (1 + 1e-10)
            assert math.sqrt(ice.smax2) <= sv[0] * (1 + 1e-12)
            assert 1.0 / math.sqrt(ice.dn2) >= sv[-1] * (1 - 1e-12)
        ratios.append(sv[0] / sv[-1] / kap)
    assert np.median(ratios) <= 10.0


def test_partial_cholesky_against_numpy_and_truncation():
    """Alg. 3: equals numpy's Cholesky when nothing truncates; stops at the
    first non-positive pivot (salvaging the leading factor, Sec. 3.1) and when
    the condition estimate exceeds Omega."""
    rng = np.random.default_rng(1)
    X = rng.standard_normal((200, 10))
    G = X.T @ X
    p, R, _ = o.partial_cholesky(G, 1e12)
    assert p == 10
    assert np.allclose(R, np.linalg.cholesky(G).T, rtol=1e-12, atol=1e-12)
    # a repeated column makes the 5th pivot (numerically) zero
    Xd = X.copy()
    Xd[:, 4] = Xd[:, 1]
    p, R, _ = o.partial_cholesky(Xd.T @ Xd, 1e7)
    assert p == 4
    assert np.allclose(R.T @ R, (Xd.T @ Xd)[:4, :4], rtol=1e-12)
    # an indefinite matrix stops before the negative pivot
    D = np.diag([4.0, 1.0, -1.0, 2.0])
    p, R, _ = o.partial_cholesky(D, 1e7)
    assert p == 2 and np.allclose(R, np.diag([2.0, 1.0]))
    # graded columns: truncation where kappa first exceeds Omega
    Xg = X * np.logspace(0, 9, 10)[None, :]
    p, R, kaps = o.partial_cholesky(Xg.T @ Xg, 1e4, cond="svd")
    assert all(k <= 1e4 for k in kaps[:-1]) and (p == 10 or kaps[-1] > 1e4)
    assert p == len(kaps) - (1 if kaps[-1] > 1e4 else 0)


def test_newton_annihilation_and_ritz_exactness():
    """P10 + P13: a diagonal matrix of size N <= s with its exact eigenvalues
    as shifts annihilates the start vector after N steps, so GMRES ends in
    <= N iterations; the Ritz values of N Arnoldi steps are the eigenvalues."""
    lam = np.array([0.5, 1.0, 2.0, 3.5, 5.0, 7.0, 9.0, 11.0])
    A = sp.diags(lam).tocsr()
    b = np.ones(8)
    r = o.solve(A, b, opts=o.Options(s_max=8, restart=8, tol=1e-14,
                                     shifts=lam.astype(complex)))
    assert r.status == "ok" and r.iters <= 8
    assert np.allclose(r.x, 1.0 / lam, rtol=1e-12)
    ritz = _ritz_from_arnoldi(lam, 3)
    assert np.allclose(np.sort(ritz.real), lam, rtol=1e-10)
    assert np.abs(ritz.imag).max() <= 1e-10


def _leja_bruteforce(th):
    """Greedy Leja sequence by exact products over all candidates (no logs)."""
    th = list(th)
    order = sorted(range(len(th)), key=lambda k: (-th[k].real, -th[k].imag))
    out = []
    rem = order[:]
    first = max(rem, key=lambda k: (abs(th[k]), -rem.index(k)))
    out.append(first)
    rem.remove(first)
    while rem:
        def prod(k):
            p = 1.0
            for q in out:
                p *= abs(th[k] - th[q])
            return p
        best = max(prod(k) for k in rem)
        k = next(kk for kk in rem if prod(kk) >= best * (1 - 1e-12))
        out.append(k)
        rem.remove(k)
    return np.array([th[k] for k in out])


def test_leja_order_bruteforce():
    """P11: the oracle's log-sum Leja order equals the greedy definition
    evaluated by exact products, on random real point sets of <= 8 points;
    conjugate pairs stay adjacent."""
    rng = np.random.default_rng(5)
    for t in range(50):
        n = rng.integers(2, 9)
        th = rng.uniform(-3, 10, n).astype(complex)
        assert np.array_equal(o.leja_order(th), _leja_bruteforce(th))
    th = np.array([1 + 2j, 1 - 2j, 5.0, -3.0, 0.5 + 0.1j, 0.5 - 0.1j])
    lo = o.leja_order(th)
    assert lo[0] == 5.0
    for j in range(len(lo)):
        if lo[j].imag > 0:
            assert lo[j + 1] == np.conj(lo[j])


def test_complex_pair_recurrence():
    """Complex-conjugate shifts in real arithmetic: two steps of the pair
    recurrence equal (A - theta)(A - conj theta)/gamma^2 applied to V_1, and
    the change-of-basis matrix reproduces A V = V B."""
    rng = np.random.default_rng(2)
    n = 30
    A = rng.standard_normal((n, n))
    th = np.array([2.0 + 1.5j, 2.0 - 1.5j, -1.0])
    sh = o.newton_shifts(o.leja_order(th), scaled=True)
    v = rng.standard_normal(n)
    Vs = [v]
    for j in range(3):
        t, g, d = sh.record(j)
        w = A @ Vs[-1] - t * Vs[-1]
        if j >= 1:
            w -= d * Vs[-2]
        Vs.append(w / g)
    V = np.array(Vs).T
    B = o.change_of_basis(sh, 3)
    assert np.allclose(A @ V[:, :3], V @ B, atol=1e-12)
    lo = sh.ritz
    pair = [k for k in range(3) if lo[k].imag != 0]
    if pair[0] == 0:
        g0 = sh.gamma[0]
        M = (A - lo[0].real * np.eye(n)) @ (A - lo[0].real * np.eye(n)) + lo[0].imag ** 2 * np.eye(n)
        assert np.allclose(V[:, 2], M @ v / g0 ** 2, atol=1e-10)


# ---------------------------------------------------------------- mixed precision, preconditioning

def test_jacobi_right_preconditioning():
    """Column scaling A' = A D^{-1} (Eq. (equil)) as right preconditioning:
    the solution matches a dense solve and residuals are true residuals."""
    A = W.var_conv_diff_3d(10, seed=3)
    b = W.rhs(A.n, 3)
    r = o.solve(csr(A), b, opts=o.Options(s_max=16, restart=64, tol=1e-11,
                                          precond="jacobi"))
    x = np.linalg.solve(A.to_dense(), b)
    assert r.status == "ok"
    assert np.linalg.norm(csr(A) @ r.x - b) / np.linalg.norm(b) <= 1.01e-11
    assert np.linalg.norm(r.x - x) / np.linalg.norm(x) <= 1e-8


def test_fp32_inner_refinement_reaches_fp64_accuracy():
    """Float32 inner solves inside float64 refinement reach the float64
    tolerance, and the float32 basis keeps O(u32) orthogonality."""
    A = W.conv_diff_2d(32, 10.0)
    b = W.rhs(A.n, 1)
    r = o.solve_ir(csr(A), b, opts=o.Options(s_max=8, restart=64, tol=1e-10),
                   inner_tol=1e-4)
    assert r.status == "ok"
    x = np.linalg.solve(A.to_dense(), b)
    assert np.linalg.norm(r.x - x) / np.linalg.norm(x) <= 1e-8
    _, _, r32 = _conv_diff_run(work_dtype=np.float32, max_restarts=0,
                               tol=1e-300)
    assert o.loo(r32.trace["Q_first_cycle"]) <= 1e-5



def _float32_scaled_newton_kappa_crossing(lam, sh, bound, seeds):
    """First j at which a scaled Newton basis built in float32 arithmetic
    (numpy, outside the oracle's engine) has kappa(V_1:j) > bound, for
    each random start vector."""
    out = []
    L32 = lam.astype(np.float32)
    for seed in seeds:
        v = np.random.default_rng(seed).standard_normal(lam.size)
        v = (v / np.linalg.norm(v)).astype(np.float32)
        V = [v]
        for j in range(lam.size - 1):
            th, ga, _ = sh.record(j)
            V.append((L32 * V[-1] - np.float32(th) * V[-1]) / np.float32(ga))
        Vd = np.array(V, dtype=np.float64).T
        out.append(next(j for j in range(1, lam.size + 1)
                        if np.linalg.cond(Vd[:, :j]) > bound))
    return out


def test_fp32_partial_cholqr_stops_at_single_precision_bound():
    """The float32 inner model's partial CholQR (Alg. 3) uses the bound
    Omega = 0.1 u^{-1/2} of float32 (Sec. 3.2: Omega ~ 0.1 eps^{-1/2}),
    409.6.  A monomial Krylov block of Test 1's diagonal matrix, formed in
    float32, is cut before the first column at which the condition number
    of the projected block (SVD of a float64 copy, outside the oracle)
    exceeds 409.6, with the SVD and with the ICE condition estimate.  The
    same block in float64 keeps Test 1's six columns."""
    lam = np.linspace(0.1, 10.0, 2000)
    A = sp.diags(lam).tocsr()
    bound = 0.1 * 2.0 ** 12
    for seed in (1, 2):
        b = W.rhs(lam.size, seed)
        v = b / np.linalg.norm(b)
        K = [v]
        for _ in range(12):
            K.append(lam * K[-1])
        V = np.array(K[1:]).T
        for _ in range(2):
            V = V - np.outer(v, v @ V)
        kap = [np.linalg.cond(V[:, :j]) for j in range(1, 13)]
        expect = next(j for j in range(12) if kap[j] > bound)
        # away from the bound on both sides: float32 rounding cannot move it
        assert kap[expect - 1] < 0.5 * bound and kap[expect] > 2 * bound
        for cond in ("svd", "ice"):
            r = o.solve(A, b, opts=o.Options(
                s_max=12, restart=12, max_restarts=0, tol=1e-300,
                basis="monomial", work_dtype=np.float32, cond=cond,
                record=True))
            fb = r.trace["first_block"]
            assert fb["p1"] == expect and fb["p"] == expect, (cond, fb)
        r64 = o.solve(A, b, opts=o.Options(
            s_max=12, restart=12, max_restarts=0, tol=1e-300,
            basis="monomial", record=True))
        assert r64.trace["first_block"]["p"] == 6


def test_fp32_estimator_tracks_single_precision_basis_growth():
    """The float32 inner model's initial step size (Sec. 3.5 with the
    float32 unit round-off and Omega_est = 0.1 u^{-1/2} = 409.6) on Test 8's
    spectra, given the exact eigenvalues as shifts.  In the paper's own
    Test 8 the predicted s0* lies within a factor 2.2 of the column at
    which kappa(V_1:j) crosses the bound (134 vs 62, 17 vs 15).  Here the
    float32 scaled Newton basis (built with numpy in float32) crosses 409.6
    at the columns returned by _float32_scaled_newton_kappa_crossing, and
    s0* must lie within a factor 3 of the earliest of them; the first block
    then runs at s0* and partial CholQR keeps all of it."""
    for lmax in (200.0, 2000.0):
        lam = np.arange(1.0, 201.0)
        lam[-1] = lmax
        sh = o.newton_shifts(o.leja_order(lam.astype(complex)), scaled=True)
        cross = _float32_scaled_newton_kappa_crossing(
            lam, sh, 0.1 * 2.0 ** 12, seeds=(11, 12, 13))
        b = np.random.default_rng(11).standard_normal(lam.size)
        r = o.solve(sp.diags(lam).tocsr(), b, opts=o.Options(
            s_max=200, restart=200, max_restarts=0, tol=1e-300,
            work_dtype=np.float32, shifts=lam.astype(complex), record=True))
        assert 1 <= r.s0_est <= 3 * min(cross), (lmax, r.s0_est, cross)
        fb = r.trace["first_block"]
        assert fb["s_eff"] == r.s0_est and fb["p"] == fb["s_eff"]


def test_fp32_inner_cycle_is_the_gmres_minimiser():
    """One float32 inner cycle (the model of Alg. 4 in single precision)
    returns the GMRES iterate of its Krylov space to O(kappa u32): compared
    with the dense float64 minimiser after the same number of iterations,
    the difference is at most 100 kappa(A) 2^-24 and at least 2^-40
    relative (float32 rounding is really there)."""
    A = W.conv_diff_2d(16, 10.0)
    M = csr(A)
    Ad = A.to_dense()
    b = W.rhs(A.n, 3)
    kap = np.linalg.cond(Ad)
    for k in (8, 16, 24):
        r = o.solve(M, b, opts=o.Options(
            s_max=8, restart=k, max_restarts=0, tol=1e-300,
            work_dtype=np.float32))
        assert r.iters == k
        xk = o.gmres_iterates_dense(Ad, b, np.zeros(A.n), k)
        rel = np.linalg.norm(r.x - xk) / np.linalg.norm(xk)
        assert 2.0 ** -40 <= rel <= 100 * kap * 2.0 ** -24, (k, rel, kap)


# ---------------------------------------------------------------- adjoint

def test_adjoint_gradients_fd_and_dense():
    """P14: gradients of L = 0.5 ||x - x*||^2 through x = A^{-1} b, with
    lambda from an s-step solve of A^T lambda = x - x*: grad_b = lambda and
    grad_val = -lambda[row] x[col]; checked against a dense reference
    gradient and central finite differences."""
    n = 300
    A, b, xs = W.banded_problem(n, seed=4, band=40)
    M = csr(A)
    opts = o.Options(s_max=16, restart=64, tol=1e-13)
    x = o.solve(M, b, opts=opts).x
    lam = o.solve(M.T.tocsr(), x - xs, opts=opts).x
    gv = o.grad_vals(A.row_ptr, A.col, lam, x)
    Ad = A.to_dense()
    xd = np.linalg.solve(Ad, b)
    lamd = np.linalg.solve(Ad.T, xd - xs)
    assert np.linalg.norm(lam - lamd) <= 1e-10 * np.linalg.norm(lamd)
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    gd = -lamd[rows] * xd[A.col]
    assert np.linalg.norm(gv - gd) <= 1e-10 * np.linalg.norm(gd)

    def loss(val, bb):
        Mv = o.csr_matrix(n, A.row_ptr, A.col, val)
        xx = o.solve(Mv, bb, opts=opts).x
        return 0.5 * float(np.sum((xx - xs) ** 2))

    # Central differences along random directions (per-entry differences
    # are rounding-limited: the loss is O(n) while single entries are tiny).
    rng = np.random.default_rng(9)
    for t in range(3):
        dv = rng.standard_normal(A.nnz) * np.abs(A.val)
        h = 1e-6
        fd = (loss(A.val + h * dv, b) - loss(A.val - h * dv, b)) / (2 * h)
        assert abs(fd - gv @ dv) <= 1e-6 * abs(fd)
        db = rng.standard_normal(n)
        fd = (loss(A.val, b + h * db) - loss(A.val, b - h * db)) / (2 * h)
        assert abs(fd - lam @ db) <= 1e-6 * abs(fd)


def test_happy_breakdown_eigenvector_rhs():
    """b an eigenvector of a diagonal A: the first new basis vector vanishes
    (p = 0), the cycle ends with one column and x = b / lambda exactly."""
    lam = np.arange(1.0, 9.0)
    A = sp.diags(lam).tocsr()
    b = np.zeros(8)
    b[2] = 1.0
    for basis in ("monomial", "scaled_newton"):
        r = o.solve(A, b, opts=o.Options(s_max=4, restart=8, tol=1e-14,
                                         basis=basis))
        assert r.status == "ok" and r.iters == 1
        assert np.allclose(r.x, b / lam, rtol=1e-15, atol=0)


def test_monomial_prephase_matches_columnwise_prephase():
    """The monomial s-step pre-phase builds the same Krylov space and
    Hessenberg matrix as the column-wise CGS2 one (which the MGS-GMRES pin
    fixes): same Ritz values, same first-cycle residual history and
    solution, in blocks that adapt below prephase_s."""
    A = W.poisson_3d(16)
    M = csr(A)
    b = W.rhs(A.n, 2)
    kw = dict(s_max=24, restart=48, tol=1e-10, max_restarts=50)
    ra = o.solve(M, b, opts=o.Options(**kw))
    rb = o.solve(M, b, opts=o.Options(prephase="monomial", prephase_s=8, **kw))
    m0 = 24
    assert ra.s_hist[:m0] == [1] * m0
    pre = []
    tot = 0
    for p in rb.s_hist:
        pre.append(p)
        tot += p
        if tot >= m0:
            break
    assert tot == m0 and 1 < max(pre) <= 8 and len(pre) < m0
    za = np.sort_complex(ra.shifts.ritz)
    zb = np.sort_complex(rb.shifts.ritz)
    assert np.abs(za - zb).max() <= 1e-8 * np.abs(za).max()
    ha, hb = np.array(ra.res_hist[:m0]), np.array(rb.res_hist[:m0])
    assert np.all(np.abs(ha - hb) <= 1e-8 * ha)
    assert ra.iters == rb.iters
    assert np.linalg.norm(ra.x - rb.x) <= 1e-10 * np.linalg.norm(ra.x)


def _near_span_block(n, i, s, delta, seed):
    """Q_i orthonormal (n x i) and V = Q_i C + delta N: with delta small the
    block lies almost in span(Q_i), so one BCGS pass leaves components along
    Q_i of order u/delta and the second pass has real work to do."""
    rng = np.random.default_rng(seed)
    Qi, _ = np.linalg.qr(rng.standard_normal((n, i)))
    V = Qi @ rng.standard_normal((i, s)) + delta * rng.standard_normal((n, s))
    return Qi, V


@pytest.mark.parametrize("delta", [1.0, 1e-12])
def test_pythagorean_second_pass_block(delta):
    """f3 variant of the second BCGS pass against Householder QR of [Q_i V]
    with V = Q_i C + delta N (full rank): both variants keep every column,
    reconstruct V, keep [Q_i Q_k] orthonormal to rounding, and give the Q
    factor's last s columns and the R columns (signs fixed by a positive R
    diagonal) to the accuracy the problem allows, u kappa([Q_i V]) with
    kappa ~ 1/delta.  At delta = 1e-12 the first pass leaves R2 ~ 1e-4, so
    the R2^T R2 term of the Pythagorean Gram shifts G2 by ~1e-8: dropping
    it or flipping its sign breaks the orthogonality bound."""
    n, i, s = 3000, 20, 12
    Qi, V = _near_span_block(n, i, s, delta, seed=11)
    Qh, Rh = np.linalg.qr(np.concatenate([Qi, V], 1))
    sg = np.sign(np.diag(Rh))
    Qh, Rh = Qh * sg, (Rh.T * sg).T
    tol = 1e-12 / delta          # u kappa, with margin
    om = o.default_omega(o.U64)
    for pyth in (False, True):
        bq = o.block_orth(np.asfortranarray(Qi.copy()), i, V.copy(), om,
                          pythagorean=pyth)
        assert bq.p == s
        assert o.loo(np.concatenate([Qi, bq.Qk], 1)) <= 1e-12
        rec = Qi @ bq.R_top + bq.Qk @ bq.R_kk
        assert np.linalg.norm(rec - V) <= 1e-15 * math.sqrt(n) * np.linalg.norm(V)
        assert np.abs(bq.Qk - Qh[:, i:]).max() <= tol
        # R_top is in Q_i's frame (Householder's first i columns may differ
        # from Q_i by signs and rounding)
        Rt = (Qi.T @ Qh[:, :i]) @ Rh[:i, i:]
        assert np.abs(bq.R_top - Rt).max() <= 1e-10 * np.abs(Rt).max()
        Rk = Rh[i:, i:]
        assert np.abs(bq.R_kk - Rk).max() <= tol * np.abs(Rk).max()


def test_pythagorean_solves_keep_the_pins():
    """The f3 variant through whole solves: s-step iterates equal the GMRES
    minimisers, the basis stays orthonormal, the Arnoldi relation holds,
    and a full solve reaches the classical variant's solution."""
    n = 60
    A = small_nonsym(n, 3, shift=4.0)
    Ad = A.toarray()
    b = np.random.default_rng(4).standard_normal(n)
    x0 = np.random.default_rng(5).standard_normal(n) * 0.1
    for basis in ("monomial", "newton", "scaled_newton"):
        for s in (3, 5):
            r = o.solve(A, b, x0, o.Options(s_max=s, restart=17, max_restarts=0,
                                            tol=1e-300, basis=basis,
                                            use_estimator=False,
                                            orth="bcgs2_pyth"))
            xk = o.gmres_iterates_dense(Ad, b, x0, 17)
            assert np.linalg.norm(r.x - xk) <= 1e-8 * np.linalg.norm(xk)
        _, _, r = _conv_diff_run(basis=basis, max_restarts=0, tol=1e-300,
                                 orth="bcgs2_pyth")
        Q = r.trace["Q_first_cycle"]
        assert o.loo(Q) <= 1e-12
    A, b, r = _conv_diff_run(max_restarts=0, tol=1e-300, orth="bcgs2_pyth")
    H = r.trace["H_first_cycle"]
    Q = r.trace["Q_first_cycle"]
    k = H.shape[1]
    M = csr(A)
    assert (np.linalg.norm(M @ Q[:, :k] - Q @ H)
            / (sp.linalg.norm(M) * math.sqrt(k))) <= 1e-12
    _, _, ra = _conv_diff_run(max_restarts=20)
    _, _, rb = _conv_diff_run(max_restarts=20, orth="bcgs2_pyth")
    assert ra.status == rb.status == "ok"
    assert ra.s_hist == rb.s_hist
    assert np.linalg.norm(ra.x - rb.x) <= 1e-9 * np.linalg.norm(ra.x)


# ---------------------------------------------------------------- ILU(0) (f2)

def _pattern_random(n=90, seed=11):
    """Nonsymmetric sparse matrix with a full diagonal and a ragged pattern
    (dominant diagonal, so ILU(0) has nonzero pivots)."""
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=5.0 / n, random_state=rng, format="csr")
    A = A - 0.5 * A.sign()
    d = np.asarray(abs(A).sum(axis=1)).ravel() + 1.0
    return (A + sp.diags(d)).tocsr()


@pytest.mark.parametrize("which", ["laplace2d_12", "random_90"])
def test_ilu0_reproduces_A_on_its_pattern(which):
    """ILU(0)'s defining property (Saad, Sec. 10.3): L unit lower and U upper
    triangular on the pattern of A, with (L U)_ij = a_ij at every nonzero
    (i, j) of A.  Checked with a dense product."""
    if which == "laplace2d_12":
        M = csr(W.laplace_2d(12))
    else:
        M = _pattern_random()
    f = o.ILU0(M)
    Ad = M.toarray()
    mask = Ad != 0
    L, U = f.L.toarray(), f.U.toarray()
    assert np.array_equal(np.diag(L), np.ones(M.shape[0]))
    assert np.all(np.triu(L, 1) == 0) and np.all(np.tril(U, -1) == 0)
    off = ~np.eye(M.shape[0], dtype=bool)
    assert np.all(mask[(L != 0) & off]) and np.all(mask[U != 0])
    LU = L @ U
    assert np.abs(LU[mask] - Ad[mask]).max() <= 1e-13 * np.abs(Ad).max()
    # fill-in outside the pattern is what ILU(0) drops: it is not zero here
    assert np.abs(LU[~mask]).max() > 1e-3


def test_ilu0_of_tridiagonal_is_the_exact_lu():
    """A tridiagonal matrix has no fill, so ILU(0) is its exact LU
    factorisation; with a column-dominant diagonal partial pivoting keeps
    the identity permutation and scipy's dense LU gives the same factors."""
    import scipy.linalg as sla
    n = 40
    rng = np.random.default_rng(2)
    lo, up = rng.uniform(-1, 1, n - 1), rng.uniform(-1, 1, n - 1)
    A = sp.diags([lo, 3.0 + rng.uniform(0, 1, n), up], [-1, 0, 1]).tocsr()
    f = o.ILU0(A)
    P_, L_, U_ = sla.lu(A.toarray())
    assert np.array_equal(P_, np.eye(n))
    assert np.allclose(f.L.toarray(), L_, rtol=0, atol=1e-14)
    assert np.allclose(f.U.toarray(), U_, rtol=0, atol=1e-14)


def test_ilu0_five_point_closed_form():
    """ILU(0) of the 5-point Laplacian (4, -1) in natural ordering has the
    classical closed form (Meijerink and van der Vorst): pivots
    d_ij = 4 - 1/d_(i-1)j - 1/d_i(j-1), L entries -1/d of the west and
    south neighbours, U off-diagonals -1."""
    N = 15
    M = csr(W.laplace_2d(N))
    f = o.ILU0(M)
    d = np.zeros((N, N))
    for j in range(N):          # slow axis
        for i in range(N):      # fast axis
            v = 4.0
            if i > 0:
                v -= 1.0 / d[j, i - 1]
            if j > 0:
                v -= 1.0 / d[j - 1, i]
            d[j, i] = v
    dd = d.ravel()
    U, L = f.U.toarray(), f.L.toarray()
    assert np.allclose(np.diag(U), dd, rtol=1e-14)
    r = np.arange(N * N)
    west = r[(r % N) > 0]
    south = r[r >= N]
    assert np.allclose(L[west, west - 1], -1.0 / dd[west - 1], rtol=1e-14)
    assert np.allclose(L[south, south - N], -1.0 / dd[south - N], rtol=1e-14)
    assert np.all(U[west - 1, west] == -1.0) and np.all(U[south - N, south] == -1.0)


@pytest.mark.parametrize("basis", ["monomial", "scaled_newton"])
def test_ilu0_right_preconditioned_iterates_are_gmres_minimisers(basis):
    """Right preconditioning: the cycles run on A M^{-1} (M = L U) and
    x = x0 + M^{-1} u.  With fixed s the iterates are those of MGS-GMRES on
    the dense operator A M^{-1} (P1 / P15 applied to it), and the converged
    x solves A x = b."""
    A = W.conv_diff_2d(16, 10.0)
    M = csr(A)
    b = W.rhs(A.n, 7)
    f = o.ILU0(M)
    Ad = M.toarray()
    AMi = Ad @ np.linalg.inv((f.L @ f.U).toarray())
    k = 8                       # residual still above 1e-9 (it converges fast)
    r = o.solve(M, b, opts=o.Options(s_max=4, restart=k, max_restarts=0,
                                     tol=1e-300, basis=basis,
                                     use_estimator=False, precond="ilu0"))
    _, hm, _ = o.mgs_gmres(sp.csr_matrix(AMi), b, restart=k, tol=1e-300,
                           max_restarts=0)
    assert len(r.res_hist) == k and min(hm) > 1e-9
    assert np.allclose(r.res_hist, hm, rtol=1e-6, atol=0)
    u = o.gmres_iterates_dense(AMi, b, np.zeros(A.n), k)
    x = np.linalg.solve((f.L @ f.U).toarray(), u)
    assert np.linalg.norm(r.x - x) <= 1e-8 * np.linalg.norm(x)
    rc = o.solve(M, b, opts=o.Options(s_max=8, restart=32, tol=1e-12,
                                      precond="ilu0"))
    assert rc.status == "ok"
    xs = np.linalg.solve(Ad, b)
    assert np.linalg.norm(Ad @ rc.x - b) / np.linalg.norm(b) <= 1e-12
    assert np.linalg.norm(rc.x - xs) <= np.linalg.cond(Ad) * 1e-11 * np.linalg.norm(xs)
    r0 = o.solve(M, b, opts=o.Options(s_max=8, restart=32, tol=1e-12))
    assert rc.iters < r0.iters


@pytest.mark.slow
def test_E6_laplace_ilu0_single_block():
    """Sec. 4.3, 2D Laplace with an ILU preconditioner: the 400^2 matrix of
    Test 2 with right ILU(0), s0 = 400, scaled Newton: the adapted step size
    is 400 (one block of all 400 columns).  Ritz values from a separate
    400-step pre-phase (as in Test 3), Omega = 1e7, m = 400; b as in the
    Test 2 pin.  The block's residuals fall monotonically by ten orders."""
    g = golden("paper_stability_results.json")["E6"]
    A = W.laplace_2d(400)
    b = W.rhs(A.n, 1)
    r = o.solve(csr(A), b, opts=o.Options(
        s_max=400, restart=400, max_restarts=0, tol=1e-300,
        basis="scaled_newton", omega=1e7, use_estimator=False,
        ritz_reuse=False, precond="ilu0"))
    assert r.s_hist == [g["adapted_s_scaled_newton"]]
    h = np.asarray(r.res_hist)
    assert np.all(np.diff(h) <= 1e-12 * h[:-1])
    assert h[-1] <= 1e-9 and r.rel_res_true <= 1e-9
