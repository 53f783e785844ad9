"""Oracle: plain, slow, serial CPU adaptive s-step GMRES written from the paper.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module; only the test suite, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library.

Paper: Z. Xu, J. J. Alonso, E. Darve, "A numerically stable communication
avoiding s-step GMRES algorithm" (arXiv 2303.08953).  Each function cites the
section / algorithm / equation it follows.  Floating point is float64 unless
the caller asks for the float32 inner-solve model (`work_dtype=np.float32`),
in which case basis vectors, SpMV and the tall-skinny products run in float32
while every small matrix (Gram matrices after formation, Cholesky, ICE,
Hessenberg, Givens, shifts, estimator) stays float64.

Library primitives used as single steps: scipy's CSR mat-vec, numpy matmul,
numpy.linalg.eigvals (Ritz values), scipy.linalg.solve_triangular
(triangular solves, which is what the paper's "V/Z" right-division denotes),
numpy.linalg.svd (only for the optional exact condition number of Alg. 3).

Readings of points the paper leaves open are marked "Reading:" and are
listed in the design notes of the repository.

Pins: the CPU tests check this module against facts outside itself (MGS
GMRES, the GMRES minimiser by dense least squares, a dense LU solve,
orthogonality and Arnoldi-relation bounds, the step sizes the paper prints
for its Tests 1-3 and 8, closed forms, brute force on small inputs, finite
differences), and planted mistakes must fail them.  Parity unpinned: the
adapted step-size histories on the synthetic PDE workloads, for which the
paper prints no values; the GPU path is compared with this module there.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

U64 = 2.0 ** -53   # unit round-off, double
U32 = 2.0 ** -24   # unit round-off, single


def default_omega(unit_roundoff: float) -> float:
    """Condition bound Omega ~ 0.1 * eps^(-1/2) (Sec. 3.2, Alg. 3 discussion).

    For double precision this is 9.49e6, i.e. the paper's 1e7 (Sec. 4).
    """
    return 0.1 / math.sqrt(unit_roundoff)


# ---------------------------------------------------------------------------
# Sparse matrix helpers
# ---------------------------------------------------------------------------

def csr_matrix(n, row_ptr, col, val, dtype=np.float64):
    return sp.csr_matrix((np.asarray(val, dtype=dtype), np.asarray(col),
                          np.asarray(row_ptr)), shape=(n, n))


def jacobi_column_scaled(A):
    """Right Jacobi preconditioning as column scaling A' = A D^{-1}.

    Column scaling is the equilibration A' = D_r A D_c of Eq. (equil) with
    D_r = I; with D_c = diag(A)^{-1} it is right Jacobi preconditioning, so
    GMRES residuals of A' u = b are true residuals of A x = b, x = D^{-1} u.
    """
    d = A.diagonal().astype(np.float64)
    if np.any(d == 0):
        raise ValueError("zero diagonal entry: Jacobi scaling undefined")
    return (A @ sp.diags(1.0 / d)).tocsr(), d


class ILU0:
    """Incomplete LU factorisation with zero fill-in, ILU(0), as the right
    preconditioner M = L U of the 2D Laplace test with an ILU preconditioner
    (Sec. 4.3).  The paper names ILU(0) without defining it; this is the
    textbook definition (Saad, Iterative Methods for Sparse Linear Systems,
    Sec. 10.3): Gaussian elimination in row order (the IKJ form) in which
    every update that would fall outside the sparsity pattern of A is
    dropped.  L is unit lower triangular and U upper triangular, both on the
    pattern of A, and (L U)_ij = a_ij at every nonzero (i, j) of A.

    Needs every diagonal entry in the pattern and nonzero pivots.
    solve(v) returns M^{-1} v by a forward and a backward triangular solve.
    Each is one library step: SuperLU's factorisation of the triangular
    factor in its natural order with the diagonal as pivot (which leaves it
    as it is: L = L I, U = I U) followed by its solve, i.e. substitution
    with the factor; factoring once keeps the many solves cheap."""

    def __init__(self, A):
        A = sp.csr_matrix(A, dtype=np.float64, copy=True)
        A.sum_duplicates()
        A.sort_indices()
        n = A.shape[0]
        rp, ci = A.indptr, A.indices
        v = A.data
        dpos = np.full(n, -1, dtype=np.int64)
        for i in range(n):
            for e in range(rp[i], rp[i + 1]):
                if ci[e] == i:
                    dpos[i] = e
        if np.any(dpos < 0):
            raise ValueError("ILU(0) needs every diagonal entry in the pattern")
        for i in range(n):
            where = {int(ci[e]): e for e in range(rp[i], rp[i + 1])}
            # eliminate with the earlier rows k < i of row i's pattern, in
            # increasing k; updates of later entries of row i (including
            # its own lower ones, used further along this loop) stay in the
            # pattern, the rest are dropped
            for e in range(rp[i], dpos[i]):
                k = int(ci[e])
                piv = v[dpos[k]]
                if piv == 0.0 or not np.isfinite(piv):
                    raise ValueError(f"ILU(0): zero pivot in row {k}")
                v[e] = v[e] / piv
                for f in range(dpos[k] + 1, rp[k + 1]):
                    t = where.get(int(ci[f]))
                    if t is not None:
                        v[t] -= v[e] * v[f]
            if v[dpos[i]] == 0.0:
                raise ValueError(f"ILU(0): zero pivot in row {i}")
        F = sp.csr_matrix((v, ci, rp), shape=(n, n))
        self.L = (sp.tril(F, k=-1) + sp.eye(n)).tocsr()
        self.U = sp.triu(F).tocsr()
        self.n = n
        from scipy.sparse.linalg import splu
        kw = dict(permc_spec="NATURAL", diag_pivot_thresh=0.0)
        self._Ls = splu(self.L.tocsc(), **kw)
        self._Us = splu(self.U.tocsc(), **kw)
        for f in (self._Ls, self._Us):
            if (np.any(f.perm_r != np.arange(n))
                    or np.any(f.perm_c != np.arange(n))):
                raise RuntimeError("triangular factor was reordered")

    def solve(self, r):
        """M^{-1} r = U^{-1} (L^{-1} r)."""
        y = self._Ls.solve(np.asarray(r, dtype=np.float64))
        return self._Us.solve(y)


# ---------------------------------------------------------------------------
# Shifts: Leja ordering, scaled Newton coefficients, change-of-basis matrix
# ---------------------------------------------------------------------------

def leja_order(theta, tie_tol: float = 1e-10):
    """Modified Leja ordering of Ritz values (Sec. 3.4, Eq. (newton) text).

    The paper names Leja ordering without defining it.  Reading (modified
    Leja ordering of Bai, Hu and Reichel): the first point has the largest
    modulus; each next point maximises the product of distances to the points
    already chosen (evaluated as a sum of logarithms).  When a complex point
    is chosen its conjugate follows at once.  Candidates are first sorted by
    (real part desc, imaginary part desc); a score within `tie_tol` of the
    best counts as a tie and the earliest candidate in that order wins.
    Repeated values have a zero product and so come last, in sorted order.
    """
    th = np.asarray(theta, dtype=np.complex128).ravel()
    n = th.size
    order = sorted(range(n), key=lambda k: (-th[k].real, -th[k].imag))
    remaining = list(order)
    chosen = []

    def take(k):
        chosen.append(k)
        remaining.remove(k)
        if th[k].imag != 0.0:
            # its conjugate comes next (the first exact conjugate in order)
            for q in remaining:
                if th[q] == np.conj(th[k]):
                    chosen.append(q)
                    remaining.remove(q)
                    return
            raise ValueError("Ritz values are not closed under conjugation")

    mods = [abs(th[k]) for k in remaining]
    best = max(mods)
    first = next(k for k in remaining if abs(th[k]) >= best * (1 - 1e-15))
    take(first)
    while remaining:
        scores = []
        for k in remaining:
            d = np.abs(th[k] - th[chosen])
            scores.append(-np.inf if np.any(d == 0.0) else float(np.sum(np.log(d))))
        top = max(scores)
        if top == -np.inf:
            # only repeated values are left: keep their sorted order
            k = remaining[0]
        else:
            k = next(kk for kk, sc in zip(remaining, scores)
                     if sc >= top - tie_tol * max(1.0, abs(top)))
        take(k)
    return th[chosen]


@dataclass
class Shifts:
    """Per-step recurrence records of the polynomial basis (Sec. 2, Sec. 3.4).

    Step j maps V_j to V_{j+1} = ((A - theta_j I) V_j - delta_j V_{j-1}) / gamma_j,
    i.e. A V_j = gamma_j V_{j+1} + theta_j V_j + delta_j V_{j-1}: the three
    parameters are the entries of column j of the change-of-basis matrix B.
    """
    theta: np.ndarray   # real shift applied at each step
    gamma: np.ndarray   # scaling
    delta: np.ndarray   # coefficient of V_{j-1} (nonzero only for the 2nd of a complex pair)
    ritz: np.ndarray    # the Leja-ordered (complex) Ritz values
    guard_hits: int = 0

    def __len__(self):
        return self.theta.size

    def record(self, j):
        k = j % self.theta.size
        return self.theta[k], self.gamma[k], self.delta[k]


def monomial_shifts():
    """Monomial basis p_j(A) = A^j (Eq. (monomial)): theta=0, gamma=1."""
    return Shifts(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1, complex))


def newton_shifts(ritz_leja, scaled: bool = True):
    """Newton / scaled Newton recurrence records (Eqs. (newton), (scalednewton),
    (newtonrecurrence), (scalingcoeff)).

    gamma_k = |mean(theta) - theta_k| (scaled) or 1 (standard Newton).
    Reading for gamma_k = 0 (a Ritz value equal to the mean): gamma_k is
    raised to 1e-12 * max_l gamma_l, a division-by-zero guard only.
    Reading for complex conjugate pairs alpha +- i beta at steps j, j+1 (the
    paper treats real spectra and calls the extension straightforward):
    V_{j+1} = (A - alpha) V_j / gamma, V_{j+2} = ((A - alpha) V_{j+1}
    + (beta^2/gamma) V_j) / gamma, so that gamma^2 V_{j+2} equals
    (A - theta)(A - conj(theta)) V_j with both steps scaled by gamma.
    """
    th = np.asarray(ritz_leja, dtype=np.complex128)
    m = th.size
    mean = th.mean()
    if scaled:
        g = np.abs(mean - th)
        floor = 1e-12 * g.max() if g.max() > 0 else 1.0
        hits = int(np.sum(g < floor))
        g = np.maximum(g, floor)
    else:
        g = np.ones(m)
        hits = 0
    theta = th.real.copy()
    delta = np.zeros(m)
    j = 0
    while j < m:
        if th[j].imag != 0.0:
            if j + 1 >= m:
                raise ValueError("complex Ritz value without its conjugate")
            beta = abs(th[j].imag)
            delta[j + 1] = -beta * beta / g[j]
            j += 2
        else:
            j += 1
    return Shifts(theta, g.astype(np.float64), delta, th, hits)


def change_of_basis(shifts: Shifts, p: int):
    """(p+1) x p change-of-basis matrix B with A V_{1:p} = V_{1:p+1} B (Sec. 2)."""
    B = np.zeros((p + 1, p))
    for j in range(p):
        th, ga, de = shifts.record(j)
        B[j, j] = th
        B[j + 1, j] = ga
        if j >= 1 and de != 0.0:
            B[j - 1, j] = de
    return B


# ---------------------------------------------------------------------------
# Initial step-size estimator (Sec. 3.5)
# ---------------------------------------------------------------------------

def estimator_matrix_log(ritz_leja, gamma, eps):
    """log of the auxiliary matrix E of Eq. (auxiliarymatrix), as printed.

    Rows i and columns j are 1-based in the paper; here 0-based.  The
    denominators |mean - theta_k| are the scaled Newton coefficients gamma_k.
    Products are formed as sums of logarithms (same values, no overflow).
    """
    th = np.asarray(ritz_leja, dtype=np.complex128)
    s = th.size
    with np.errstate(divide="ignore"):
        lr = np.log(np.abs(th[:, None] - th[None, :])) - np.log(gamma)[None, :]
    L = np.full((s, s), -np.inf)
    le = math.log(eps)
    for i in range(s):
        for j in range(s):
            if j < i:
                L[i, j] = lr[i, :j].sum()
            elif j == i:
                L[i, j] = lr[i, :j].sum() + le
            else:
                L[i, j] = lr[i, :i].sum() + le + lr[i, i + 1:j].sum()
    return L


def estimator(ritz_leja, gamma, eps, omega_est):
    """Initial step size s0* = argmax_j { ||E_j|| < Omega_est } (Sec. 3.5).

    Reading: ||E_j|| is the 2-norm of column j, and s0* is the last j before
    the first column whose norm reaches Omega_est (the prefix reading, since
    the step sizes that matter are the leading ones), clamped to >= 1.
    Returns (s0*, log10 of the column norms).
    """
    L = estimator_matrix_log(ritz_leja, gamma, eps)
    s = L.shape[0]
    norms = np.empty(s)
    for j in range(s):
        col = L[:, j]
        mx = col.max()
        if mx == -np.inf:
            norms[j] = -np.inf
        else:
            norms[j] = mx + 0.5 * math.log(float(np.sum(np.exp(2.0 * (col - mx)))))
    crossing = np.nonzero(norms >= math.log(omega_est))[0]
    s0 = int(crossing[0]) if crossing.size else s
    return max(1, s0), norms / math.log(10.0)


# ---------------------------------------------------------------------------
# Partial Cholesky with incremental condition estimation (Alg. 3)
# ---------------------------------------------------------------------------

def _top_eig_2x2(a, b, c):
    """Largest eigenvalue of [[a, b], [b, c]] and a unit eigenvector."""
    lam = 0.5 * (a + c) + math.hypot(0.5 * (a - c), b)
    if b == 0.0:
        return lam, ((1.0, 0.0) if a >= c else (0.0, 1.0))
    if a >= c:
        u, v = lam - c, b
    else:
        u, v = b, lam - a
    nrm = math.hypot(u, v)
    return lam, (u / nrm, v / nrm)


class ICE:
    """Incremental condition estimator for a growing upper-triangular R.

    Alg. 3 calls ICE after each new column (Bischof 1990/1991, cited in
    Sec. 3.2); the paper does not print its formulas.  Reading: keep unit
    approximate singular vectors and update both extreme singular value
    estimates from the new column (v; g) = R(1:j, j) by a 2x2 symmetric
    eigenproblem in (sin, cos), O(j) work per column:
      largest:  y' = [s y; c],  |y'^T R'|^2 = s^2 smax^2 + (s a + c g)^2,
                a = y^T v, maximised over s^2 + c^2 = 1;
      smallest: d = R^{-T} x,   d' = [s d; (c - s a)/g],  a = v^T d,
                |d'|^2 = s^2 |d|^2 + (c - s a)^2 / g^2 maximised; smin = 1/|d'|.
    Both estimates lie inside [sigma_min, sigma_max], so the estimate never
    exceeds the true condition number.
    """

    def __init__(self):
        self.y = np.zeros(0)
        self.d = np.zeros(0)
        self.smax2 = 0.0
        self.dn2 = 0.0

    def add_column(self, v, g):
        v = np.asarray(v, dtype=np.float64)
        if self.y.size == 0:
            self.y = np.array([1.0])
            self.d = np.array([1.0 / g])
            self.smax2 = g * g
            self.dn2 = 1.0 / (g * g)
            return 1.0
        a = float(self.y @ v)
        lam, (s, c) = _top_eig_2x2(self.smax2 + a * a, a * g, g * g)
        self.y = np.concatenate([s * self.y, [c]])
        self.smax2 = lam
        a2 = float(v @ self.d)
        lam2, (s2, c2) = _top_eig_2x2(self.dn2 + (a2 / g) ** 2, -a2 / (g * g),
                                      1.0 / (g * g))
        self.d = np.concatenate([s2 * self.d, [(c2 - s2 * a2) / g]])
        self.dn2 = lam2
        return math.sqrt(self.smax2 * self.dn2)


def partial_cholesky(G, omega, cond="ice"):
    """Partial Cholesky of an SPD-or-not Gram matrix (Alg. 3).

    Returns (p, R, kappas): R is p x p upper triangular with
    G[:p, :p] = R^T R, and kappas[j] is the condition estimate after column
    j+1.  Readings: the off-diagonal update uses the standard Cholesky sum
    over k < i (the printed upper limit j-1 would use entries not yet
    computed); a non-positive or non-finite pivot stops the factorization
    before that column (salvaging the factor, Sec. 3.1); kappa_1 = 1, and the
    factorization stops before column j when kappa_j > Omega.
    `cond="svd"` takes kappa from the singular values of R(1:j,1:j) (the SVD
    branch of Alg. 3).
    """
    G = np.asarray(G, dtype=np.float64)
    m = G.shape[0]
    R = np.zeros((m, m))
    kappas = []
    ice = ICE()
    p = m
    for j in range(m):
        for i in range(j):
            R[i, j] = (G[i, j] - R[:i, i] @ R[:i, j]) / R[i, i]
        piv = G[j, j] - R[:j, j] @ R[:j, j]
        if not (np.isfinite(piv) and piv > 0.0) or not np.all(np.isfinite(R[:j, j])):
            p = j
            break
        R[j, j] = math.sqrt(piv)
        if cond == "svd":
            sv = np.linalg.svd(R[:j + 1, :j + 1], compute_uv=False)
            kap = sv[0] / sv[-1]
        else:
            kap = ice.add_column(R[:j, j], R[j, j])
        kappas.append(kap)
        if kap > omega:
            p = j
            break
    return p, R[:p, :p].copy(), kappas


# ---------------------------------------------------------------------------
# Block orthogonalisation: BCGS2 + partial CholQR (Alg. 4)
# ---------------------------------------------------------------------------

@dataclass
class BlockQR:
    """Result of one block orthogonalisation.  p = 0 is a (happy) breakdown:
    the first new vector lies in span(Q_1:i); R_top then holds its
    coefficients (i x 1) and R_kk = [[0]], which still defines one last
    Hessenberg column with a zero subdiagonal entry."""
    p: int                  # accepted block size (0 = breakdown)
    Qk: np.ndarray          # n x p new orthonormal columns (work dtype)
    R_top: np.ndarray       # i x p    R(1:i, k)
    R_kk: np.ndarray        # p x p    R(k, k)
    p1: int                 # size accepted by the first partial CholQR
    kappas1: list = field(default_factory=list)


def _right_divide(V, Z):
    """V / Z for upper-triangular Z: solves X Z = V by substitution."""
    return sla.solve_triangular(Z, V.T, trans="T", lower=False,
                                check_finite=False).T


def block_orth(Q, i, V, omega, work_dtype=np.float64, cond="ice",
               pythagorean=False):
    """BCGS2 with partial CholQR on V (n x s) against Q[:, :i] (Alg. 4).

    Inter-orthogonalisation is block classical Gram-Schmidt applied twice;
    each intra step is a partial Cholesky QR (Alg. 3); the two R factors are
    combined as in Alg. 2/4 ("Combine both steps").

    pythagorean=True is the low-synchronisation variant of the second pass
    (not in the paper; its stability is checked by the orthogonality and
    GMRES-minimiser pins, not proved here).  With U = Qk - Q_i R2 and
    Q_i^T Q_i = I, U^T U = Qk^T Qk - R2^T R2 (Pythagoras), so the second
    Gram is taken from Qk^T Qk, which the projection pass can form from
    the same data, instead of from U after the update; the update and the
    second triangular solve then become one step.  The first pass is the
    paper's.
    """
    wd = work_dtype
    Qi = Q[:, :i]
    W = Qi.T @ V                                     # first BCGS
    V = V - Qi @ W
    G = (V.T @ V).astype(np.float64)
    p1, Z, kap1 = partial_cholesky(G, omega, cond)   # first partial CholQR
    if p1 == 0:
        # breakdown: V_2 lies in span(Q_1:i); its coefficients are W[:, 0]
        return BlockQR(0, V[:, :0], W[:, :1].astype(np.float64),
                       np.zeros((1, 1)), 0, kap1)
    Qk = _right_divide(V[:, :p1], Z.astype(wd)).astype(wd)
    R2 = Qi.T @ Qk                                   # second BCGS
    if pythagorean:
        R2d = R2.astype(np.float64)
        G2 = (Qk.T @ Qk).astype(np.float64) - R2d.T @ R2d
        Qk = Qk - Qi @ R2
    else:
        Qk = Qk - Qi @ R2
        G2 = (Qk.T @ Qk).astype(np.float64)
    p, Zt, _ = partial_cholesky(G2, omega, cond)     # second partial CholQR
    if p == 0:
        # breakdown after the first pass: the first column's coefficients
        R_top = W[:, :1].astype(np.float64) + R2[:, :1].astype(np.float64) * Z[0, 0]
        return BlockQR(0, V[:, :0], R_top, np.zeros((1, 1)), p1, kap1)
    Qk = _right_divide(Qk[:, :p], Zt.astype(wd)).astype(wd)
    Zp = Z[:p, :p]
    R_top = W[:, :p].astype(np.float64) + R2[:, :p].astype(np.float64) @ Zp
    R_kk = Zt @ Zp
    return BlockQR(p, Qk, R_top, R_kk, p1, kap1)


# ---------------------------------------------------------------------------
# Hessenberg recovery through the change-of-basis matrix
# ---------------------------------------------------------------------------

def hessenberg_block(Hraw, i, p, R_top, R_kk, B):
    """New Hessenberg columns i..i+p-1 (1-based) of the block started at Q_i.

    Alg. 1/4 name this step without giving a formula and point to the
    s-step literature.  Derivation used here: with
    V_{1:p+1} = Q_{1:i+p} Rt, Rt = [e_i | R(1:i+p, k)], and A V_{1:p} =
    V_{1:p+1} B_p, split Rt(1:i+p-1, 1:p) = [X; T] (X: rows 1..i-1, T: rows
    i..i+p-1, upper triangular with T_11 = 1).  The Arnoldi relation
    A Q_{1:c} = Q_{1:c+1} H then gives
        H(1:i+p, i:i+p-1) = (Rt B_p - [H(1:i, 1:i-1) X; 0]) T^{-1}.
    Hraw holds the un-rotated Hessenberg matrix; the new columns are written
    into it in place (0-based columns i-1 .. i+p-2).
    """
    Rt = np.zeros((i + p, p + 1))
    Rt[i - 1, 0] = 1.0
    Rt[:i, 1:] = R_top
    Rt[i:, 1:] = R_kk
    X = Rt[:i - 1, :p]
    T = Rt[i - 1:i + p - 1, :p]
    M = Rt @ B
    if i > 1:
        M[:i, :] -= Hraw[:i, :i - 1] @ X
    Hnew = _right_divide(M, T)
    Hraw[:i + p, i - 1:i + p - 1] = Hnew
    return Hnew


class Givens:
    """Givens QR of the Hessenberg matrix for the least-squares problem
    min || beta e_1 - H y || (Alg. 1/4: "apply Givens rotation", final LSQ).

    Convention: r = hypot(a, b), c = a/r, s = b/r; c = 1, s = 0 when b = 0.
    """

    def __init__(self, m, beta):
        self.Hr = np.zeros((m + 1, m))
        self.c = np.zeros(m)
        self.s = np.zeros(m)
        self.g = np.zeros(m + 1)
        self.g[0] = beta

    def add_column(self, col, h):
        """Rotate column `col` (0-based) given its un-rotated entries h[0:col+2]."""
        h = np.array(h[:col + 2], dtype=np.float64)
        for r in range(col):
            a, b = h[r], h[r + 1]
            h[r] = self.c[r] * a + self.s[r] * b
            h[r + 1] = -self.s[r] * a + self.c[r] * b
        a, b = h[col], h[col + 1]
        if b == 0.0:
            cc, ss, rr = 1.0, 0.0, a
        else:
            rr = math.hypot(a, b)
            cc, ss = a / rr, b / rr
        self.c[col], self.s[col] = cc, ss
        h[col], h[col + 1] = rr, 0.0
        self.Hr[:col + 2, col] = h
        gc = self.g[col]
        self.g[col] = cc * gc
        self.g[col + 1] = -ss * gc
        return abs(self.g[col + 1])

    def solve(self, k):
        """Back substitution for y in H_r(1:k, 1:k) y = g(1:k)."""
        if k == 0:
            return np.zeros(0)
        return sla.solve_triangular(self.Hr[:k, :k], self.g[:k], lower=False,
                                    check_finite=False)


# ---------------------------------------------------------------------------
# Adaptive s-step GMRES (Alg. 4 with restarts, Ritz pre-phase, estimator)
# ---------------------------------------------------------------------------

@dataclass
class Options:
    s_max: int = 8
    restart: int = 64
    max_restarts: int = 1000
    tol: float = 1e-10
    basis: str = "scaled_newton"      # "scaled_newton" | "newton" | "monomial"
    precond: str = "none"             # "none" | "jacobi" | "ilu0"
    omega: float = 0.0                # 0 => 0.1 u^{-1/2} of the work precision
    omega_est: float = 0.0            # 0 => same rule
    use_estimator: bool = True
    ritz_reuse: bool = True
    shifts: object = None             # optional complex Ritz values (skip pre-phase)
    prephase: str = "cgs2"            # "cgs2": s = 1 steps; "monomial": s-step blocks
    prephase_s: int = 8               # first block size of the monomial pre-phase
    cond: str = "ice"                 # "ice" | "svd"
    orth: str = "bcgs2"               # "bcgs2" | "bcgs2_pyth" (second Gram by Pythagoras)
    work_dtype: object = np.float64   # float32 => single-precision inner model
    record: bool = False              # keep per-block traces for tests


@dataclass
class Result:
    x: np.ndarray
    status: str
    res_hist: list
    s_hist: list
    iters: int
    restarts: int
    rel_res_true: float
    s0_est: int
    shifts: Shifts | None
    blocks: list = field(default_factory=list)   # (cycle, i, s_eff, p1, p)
    true_res_restarts: list = field(default_factory=list)
    trace: dict = field(default_factory=dict)




class _State:
    """What a solve carries across cycles: the basis shifts and step size."""

    def __init__(self, shifts, s_init):
        self.shifts = shifts
        self.s_init = s_init
        self.s0_est = 0


class _Engine:
    """Adaptive s-step GMRES cycles on one fixed (possibly scaled) matrix."""

    def __init__(self, A, opts: Options, prec=None):
        self.A64 = A.astype(np.float64)
        self.wd = np.dtype(opts.work_dtype)
        self.Aw = A.astype(self.wd)
        self.prec = prec        # right preconditioner (M^{-1} by .solve)
        if prec is not None and self.wd != np.float64:
            raise ValueError("the ILU(0) preconditioner is float64 only")
        self.o = opts
        self.u = U32 if self.wd == np.float32 else U64
        self.omega = opts.omega if opts.omega > 0 else default_omega(self.u)
        self.omega_est = (opts.omega_est if opts.omega_est > 0
                          else default_omega(self.u))

    def mpk(self, q, shifts: Shifts, s_eff):
        """Matrix powers kernel of Alg. 4 with the recurrence of
        Eq. (newtonrecurrence): V_1 = Q_i, V_{j+1} = ((A - theta_j) V_j -
        delta_j V_{j-1}) / gamma_j.  Returns V_2 .. V_{s_eff+1} (n x s_eff).
        The shift records restart at the first one in every block.
        """
        wt = self.wd.type
        V = np.empty((q.size, s_eff + 1), dtype=self.wd, order="F")
        V[:, 0] = q
        for j in range(s_eff):
            th, ga, de = shifts.record(j)
            # with a right preconditioner the Krylov operator is A M^{-1}
            z = V[:, j] if self.prec is None else self.prec.solve(V[:, j])
            w = self.Aw @ z - wt(th) * V[:, j]
            if j >= 1 and de != 0.0:
                w = w - wt(de) * V[:, j - 1]
            V[:, j + 1] = w / wt(ga)
        return V[:, 1:]

    def finish_prephase(self, Hraw, m0, st: _State):
        """Ritz values of H(1:m0, 1:m0) from the column-wise pre-phase (Sec.
        3.4 takes them from a short run of standard Arnoldi / GMRES), Leja
        order, (scaled) Newton records, and the initial step size from the
        estimator of Sec. 3.5 (scaled Newton only)."""
        ritz = (np.linalg.eigvals(Hraw[:m0, :m0]) if m0 > 0
                else np.array([0.0 + 0.0j]))
        self.set_shifts(st, ritz, estimate=m0 > 0)

    def set_shifts(self, st: _State, ritz, estimate=True):
        """Shifts from Ritz values (Leja order, recurrence records) and the
        initial step size of Sec. 3.5.  Reading: shifts the caller passes
        in stand in for the pre-phase's Ritz values, so the estimator sets
        the initial step size from them in the same way."""
        o = self.o
        st.shifts = _make_shifts(o.basis, ritz)
        st.s_init = o.s_max
        if o.basis == "scaled_newton" and o.use_estimator and estimate:
            s0, _ = estimator(st.shifts.ritz, st.shifts.gamma, self.u,
                              self.omega_est)
            st.s0_est = s0
            st.s_init = max(1, min(o.s_max, s0))

    def cycle(self, Q, r, beta, beta0, st: _State, logs, cycle_id,
              prephase_only=False):
        """One restart cycle of Alg. 4 from the residual r (||r|| = beta).

        When the shifts are not known yet, the first m0 = min(s_max, m)
        columns are built with the monomial basis -- by default with s = 1,
        the s = 1 case of Alg. 4, i.e. column-wise CGS2 Arnoldi (Sec. 3.3);
        with prephase="monomial" in blocks of Alg. 4 itself, starting at
        prephase_s and adapting (non-increasing) like any block, the last
        one cut to end at exactly m0 columns -- and the shifts are derived
        from them before the scaled Newton blocks continue.  Both build the
        same Krylov space and Hessenberg matrix (up to rounding).
        Returns (dx, k, converged): the update Q(:, 1:k) y of this cycle.
        """
        o = self.o
        m = o.restart
        res_hist, s_hist, blocks, trace = logs
        Q[:, 0] = (r / beta).astype(self.wd)
        Hraw = np.zeros((m + 1, m))
        gv = Givens(m, beta)
        mono = monomial_shifts()
        m0 = min(o.s_max, m) if st.shifts is None else 0
        last = m0 if prephase_only else m
        tol = -1.0 if prephase_only else o.tol
        nb, k, conv = 1, 0, False
        s = st.s_init
        s_pre = max(1, min(o.prephase_s, m0)) if o.prephase == "monomial" else 1
        while nb <= last and not conv:
            if st.shifts is None and nb > m0:
                self.finish_prephase(Hraw, nb - 1, st)
                s = st.s_init
            in_pre = st.shifts is None
            sh = mono if in_pre else st.shifts
            if in_pre:
                s_eff = min(s_pre, m0 + 1 - nb, m + 1 - nb)
            else:
                s_eff = min(s, m + 1 - nb)
            V = self.mpk(Q[:, nb - 1], sh, s_eff)
            bq = block_orth(Q, nb, V, self.omega, self.wd, o.cond,
                            pythagorean=(o.orth == "bcgs2_pyth" and s_eff > 1))
            if trace is not None and not in_pre and "first_block" not in trace:
                trace["first_block"] = dict(kappas=list(bq.kappas1), p1=bq.p1,
                                            p=bq.p, s_eff=s_eff)
            if not prephase_only:
                blocks.append((cycle_id, nb, s_eff, bq.p1, bq.p))
            p = bq.p
            if p == 0:
                # happy breakdown: the Krylov space is invariant.  Add the last
                # Hessenberg column (zero subdiagonal) and end the cycle.
                hessenberg_block(Hraw, nb, 1, bq.R_top, bq.R_kk,
                                 change_of_basis(sh, 1))
                res = gv.add_column(nb - 1, Hraw[:, nb - 1]) / beta0
                k = nb
                if not prephase_only:
                    res_hist.append(res)
                    s_hist.append(0)
                conv = True
                break
            Q[:, nb:nb + p] = bq.Qk
            hessenberg_block(Hraw, nb, p, bq.R_top, bq.R_kk,
                             change_of_basis(sh, p))
            if not prephase_only:
                s_hist.append(p)
            for c in range(nb - 1, nb - 1 + p):
                res = gv.add_column(c, Hraw[:, c]) / beta0
                k = c + 1
                if not prephase_only:
                    res_hist.append(res)
                if res <= tol:
                    conv = True
                    break
            nb += p
            if not in_pre:
                s = p                  # Alg. 4: the step size never grows
            elif o.prephase == "monomial":
                s_pre = p
        if st.shifts is None:
            self.finish_prephase(Hraw, k, st)
        if trace is not None and "H_first_cycle" not in trace and not prephase_only:
            trace["H_first_cycle"] = Hraw[:k + 1, :k].copy()
            trace["Q_first_cycle"] = Q[:, :k + 1].copy()
        if prephase_only:
            return np.zeros(Q.shape[0]), 0, False
        y = gv.solve(k)
        dx = Q[:, :k].astype(np.float64) @ y
        return dx, k, conv


def _make_shifts(basis, ritz):
    if basis == "monomial":
        return monomial_shifts()
    return newton_shifts(leja_order(ritz), scaled=(basis == "scaled_newton"))


def solve(A, b, x0=None, opts: Options | None = None) -> Result:
    """Adaptive s-step GMRES(m) with restarts (Alg. 4, Secs. 3.3-3.5).

    A is a scipy sparse matrix.  Convergence is judged on
    ||b - A x|| / ||b - A x0|| (the Sec. 4 metric): per column from the
    Givens estimate, and decisively from the true residual at each cycle end.
    Readings: the step size resets to s_init at every restart and never grows
    inside a cycle; the shifts are computed once per solve; with ritz_reuse
    the pre-phase columns are the first iterations of the first cycle.
    Right Jacobi preconditioning is column scaling (opts.precond="jacobi").
    Right ILU(0) preconditioning (opts.precond="ilu0") runs the cycles on
    A M^{-1} with M = L U and updates x += M^{-1} Q y, so the residuals are
    those of A x = b.
    """
    o = opts or Options()
    if o.orth not in ("bcgs2", "bcgs2_pyth"):
        raise ValueError(f"unknown orth {o.orth!r}")
    if o.precond not in ("none", "jacobi", "ilu0"):
        raise ValueError(f"unknown preconditioner {o.precond!r}")
    A = A.tocsr().astype(np.float64)
    n = A.shape[0]
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    dscale = None
    if o.precond == "jacobi":
        A, dscale = jacobi_column_scaled(A)
        x = x * dscale                               # u0 = D x0
    prec = ILU0(A) if o.precond == "ilu0" else None
    eng = _Engine(A, o, prec)
    r = b - eng.A64 @ x
    beta0 = float(np.linalg.norm(r))
    res_hist, s_hist, blocks, trueres = [], [], [], []
    trace = {} if o.record else None
    logs = (res_hist, s_hist, blocks, trace)

    def out(status, iters, restarts, rel, st):
        xo = x / dscale if dscale is not None else x
        if trace is not None:
            trace["Q_last"] = Q
        return Result(xo, status, res_hist, s_hist, iters, restarts, rel,
                      st.s0_est if st else 0, st.shifts if st else None,
                      blocks, trueres, trace if trace is not None else {})

    Q = None
    if beta0 == 0.0:
        return out("ok", 0, 0, 0.0, None)
    if not np.isfinite(beta0):
        return out("numeric", 0, 0, float("nan"), None)
    m = o.restart
    Q = np.zeros((n, m + 1), dtype=eng.wd, order="F")
    st = _State(None, o.s_max)
    if o.shifts is not None:
        eng.set_shifts(st, np.asarray(o.shifts, dtype=complex))
    elif o.basis == "monomial":
        st.shifts = monomial_shifts()
    beta = beta0
    iters = restarts = 0
    rel = 1.0
    status = "not_converged"
    if st.shifts is None and not o.ritz_reuse:
        eng.cycle(Q, r, beta, beta0, st, logs, -1, prephase_only=True)
    while True:
        dx, k, _ = eng.cycle(Q, r, beta, beta0, st, logs, restarts)
        x = x + (dx if prec is None else prec.solve(dx))
        iters += k
        r = b - eng.A64 @ x
        beta = float(np.linalg.norm(r))
        rel = beta / beta0
        trueres.append(rel)
        if not np.isfinite(rel):
            status = "numeric"
            break
        if rel <= o.tol:
            status = "ok"
            break
        if restarts >= o.max_restarts or k == 0:
            break
        restarts += 1
    return out(status, iters, restarts, rel, st)


# ---------------------------------------------------------------------------
# Mixed precision: float32 inner s-step GMRES inside float64 refinement
# ---------------------------------------------------------------------------

@dataclass
class IRResult:
    x: np.ndarray
    status: str
    outer: int
    iters: int
    rel_res_true: float
    res_true_hist: list
    # per outer step: (||r|| / ||r0||, inner block sizes, inner Givens
    # estimates relative to the inner right-hand side r / ||r||)
    inner: list = field(default_factory=list)


def solve_ir(A, b, x0=None, opts: Options | None = None, inner_tol=1e-4,
             inner_restarts=0, max_outer=200) -> IRResult:
    """Float32 inner solves inside a float64 iterative-refinement loop.

    Not in the paper (which is float64 throughout); this is the mixed
    precision variant of the same algorithm: r = b - A x in float64; the
    correction equation A d = r/||r|| is solved by the float32 model of
    Alg. 4 (one cycle plus `inner_restarts` restarts, stopping at relative
    residual `inner_tol`), and x += ||r|| d in float64.  Shifts and the
    initial step size are computed once, in the first inner solve, and
    reused by every later one.
    """
    o = opts or Options()
    A = A.tocsr().astype(np.float64)
    n = A.shape[0]
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    dscale = None
    if o.precond == "ilu0":
        raise ValueError("the ILU(0) preconditioner is float64 only")
    if o.precond == "jacobi":
        A, dscale = jacobi_column_scaled(A)
        x = x * dscale
    inner = Options(**{**o.__dict__, "work_dtype": np.float32, "tol": inner_tol,
                       "max_restarts": inner_restarts, "precond": "none"})
    eng = _Engine(A, inner)
    r = b - A @ x
    beta0 = float(np.linalg.norm(r))
    hist = [1.0]
    inner_logs = []
    if beta0 == 0.0:
        return IRResult(x, "ok", 0, 0, 0.0, hist, inner_logs)
    Q = np.zeros((n, inner.restart + 1), dtype=np.float32, order="F")
    st = _State(None, inner.s_max)
    if o.shifts is not None:
        eng.set_shifts(st, np.asarray(o.shifts, dtype=complex))
    elif o.basis == "monomial":
        st.shifts = monomial_shifts()
    iters = 0
    status = "not_converged"
    outer = 0
    rel = 1.0
    while outer < max_outer:
        beta = float(np.linalg.norm(r))
        rel = beta / beta0
        if rel <= o.tol:
            status = "ok"
            break
        if not np.isfinite(rel):
            status = "numeric"
            break
        outer += 1
        rn = (r / beta)
        d = np.zeros(n)
        rr, bb = rn.copy(), 1.0
        step_s, step_res = [], []
        inner_logs.append((rel, step_s, step_res))
        for rs in range(inner_restarts + 1):
            logs = (step_res, step_s, [], None)
            dx, k, conv = eng.cycle(Q, rr, bb, 1.0, st, logs, rs)
            iters += k
            d += dx
            if conv or k == 0:
                break
            rr = rn - (eng.Aw @ d.astype(np.float32)).astype(np.float64)
            bb = float(np.linalg.norm(rr))
        x = x + beta * d
        r = b - A @ x
        hist.append(float(np.linalg.norm(r)) / beta0)
    xo = x / dscale if dscale is not None else x
    return IRResult(xo, status, outer, iters, rel, hist, inner_logs)


# ---------------------------------------------------------------------------
# Classical GMRES (MGS Arnoldi) -- the baseline the paper compares against
# ---------------------------------------------------------------------------

def mgs_gmres(A, b, x0=None, restart=64, tol=1e-10, max_restarts=100):
    """GMRES(m) with modified Gram-Schmidt Arnoldi and Givens rotations
    (the MGS-GMRES baseline of Secs. 4-5).  Returns (x, res_hist, iters)."""
    A = A.tocsr().astype(np.float64)
    n = A.shape[0]
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    r = b - A @ x
    beta0 = float(np.linalg.norm(r))
    hist = []
    iters = 0
    if beta0 == 0.0:
        return x, hist, 0
    for _ in range(max_restarts + 1):
        beta = float(np.linalg.norm(r))
        Q = np.zeros((n, restart + 1))
        Q[:, 0] = r / beta
        gv = Givens(restart, beta)
        k = 0
        for j in range(restart):
            w = A @ Q[:, j]
            h = np.zeros(j + 2)
            for l in range(j + 1):
                h[l] = Q[:, l] @ w
                w = w - h[l] * Q[:, l]
            h[j + 1] = np.linalg.norm(w)
            res = gv.add_column(j, h) / beta0
            hist.append(res)
            k = j + 1
            if h[j + 1] == 0.0 or res <= tol:
                break
            Q[:, j + 1] = w / h[j + 1]
        y = gv.solve(k)
        x = x + Q[:, :k] @ y
        iters += k
        r = b - A @ x
        if np.linalg.norm(r) / beta0 <= tol:
            break
    return x, hist, iters


def gmres_iterates_dense(A, b, x0, k):
    """The GMRES iterate after k steps by its definition: the minimiser of
    ||b - A x|| over x0 + K_k(A, r0), with the Krylov space spanned by an
    orthonormal basis built by Householder QR (for tiny dense tests)."""
    A = np.asarray(A, dtype=np.float64)
    r0 = b - A @ x0
    K = np.empty((A.shape[0], k))
    v = r0 / np.linalg.norm(r0)
    for j in range(k):
        K[:, j] = v
        v = A @ v
        v = v / np.linalg.norm(v)
    Qb, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(A @ Qb, r0, rcond=None)
    return x0 + Qb @ y


# ---------------------------------------------------------------------------
# Adjoint (gradients through the solve)
# ---------------------------------------------------------------------------

def grad_vals(row_ptr, col, lam, x):
    """d loss / d A.val for x = A^{-1} b: -lambda[row(k)] * x[col(k)] where
    A^T lambda = d loss / d x (standard adjoint of a linear solve; not in the
    paper)."""
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    return -np.asarray(lam)[rows] * np.asarray(x)[np.asarray(col)]


def loo(Q):
    """Loss of orthogonality ||I - Q^T Q||_F (Sec. 2.2)."""
    Q = np.asarray(Q, dtype=np.float64)
    return float(np.linalg.norm(np.eye(Q.shape[1]) - Q.T @ Q))
