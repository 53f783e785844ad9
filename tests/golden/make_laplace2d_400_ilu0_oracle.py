"""Writes laplace2d_400_ilu0_oracle.npz: the oracle's solve of the 2D
Laplace 400^2 system with right ILU(0) (the setting of the paper's Sec. 4.3
test with an ILU preconditioner), at the largest step size the GPU library
takes (s0 = 256): Ritz values from a separate 256-step pre-phase, no
estimator, Omega = 1e7, m = 400, tol 1e-8, one cycle.  Stores the block
sizes, the residual estimates, the true residual and x at 4096 sampled
rows.  Calls only the oracle.

Run from the repository root: python tests/golden/make_laplace2d_400_ilu0_oracle.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import sstep_gmres as o  # noqa: E402

OPTS = dict(s_max=256, restart=400, max_restarts=0, tol=1e-8,
            basis="scaled_newton", omega=1e7, use_estimator=False,
            ritz_reuse=False, precond="ilu0")


def main():
    A = W.laplace_2d(400)
    b = W.rhs(A.n, 1)
    M = o.csr_matrix(A.n, A.row_ptr, A.col, A.val)
    r = o.solve(M, b, opts=o.Options(**OPTS))
    idx = np.sort(np.random.default_rng(2025).choice(A.n, 4096, replace=False))
    np.savez_compressed(
        os.path.join(HERE, "laplace2d_400_ilu0_oracle.npz"),
        s_hist=np.asarray(r.s_hist, dtype=np.int32),
        res_hist=np.asarray(r.res_hist), iters=r.iters,
        rel_res_true=r.rel_res_true, status=r.status,
        sample_idx=idx.astype(np.int64), x_samples=r.x[idx])
    print(r.status, r.iters, r.s_hist, r.rel_res_true)


if __name__ == "__main__":
    main()
