"""Write poisson3d_128_oracle.npz: the CPU oracle's float64 solve of the 3D
Poisson benchmark system, for the GPU whole-solve parity test.

System: 7-point Poisson on a 128^3 interior grid (n = 2,097,152), b ~ N(0,1)
seed 2, x0 = 0, scaled Newton basis, s_max 32, restart 128, tol 1e-10
(Alg. 4 with restarts).  Stored: iteration and restart counts, the block
sizes, the Givens residual history, the final true relative residual,
||x||_2, and x at 8192 indices drawn with numpy default_rng(2024).

Run from the repository root: python tests/golden/make_poisson3d_128_oracle.py
It calls only workloads/ (the seeded inputs) and oracle/; it takes a few
minutes on 8 cores.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import sstep_gmres as o  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                   "poisson3d_128_oracle.npz")
N_SAMPLES = 8192
SAMPLE_SEED = 2024


def sample_indices(n):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(
        n, N_SAMPLES, replace=False))


def main():
    A = W.poisson_3d(128)
    b = W.rhs(A.n, 2)
    M = o.csr_matrix(A.n, A.row_ptr, A.col, A.val)
    t0 = time.time()
    r = o.solve(M, b, opts=o.Options(s_max=32, restart=128, tol=1e-10,
                                     max_restarts=1000))
    t = time.time() - t0
    true = np.linalg.norm(b - M @ r.x) / np.linalg.norm(b)
    idx = sample_indices(A.n)
    np.savez(OUT, iters=r.iters, restarts=r.restarts, s0_est=r.s0_est,
             s_hist=np.asarray(r.s_hist, dtype=np.int32),
             res_hist=np.asarray(r.res_hist), rel_res_true=true,
             x_norm=np.linalg.norm(r.x), sample_idx=idx.astype(np.int64),
             x_samples=r.x[idx], oracle_seconds=t)
    print(f"{r.status}: {r.iters} iterations, {r.restarts} restarts, "
          f"true residual {true:.3e}, {t:.0f} s -> {OUT}")


if __name__ == "__main__":
    main()
